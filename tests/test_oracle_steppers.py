"""Pins for the oracle's exponential steppers and whole-run accuracy (CPU).

  * discrete mass conservation across steps (every phi combination lives in
    the span of mass-free vectors on a periodic mesh);
  * observed temporal order against a tiny-step RK4 solution of the same
    semi-discretization: EPI2 -> 2, EPI3 and EXPRB32 -> 3 (paper Section 5.1,
    Table expo-burgers-tconv-smooth gives orders 2 and 3 for EPI2/EXPRB32),
    EXPRB42 -> 4 (the fourth-order scheme of Section 5.2);
  * Burgers with u0 = 0.5 + sin x against the characteristic solution before
    the shock (t_b = 1): spatial order about p + 1;
  * Euler: exact translating isentropic vortex (Section 5.2): spatial order at
    least p + 1/2 (the paper observes k + 1/2, Table
    expo-euler-isentropic-sconv-uni);
  * a replayed Krylov schedule reproduces a step bit for bit;
  * Krylov iterations per step grow with the Courant number (Section 5.2.5).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs
from tests import _textbook as tb

SCHEMES = {"epi2": oracle.EPI2, "epi3": oracle.EPI3, "exprb32": oracle.EXPRB32,
           "exprb42": oracle.EXPRB42}


def burgers_c1(K=64, p=2):
    m = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=2 * math.pi)
    x, _ = m.nodes()
    return m, inputs.burgers_ic(x), x


def vortex_mesh(n, p, beta=5.0):
    m = oracle.Mesh(oracle.EULER2D, n, p, ny=n, x0=0.0, x1=10.0, y0=0.0, y1=10.0)
    x, y = m.nodes()
    return m, inputs.vortex(x, y, beta=beta).reshape(-1), x, y


def run(m, scheme, q, dt, nsteps, **kw):
    qp = None
    for _ in range(nsteps):
        q, qprev = m.step(scheme, dt, q, qp, **kw)
        qp = qprev
    return q


def l2(m, e):
    w = m.mass()
    e = e.reshape(m.nvar, -1)
    return math.sqrt(sum(np.dot(w, e[c] ** 2) for c in range(m.nvar)))


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_mass_conservation(scheme):
    m, u, _ = burgers_c1()
    w = m.mass()
    u1 = run(m, SCHEMES[scheme], u, 0.05, 4)
    assert abs(np.dot(w, u1) - np.dot(w, u)) < 1e-12 * np.dot(w, np.abs(u))
    me, q, _, _ = vortex_mesh(4, 2)
    wq = me.mass()
    q1 = run(me, SCHEMES[scheme], q, 0.1, 2).reshape(4, -1)
    q0 = q.reshape(4, -1)
    for c in range(4):
        assert abs(np.dot(wq, q1[c]) - np.dot(wq, q0[c])) < 1e-12 * np.dot(wq, np.abs(q0[c])) + 1e-14


# The linear operator freezes the Lax-Friedrichs dissipation at q^n (the split
# is made at the continuous level, Section 2.2), so it differs from the exact
# Jacobian of R by a term proportional to the face jumps of q^n, O(h^{p+1}).
# That defect adds an O(dt h^{p+1}) error, so the classical orders are pinned on
# a resolved mesh where it is far below the temporal error.
@pytest.mark.parametrize("scheme,order", [("epi2", 2.0), ("epi3", 3.0), ("exprb32", 3.0),
                                          ("exprb42", 4.0)])
def test_temporal_order_burgers(scheme, order):
    m, u, _ = burgers_c1(K=64, p=4)
    T = 0.5
    ref = m.rk4(u, 2.5e-4, 2000)
    errs = []
    dts = [0.1, 0.05, 0.025, 0.0125]
    for dt in dts:
        un = run(m, SCHEMES[scheme], u, dt, int(round(T / dt)), tol=1e-13, m_min=5, m_max=40)
        errs.append(l2(m, un - ref))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - order) < 0.25, (errs, orders)


@pytest.mark.parametrize("scheme,order", [("epi2", 2.0), ("epi3", 3.0)])
def test_temporal_order_euler(scheme, order):
    m, q, _, _ = vortex_mesh(16, 4, beta=3.0)
    T = 1.0
    ref = m.rk4(q, 2.5e-3, 400)
    errs = []
    for dt in [0.25, 0.125, 0.0625]:
        qn = run(m, SCHEMES[scheme], q, dt, int(round(T / dt)), tol=1e-13, m_min=5, m_max=60)
        errs.append(l2(m, qn - ref))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - order) < 0.3, (errs, orders)


# With the Lax-Friedrichs flux (not an upwind flux) nodal DG converges at
# about p + 1/2 for smooth solutions; the paper observes k + 1/2 for the vortex
# (Table expo-euler-isentropic-sconv-uni).  Measured on the finest pair:
# Burgers 1.48 / 2.41 / 3.78 for p = 1 / 2 / 3.
@pytest.mark.parametrize("p", [1, 2, 3])
def test_burgers_characteristics_spatial_order(p):
    T = 0.5
    errs = []
    for K in [64, 128, 256]:
        m, u, x = burgers_c1(K=K, p=p)
        dx = (2 * math.pi / K) / 2 * np.min(np.diff(oracle.lgl(p)[0]))
        nsteps = int(math.ceil(T / (0.1 * dx / 1.5)))
        un = m.rk4(u, T / nsteps, nsteps)
        exact = tb.burgers_characteristic(x, T, lambda s: 0.5 + np.sin(s), np.cos)
        errs.append(l2(m, un - exact))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert orders[-1] > p + 0.35 and orders[-1] >= orders[0] - 0.05, (errs, orders)


def test_burgers_c1_epi2_vs_characteristics():
    # the C1 configuration itself: K = 64, p = 2, EPI2, dt = 1e-2, t = 0.5; its
    # error is the spatial error of the semi-discretization plus a small
    # temporal part
    m, u, x = burgers_c1()
    un = run(m, oracle.EPI2, u, 1e-2, 50, tol=1e-10, m_min=5, m_max=30)
    fine = m.rk4(u, 5e-4, 1000)
    exact = tb.burgers_characteristic(x, 0.5, lambda s: 0.5 + np.sin(s), np.cos)
    err, err_space = l2(m, un - exact), l2(m, fine - exact)
    assert err < 1.2 * err_space and err_space / l2(m, exact) < 3e-4, (err, err_space)


# Measured on 16^2 -> 32^2 quads: 2.58 / 3.19 / 4.44 for p = 2 / 3 / 4.  Coarser
# meshes under-resolve the beta = 5 vortex and collocation DG without
# de-aliasing blows up there, so the pair starts at 16^2.
@pytest.mark.parametrize("p", [2, 3, 4])
def test_vortex_spatial_order(p):
    T = 0.5
    errs = []
    for n in [16, 32]:
        m, q, x, y = vortex_mesh(n, p)
        c, dx = m.max_speed(q)
        nsteps = int(math.ceil(T / (0.2 * dx / c)))
        qn = m.rk4(q, T / nsteps, nsteps)
        exact = inputs.vortex(x, y, t=T).reshape(-1)
        errs.append(l2(m, qn - exact))
    order = math.log(errs[0] / errs[1]) / math.log(2)
    assert order > p + 0.1, (errs, order)


def test_vortex_epi3_matches_exact():
    m, q, x, y = vortex_mesh(16, 4)
    c, dx = m.max_speed(q)
    dt = 5.0 * dx / c  # Courant number 5
    nsteps = int(math.ceil(0.5 / dt))
    dt = 0.5 / nsteps
    qn = run(m, oracle.EPI3, q, dt, nsteps, tol=1e-10, m_min=10, m_max=64)
    exact = inputs.vortex(x, y, t=0.5).reshape(-1)
    assert l2(m, qn - exact) / l2(m, exact) < 2e-4


def test_replayed_step_is_bitwise():
    m, q, _, _ = vortex_mesh(4, 3)
    q1, qp1, st = m.step(oracle.EXPRB32, 0.3, q, None, tol=1e-10, m_min=5, m_max=20, stats=True)
    q2, qp2 = m.step(oracle.EXPRB32, 0.3, q, None, tol=1e-10, m_min=5, m_max=20, forced=st["log"])
    assert st["phi_calls"] == 2
    assert np.array_equal(q1, q2)


def test_krylov_iterations_grow_with_courant():
    m, q, _, _ = vortex_mesh(8, 3)
    c, dx = m.max_speed(q)
    iters = []
    for cr in [1.0, 5.0, 20.0]:
        _, _, st = m.step(oracle.EPI2, cr * dx / c, q, None, tol=1e-10, m_min=5, m_max=64,
                          stats=True)
        iters.append(st["krylov_iters"])
    assert iters[0] < iters[1] < iters[2], iters
