"""Pins for the oracle's DG residual R(q) and linear operator L(q~) v (CPU only).

What fixes each part, independently of the oracle's code:
  * free-stream preservation: R(constant state) = 0;
  * discrete conservation on a periodic mesh: sum of mass * R = 0 per variable;
  * exactness on polynomials: with a constant reference state and a field v
    that is one polynomial of degree <= p across elements (no jumps), L v is
    the exact -A_x v_x - A_y v_y on elements away from the periodic seam;
  * complex-step derivative of R with the dissipation frozen at q~ equals L
    (the split of Section 3 is a directional derivative of the flux);
  * Burgers with constant u~ = a: energy identity of the upwind (LF) scheme,
    v^T M L v = -|a|/2 sum_faces (v^- - v^+)^2, which fixes the sign of the
    face term and the dissipation coefficient;
  * piecewise-constant states: R on the face nodes reduces to the textbook
    Rusanov flux difference, and is zero inside the elements.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs
from tests import _textbook as tb


def burgers_mesh(K=16, p=3):
    return oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=2 * math.pi)


def euler_mesh(nx=5, ny=4, p=3):
    return oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, x0=0.0, x1=2.0, y0=-1.0, y1=0.5)


def euler_random(m, seed):
    q = inputs.random_euler_state(m.K * m.Np, seed)
    return q.reshape(-1)


# --------------------------------------------------------------------- free stream
@pytest.mark.parametrize("p", [1, 2, 4])
def test_free_stream(p):
    mb = burgers_mesh(p=p)
    r = mb.rhs(np.full(mb.n, 0.7))
    assert np.max(np.abs(r)) < 1e-14
    me = euler_mesh(p=p)
    q = inputs.primitive_to_conservative(np.full(me.K * me.Np, 1.3), 0.4, -0.25, 0.9)
    r = me.rhs(q.reshape(-1))
    assert np.max(np.abs(r)) < 1e-13


# --------------------------------------------------------------------- conservation
@pytest.mark.parametrize("p", [1, 3, 5])
def test_conservation(p):
    mb = burgers_mesh(p=p)
    u = inputs.random_vector(mb.n, 3) + 0.3
    r = mb.rhs(u)
    w = mb.mass()
    assert abs(np.dot(w, r)) < 1e-13 * np.dot(w, np.abs(r))
    v = inputs.random_vector(mb.n, 4)
    lv = mb.jvp(u, v)
    assert abs(np.dot(w, lv)) < 1e-13 * np.dot(w, np.abs(lv))

    me = euler_mesh(p=p)
    q = euler_random(me, 5)
    r = me.rhs(q).reshape(4, -1)
    w = me.mass()
    for c in range(4):
        assert abs(np.dot(w, r[c])) < 1e-13 * np.dot(w, np.abs(r[c])), c
    v = inputs.random_vector(me.n, 6)
    lv = me.jvp(q, v).reshape(4, -1)
    for c in range(4):
        assert abs(np.dot(w, lv[c])) < 1e-13 * np.dot(w, np.abs(lv[c])), c


# --------------------------------------------------------------------- polynomial exactness
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_jvp_polynomial_exact_burgers(p):
    K = 10
    m = oracle.Mesh(oracle.BURGERS1D, K, p, x0=-1.0, x1=2.0)
    x, _ = m.nodes()
    a = -0.8
    coef = [0.3, -1.1, 0.7, 0.25, -0.4][: p + 1]
    v = sum(c * x ** k for k, c in enumerate(coef))
    dv = sum(k * c * x ** (k - 1) for k, c in enumerate(coef) if k > 0)
    lv = m.jvp(np.full(m.n, a), v)
    inner = slice(m.Np, (K - 1) * m.Np)  # elements 1 .. K-2
    np.testing.assert_allclose(lv[inner], -a * dv[inner], atol=1e-11)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_jvp_polynomial_exact_euler(p):
    nx, ny = 5, 4
    m = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, x0=0.0, x1=2.0, y0=-1.0, y1=0.5)
    x, y = m.nodes()
    qt = np.array([1.2, 0.3, -0.5, 2.9])
    qref = np.repeat(qt[:, None], m.K * m.Np, axis=1).reshape(-1)
    rng = np.random.default_rng(11)
    v = np.zeros((4, x.size))
    dvx = np.zeros_like(v)
    dvy = np.zeros_like(v)
    for c in range(4):
        cx = rng.uniform(-1, 1, p + 1)
        cy = rng.uniform(-1, 1, p + 1)
        px = sum(cx[k] * x ** k for k in range(p + 1))
        py = sum(cy[k] * y ** k for k in range(p + 1))
        dpx = sum(k * cx[k] * x ** (k - 1) for k in range(1, p + 1))
        dpy = sum(k * cy[k] * y ** (k - 1) for k in range(1, p + 1))
        v[c] = px * py
        dvx[c] = dpx * py
        dvy[c] = px * dpy
    Ax = tb.flux_jacobian_cs(qt, 0)
    Ay = tb.flux_jacobian_cs(qt, 1)
    expect = -(Ax @ dvx + Ay @ dvy)
    lv = m.jvp(qref, v.reshape(-1)).reshape(4, m.K, m.Np)
    expect = expect.reshape(4, m.K, m.Np)
    for e in range(m.K):
        ex, ey = e % nx, e // nx
        if 1 <= ex <= nx - 2 and 1 <= ey <= ny - 2:
            np.testing.assert_allclose(lv[:, e], expect[:, e], atol=1e-10)


# --------------------------------------------------------------------- complex step
@pytest.mark.parametrize("p", [1, 2, 4])
def test_jvp_equals_complex_step(p):
    mb = burgers_mesh(p=p)
    u = inputs.random_vector(mb.n, 7) + 0.2
    v = inputs.random_vector(mb.n, 8)
    a, b = mb.jvp(u, v), mb.jvp_complex_step(u, v)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    me = euler_mesh(p=p)
    q = euler_random(me, 9)
    v = inputs.random_vector(me.n, 10)
    a, b = me.jvp(q, v), me.jvp_complex_step(q, v)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_jvp_linear():
    me = euler_mesh(p=2)
    q = euler_random(me, 1)
    v1 = inputs.random_vector(me.n, 2)
    v2 = inputs.random_vector(me.n, 3)
    lhs = me.jvp(q, 2.5 * v1 - 0.75 * v2)
    rhs = 2.5 * me.jvp(q, v1) - 0.75 * me.jvp(q, v2)
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * np.linalg.norm(rhs)


def test_euler_split_homogeneity():
    # Euler flux is homogeneous of degree one: A(q) q = F(q), hence
    # L(q) q = R(q) exactly (the nonlinear part N vanishes at the reference).
    me = euler_mesh(p=3)
    q = euler_random(me, 21)
    a, b = me.jvp(q, q), me.rhs(q)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


# --------------------------------------------------------------------- energy identity
@pytest.mark.parametrize("a", [0.9, -1.3])
@pytest.mark.parametrize("p", [1, 3])
def test_burgers_upwind_energy(a, p):
    K = 12
    m = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=3.0)
    v = inputs.random_vector(m.n, 12)
    lv = m.jvp(np.full(m.n, a), v)
    w = m.mass()
    lhs = np.dot(w * v, lv)
    vv = v.reshape(K, m.Np)
    jumps = vv[:, -1] - np.roll(vv[:, 0], -1)  # v^- (left elem, node p) - v^+ (right elem, node 0)
    rhs = -0.5 * abs(a) * np.sum(jumps ** 2)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


# --------------------------------------------------------------------- Rusanov two-state
@pytest.mark.parametrize("p", [1, 3])
def test_piecewise_constant_rusanov(p):
    nx, ny = 4, 3
    m = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.5)
    hx, hy = 1.0, 0.5
    xi, wq, _ = oracle.lgl(p)
    states = inputs.random_euler_state(m.K, 31, spread=0.3)  # one constant state per element
    q = np.repeat(states[:, :, None], m.Np, axis=2)  # (4, K, Np)
    r = m.rhs(q.reshape(-1)).reshape(4, m.K, p + 1, p + 1)  # (c, e, j, i)
    for e in range(m.K):
        ex, ey = e % nx, e // nx
        qe = states[:, e]
        right = ey * nx + (ex + 1) % nx
        left = ey * nx + (ex - 1) % nx
        top = ((ey + 1) % ny) * nx + ex
        bot = ((ey - 1) % ny) * nx + ex
        fr = tb.rusanov(qe, states[:, right], 0) - tb.euler_flux(qe, 0)
        fl = tb.rusanov(states[:, left], qe, 0) - tb.euler_flux(qe, 0)
        ft = tb.rusanov(qe, states[:, top], 1) - tb.euler_flux(qe, 1)
        fb = tb.rusanov(states[:, bot], qe, 1) - tb.euler_flux(qe, 1)
        expect = np.zeros((4, p + 1, p + 1))
        expect[:, :, p] += -(2 / hx) / wq[p] * fr[:, None]
        expect[:, :, 0] += +(2 / hx) / wq[0] * fl[:, None]
        expect[:, p, :] += -(2 / hy) / wq[p] * ft[:, None]
        expect[:, 0, :] += +(2 / hy) / wq[0] * fb[:, None]
        np.testing.assert_allclose(r[:, e], expect, atol=1e-12)
