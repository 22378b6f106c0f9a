"""Pins of the oracle's cost-based adaptivity (adapt = 1: the Krylov size and
the substep chosen by pricing two candidates after each check, after KIOPS,
which the paper cites for its phi evaluations in Section 2.3).

  * accuracy: sum_k tau^k phi_k(tau A) b_k within 10 tol nu of the dense
    augmented exponential, on DG linear operators (Burgers, Euler) at Courant
    numbers that need one and several substeps, p = 0 .. 3, with full and
    incomplete orthogonalization;
  * the error is checked only at the target size of a substep: every check
    ends in an accepted substep or a rejection (checks = substeps + rejects),
    and far fewer checks are made than by the fixed controller;
  * a replay of the logged schedule reproduces the result bitwise (the
    accepted substeps are the whole result);
  * a happy breakdown before the first target size is exact;
  * a tighter tolerance never takes fewer Krylov iterations.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs


def euler_case():
    om = oracle.Mesh(oracle.EULER2D, 4, 2, ny=3, x0=0.0, x1=10.0, y0=0.0, y1=10.0)
    x, y = om.nodes()
    q = inputs.vortex(x, y, beta=3.0).reshape(-1)
    c, dx = om.max_speed(q)
    return om, q, dx / c


def burgers_case():
    om = oracle.Mesh(oracle.BURGERS1D, 64, 2, x0=0.0, x1=2 * math.pi)
    x, _ = om.nodes()
    u = inputs.burgers_ic(x)
    c, dx = om.max_speed(u)
    return om, u, dx / c


def nu_of(tau, bs):
    return sum(tau ** k * np.linalg.norm(b) / math.factorial(k)
               for k, b in enumerate(bs) if b is not None)


@pytest.mark.parametrize("case,cr,p,iop", [("euler", 5.0, 1, 0), ("euler", 40.0, 2, 0),
                                           ("euler", 40.0, 3, 2), ("burgers", 30.0, 0, 0),
                                           ("burgers", 30.0, 2, 0), ("burgers", 3.0, 1, 2)])
def test_adapt_accuracy_and_checks(case, cr, p, iop):
    om, q, unit = euler_case() if case == "euler" else burgers_case()
    tau = cr * unit
    R = om.rhs(q)
    bs = [q if p == 0 else None] + [R * 0.5 ** k for k in range(p)]
    A = om.assemble_jvp(q)
    dense = oracle.phi_dense(A, tau, bs)
    nu = nu_of(tau, bs)
    out, st = om.phi_krylov(q, tau, bs, tol=1e-10, m_min=8, m_max=64, stats=True, iop=iop,
                            adapt=1)
    assert np.linalg.norm(out - dense) <= 10 * 1e-10 * nu, np.linalg.norm(out - dense) / nu
    assert st["checks"] == st["substeps"] + st["rejects"], st
    fixed, sf = om.phi_krylov(q, tau, bs, tol=1e-10, m_min=8, m_max=64, stats=True, iop=iop)
    assert st["checks"] * 3 <= sf["checks"], (st["checks"], sf["checks"])
    # replay of the logged schedule: bitwise the adaptive result
    rep = om.phi_krylov(q, tau, bs, tol=1e-10, m_max=64, forced=st["log"], iop=iop)
    assert np.array_equal(rep, out)


def test_adapt_breakdown_tiny_system():
    om = oracle.Mesh(oracle.BURGERS1D, 1, 1, x0=0.0, x1=1.0)
    u = np.array([0.7, 0.3])
    bs = [u, np.array([0.1, -0.2]), np.array([0.3, 0.05])]
    out, st = om.phi_krylov(u, 0.4, bs, tol=1e-10, m_min=6, m_max=10, stats=True, adapt=1)
    dense = oracle.phi_dense(om.assemble_jvp(u), 0.4, bs)
    assert st["breakdown"] >= 1 and st["substeps"] == 1
    assert np.linalg.norm(out - dense) <= 1e-13 * np.linalg.norm(dense)


def test_adapt_tolerance_monotone():
    om, q, unit = euler_case()
    R = om.rhs(q)
    its = []
    for tol in (1e-6, 1e-8, 1e-10, 1e-12):
        _, st = om.phi_krylov(q, 20 * unit, [None, R], tol=tol, m_min=8, m_max=64, stats=True,
                              adapt=1)
        its.append(st["krylov_iters"])
    assert its == sorted(its), its
