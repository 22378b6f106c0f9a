"""The cost-based Krylov adaptivity (adapt = 1, after KIOPS, Section 2.3) on
the GPU against the oracle's.

Both sides check the error only at the target size of a substep and take the
same decisions from the same error ratios, so:
  * the accepted substeps (size, length, last flag) are identical, and so
    are the numbers of rejections and of checks, on phi evaluations that take
    one and several substeps (Burgers and Euler, p = 0 .. 3, full and
    incomplete orthogonalization, FP64); at Courant 40, where the estimates
    come from exponentials with about eight squarings and the smallest have
    about one correct digit, the substeps agree in number and their sizes
    within two vectors;
  * the results agree within 1e-12 relative when the schedule is replayed and
    within 10 tol nu on the adaptive runs;
  * steps of EPI2, EPI3 and EXPRB32 with adapt = 1 take the oracle's decisions
    and agree within 1e-10 relative;
  * served solves with adapt = 1 are bitwise equal to expdg_step.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2011_01316_amd import binding as B
from paper_2011_01316_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def meshes(case):
    if case == "euler":
        kw = dict(x0=0.0, x1=10.0, y0=0.0, y1=10.0)
        om = oracle.Mesh(oracle.EULER2D, 6, 3, ny=5, **kw)
        gm = B.Mesh(B.EULER2D, 6, 3, ny=5, m_max=64, **kw)
        x, y = om.nodes()
        q = inputs.vortex(x, y, beta=3.0).reshape(-1)
    else:
        om = oracle.Mesh(oracle.BURGERS1D, 64, 2, x0=0.0, x1=2 * math.pi)
        gm = B.Mesh(B.BURGERS1D, 64, 2, x0=0.0, x1=2 * math.pi, m_max=64)
        x, _ = om.nodes()
        q = inputs.burgers_ic(x)
    c, dx = om.max_speed(q)
    return om, gm, q, dx / c


@pytest.mark.parametrize("case,cr,p,iop", [("euler", 5.0, 1, 0), ("euler", 40.0, 2, 0),
                                           ("euler", 40.0, 3, 2), ("burgers", 30.0, 0, 0),
                                           ("burgers", 30.0, 2, 0), ("burgers", 3.0, 1, 2)])
def test_adapt_phi_decisions(case, cr, p, iop):
    print(f"adapt phi: {case} Courant {cr} p {p} iop {iop}", flush=True)
    om, gm, q, unit = meshes(case)
    tau = cr * unit
    R = om.rhs(q)
    bs = [q if p == 0 else None] + [R * 0.5 ** k for k in range(p)]
    nu = sum(tau ** k * np.linalg.norm(b) / math.factorial(k)
             for k, b in enumerate(bs) if b is not None)
    ref, st = om.phi_krylov(q, tau, bs, tol=1e-10, m_min=8, m_max=64, stats=True, iop=iop,
                            adapt=1)
    with gm:
        qt = dev(q)
        bt = [None if b is None else dev(b) for b in bs]
        w = torch.empty_like(qt)
        gs = B.make_stats()
        gm.phi_krylov(qt, tau, bt, w, B.make_opts(1e-10, 8, 64, iop=iop, adapt=1), gs)
        got = host(w)
        gs = B.stats_dict(gs)
        gm.phi_krylov(qt, tau, bt, w, B.make_opts(1e-10, 8, 64, iop=iop, forced=st["log"]))
        rep = host(w)
    if cr < 40:
        assert [(m, l) for (m, _, l) in gs["log"]] == [(m, l) for (m, _, l) in st["log"]]
        assert np.allclose([d for (_, d, _) in gs["log"]], [d for (_, d, _) in st["log"]],
                           rtol=1e-14, atol=0)
        assert gs["rejects"] == st["rejects"] and gs["checks"] == st["checks"], (gs, st)
        assert gs["m_next"] == st["m_next"]
    else:
        # Courant 40: the error estimates come from exponentials with about
        # eight squarings, so a tiny estimate (1e-12 of the largest entry)
        # has about one correct digit on either side, and a size derived from
        # it may differ by a vector or two; the substeps agree in number
        assert len(gs["log"]) == len(st["log"]), (gs["log"], st["log"])
        assert all(abs(a[0] - b[0]) <= 2 for a, b in zip(gs["log"], st["log"]))
    # replayed schedule: 1e-12, or 2e-11 at Courant 30 and 40 where every
    # substep's small exponential takes about eight squarings (as for the
    # fixed controller's stress cases)
    assert rel(rep, ref) <= (2e-11 if cr >= 30 else 1e-12), rel(rep, ref)
    assert np.linalg.norm(got - ref) <= 10 * 1e-10 * nu


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32])
def test_adapt_steps(scheme):
    print(f"adapt steps: scheme {scheme}", flush=True)
    om, gm, q0, unit = meshes("euler")
    dt = 8.0 * unit
    with gm:
        q = dev(q0)
        qp = torch.empty_like(q)
        oq, oqp = q0, None
        for k in range(3):
            oq, oqp, st = om.step(scheme, dt, oq, oqp, tol=1e-10, m_min=8, m_max=64,
                                  stats=True, adapt=1)
            gs = B.make_stats()
            gm.step(scheme, dt, q, qp, k > 0, B.make_opts(1e-10, 8, 64, adapt=1), gs)
            gs = B.stats_dict(gs)
            assert [(m, l) for (m, _, l) in gs["log"]] == [(m, l) for (m, _, l) in st["log"]]
            assert gs["rejects"] == st["rejects"]
        assert rel(host(q), oq) <= 1e-10


def test_adapt_served_bitwise():
    # served solves with adapt = 1 (a mix of equations and sizes in one
    # server) against expdg_step on their own meshes
    from tests.test_gpu_serve import burgers_case, euler_case, serve_all, standalone
    print("adapt served mix", flush=True)
    cases = [burgers_case(40, 1, 0.1), euler_case(10, 2, 4.0, 6.0, 3.0),
             burgers_case(200, 4, 2.0, scheme=B.EPI2), euler_case(12, 3, 5.0, 5.0, 5.0)]
    for r, _ in cases:
        r.adapt = 1
    with B.Server(hbm_budget=1 << 30, max_active=8) as srv:
        got = serve_all(srv, cases)
    for k, (r, q0) in enumerate(cases):
        want, _ = standalone(r, q0)
        np.testing.assert_array_equal(got[k][0], want)
