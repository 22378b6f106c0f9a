"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (FP64 path):
  * operators (R, L v): max |gpu - oracle| <= 1e-12 * max |oracle| per call.
    Both sides evaluate the same sums in a different order; a (p+1)-term
    derivative, a face flux and a lift each lose a few ulps (2^-52 ~ 2.2e-16)
    relative to the largest term, far below 1e-12.
  * small exponential: normwise 1e-13 (Pade(6,6) with identical scaling s;
    rounding grows with the s squarings).
  * phi combinations and steps on a replayed (forced) schedule: relative l2
    <= 1e-12 (the target for the FP64 path).
  * adaptive runs: identical substep decisions where the error estimate is not
    within rounding of a threshold, and the result within 10 tol nu of the
    oracle's.
Inputs come from paper_2011_01316_amd.inputs at the oracle's nodes.
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
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxrel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def burgers_pair(K, p, m_max=64, precision=B.FP64, x1=2 * math.pi):
    om = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=x1)
    gm = B.Mesh(B.BURGERS1D, K, p, x0=0.0, x1=x1, m_max=m_max, precision=precision)
    return om, gm


def euler_pair(nx, ny, p, m_max=64, precision=B.FP64, L=(0.0, 10.0, 0.0, 10.0)):
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, x0=L[0], x1=L[1], y0=L[2], y1=L[3])
    gm = B.Mesh(B.EULER2D, nx, p, ny=ny, x0=L[0], x1=L[1], y0=L[2], y1=L[3], m_max=m_max,
                precision=precision)
    return om, gm


# ------------------------------------------------------------------ geometry
@pytest.mark.parametrize("eq,nx,ny,p", [(1, 7, 1, 3), (2, 3, 5, 4), (2, 1, 1, 6)])
def test_nodes_match_oracle(eq, nx, ny, p):
    om = oracle.Mesh(eq, nx, p, ny=ny, x0=-1.0, x1=2.0, y0=0.5, y1=1.5)
    with B.Mesh(eq, nx, p, ny=ny, x0=-1.0, x1=2.0, y0=0.5, y1=1.5) as gm:
        x, y = gm.nodes()
        assert gm.n == om.n
    ox, oy = om.nodes()
    np.testing.assert_allclose(x, ox, atol=1e-15)
    if eq == 2:
        np.testing.assert_allclose(y, oy, atol=1e-15)


# ------------------------------------------------------------------ operators
BURGERS_SHAPES = [(1, 1), (2, 2), (3, 1), (17, 3), (64, 2), (100, 4), (9, 5), (33, 6)]
EULER_SHAPES = [(1, 1, 1), (1, 1, 4), (2, 3, 2), (5, 4, 3), (7, 3, 4), (3, 2, 5), (2, 2, 6),
                (64, 64, 4), (33, 17, 3)]


@pytest.mark.parametrize("K,p", BURGERS_SHAPES)
def test_burgers_operators(K, p):
    om, gm = burgers_pair(K, p)
    with gm:
        u = inputs.random_vector(om.n, K * 10 + p) + 0.2
        v = inputs.random_vector(om.n, K * 10 + p + 1)
        qt, vt = dev(u), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        assert maxrel(host(r), om.rhs(u)) < 1e-12
        assert maxrel(host(w), om.jvp(u, v)) < 1e-12


@pytest.mark.parametrize("nx,ny,p", EULER_SHAPES)
def test_euler_operators(nx, ny, p):
    om, gm = euler_pair(nx, ny, p, L=(0.0, 2.0, -1.0, 0.5))
    with gm:
        q = inputs.random_euler_state(om.K * om.Np, nx * 100 + ny * 10 + p).reshape(-1)
        v = inputs.random_vector(om.n, 7 + p)
        qt, vt = dev(q), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        assert maxrel(host(r), om.rhs(q)) < 1e-12
        assert maxrel(host(w), om.jvp(q, v)) < 1e-12


def test_vortex_operators_full_size():
    # the 64 x 64, p = 4 vortex workload itself (409,600 DOF), every entry
    om, gm = euler_pair(64, 64, 4)
    with gm:
        x, y = om.nodes()
        q = inputs.vortex(x, y).reshape(-1)
        v = om.rhs(q)
        qt, vt = dev(q), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        assert maxrel(host(r), om.rhs(q)) < 1e-12
        assert maxrel(host(w), om.jvp(q, v)) < 1e-12


def test_operator_errors_are_reported():
    with B.Mesh(B.BURGERS1D, 4, 2) as gm:
        qt = dev(np.ones(gm.n))
        with pytest.raises(B.ExpdgError) as ei:
            gm.jvp(qt, qt, qt)
        assert ei.value.code == B.EINVAL


# ------------------------------------------------------------------ small exponential
@pytest.mark.parametrize("n", [1, 2, 5, 17, 31, 33, 64, 65])
def test_small_expm(n):
    rng = np.random.default_rng(n)
    for scale in [0.1, 3.0, 40.0]:
        A = rng.standard_normal((n, n)) * scale / math.sqrt(n)
        A -= np.eye(n) * max(0.0, np.max(np.linalg.eigvals(A).real))
        Ad = dev(A)
        Ed = torch.empty_like(Ad)
        B.expdg_small_expm(n, Ad, Ed)
        E = host(Ed)
        ref = oracle.expm(A)
        assert np.linalg.norm(E - ref) <= 1e-13 * max(1.0, np.linalg.norm(ref)) * max(1.0, scale), scale


# ------------------------------------------------------------------ phi combinations
def run_phi(om, gm, qref, tau, bs, tol=1e-10, m_min=5, m_max=30, check_every=1):
    ref, st = om.phi_krylov(qref, tau, bs, tol=tol, m_min=m_min, m_max=m_max,
                            check_every=check_every, stats=True)
    bt = [None if b is None else dev(b) for b in bs]
    qt = dev(qref)
    w = torch.empty_like(qt)
    # replay of the oracle's schedule
    gm.phi_krylov(qt, tau, bt, w, B.make_opts(tol, m_min, m_max, check_every, forced=st["log"]))
    forced = host(w)
    # free adaptive run
    gs = B.make_stats()
    gm.phi_krylov(qt, tau, bt, w, B.make_opts(tol, m_min, m_max, check_every), gs)
    adaptive = host(w)
    return ref, st, forced, adaptive, B.stats_dict(gs)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_phi_burgers_c1(p):
    om, gm = burgers_pair(64, 2, m_max=30)
    with gm:
        x, _ = om.nodes()
        u = inputs.burgers_ic(x)
        R = om.rhs(u)
        bs = [u if p == 0 else None] + [R * (0.5 ** k) for k in range(p)]
        ref, st, forced, adaptive, gs = run_phi(om, gm, u, 0.05, bs)
        assert rel(forced, ref) < 1e-12
        nu = sum(0.05 ** k * np.linalg.norm(bs[k]) / math.factorial(k)
                 for k in range(p + 1) if bs[k] is not None)
        assert np.linalg.norm(adaptive - ref) <= 10 * 1e-10 * nu
        assert [m for (m, _, _) in gs["log"]] == [m for (m, _, _) in st["log"]]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_phi_euler_substeps(p):
    # a small mesh at large Courant number: several substeps and rejections
    om, gm = euler_pair(6, 5, 3, m_max=16)
    with gm:
        x, y = om.nodes()
        q = inputs.vortex(x, y, beta=3.0).reshape(-1)
        R = om.rhs(q)
        b = [None, R, inputs.random_vector(om.n, 3) * 0.1, inputs.random_vector(om.n, 4)][: p + 1]
        c, dx = om.max_speed(q)
        tau = 40.0 * dx / c
        ref, st, forced, adaptive, gs = run_phi(om, gm, q, tau, b, m_min=4, m_max=16)
        assert st["substeps"] > 1
        nu = sum(tau ** k * np.linalg.norm(b[k]) / math.factorial(k)
                 for k in range(1, p + 1))
        # Stress case (Courant number 40, m_max 16): every substep's small
        # exponential takes s ~ 8 squarings (rounding ~2^s u ~ 6e-14) and the
        # substeps compound it, so the bar is 2e-11 here rather than 1e-12.
        err = np.linalg.norm(forced - ref)
        assert err < 2e-11 * np.linalg.norm(ref), (err / np.linalg.norm(ref), err / nu, st["substeps"])
        assert np.linalg.norm(adaptive - ref) <= 20 * 1e-10 * nu
        assert gs["substeps"] == st["substeps"] and gs["rejects"] == st["rejects"]


def test_phi_breakdown_tiny_system():
    # 1 element, p = 1 Burgers: 2 DOF + 2 augmented entries, the Krylov space
    # is exhausted (happy breakdown) before m_min
    om, gm = burgers_pair(1, 1, m_max=10, x1=1.0)
    with gm:
        u = np.array([0.7, 0.3])
        bs = [u, np.array([0.1, -0.2]), np.array([0.3, 0.05])]
        ref, st, forced, adaptive, gs = run_phi(om, gm, u, 0.4, bs, m_min=6, m_max=10)
        dense = oracle.phi_dense(om.assemble_jvp(u), 0.4, bs)
        assert st["breakdown"] >= 1 and gs["breakdown"] >= 1
        assert rel(ref, dense) < 1e-12
        assert rel(forced, ref) < 1e-12 and rel(adaptive, ref) < 1e-12


def test_phi_breakdown_euler_fused_dots():
    # 1 x 1 mesh, p = 1 Euler: 16 DOF + 2 augmented entries.  The Krylov space
    # is exhausted before m_max, so the breakdown is detected by the step
    # finish of the 2D path (dot pass in the linear operator's epilogue).
    om, gm = euler_pair(1, 1, 1, m_max=30, L=(0.0, 1.0, 0.0, 1.0))
    with gm:
        x, y = om.nodes()
        q = inputs.vortex(x * 10.0, y * 10.0, beta=2.0).reshape(-1)
        R = om.rhs(q)
        bs = [None, R, inputs.random_vector(om.n, 7) * 0.1]
        c, dx = om.max_speed(q)
        tau = 2.0 * dx / c
        ref, st, forced, adaptive, gs = run_phi(om, gm, q, tau, bs, m_min=6, m_max=30)
        dense = oracle.phi_dense(om.assemble_jvp(q), tau, bs)
        assert st["breakdown"] >= 1 and gs["breakdown"] >= 1
        assert rel(ref, dense) < 1e-12
        assert rel(forced, ref) < 1e-12 and rel(adaptive, ref) < 1e-12


def test_phi_forced_full_basis():
    # one substep with the largest basis (m = 64): the step that finishes the
    # last dimension writes basis slot 65 and Hessenberg column 64, the edges
    # of the workspace
    om, gm = euler_pair(4, 4, 3, m_max=64)
    with gm:
        x, y = om.nodes()
        q = inputs.vortex(x, y, beta=3.0).reshape(-1)
        R = om.rhs(q)
        c, dx = om.max_speed(q)
        tau = 3.0 * dx / c
        bs = [None, R, inputs.random_vector(om.n, 11) * 0.1]
        sched = [(64, tau, 1)]
        ref = om.phi_krylov(q, tau, bs, forced=sched)
        qt = dev(q)
        bt = [None if b is None else dev(b) for b in bs]
        w = torch.empty_like(qt)
        st = B.make_stats()
        gm.phi_krylov(qt, tau, bt, w, B.make_opts(forced=sched), st)
        assert B.stats_dict(st)["krylov_iters"] == 65
        assert rel(host(w), ref) < 1e-12, rel(host(w), ref)


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32, B.EXPRB42])
def test_integrate_equals_steps(scheme):
    # several steps in one call: bitwise the same as one call per step
    om, gm = euler_pair(12, 12, 3, m_max=40)
    with gm:
        x, y = om.nodes()
        q0 = dev(inputs.vortex(x, y, beta=4.0).reshape(-1))
        c, dx = om.max_speed(host(q0))
        dt = 5.0 * dx / c
        opts = B.make_opts(1e-10, 8, 40)
        qa, pa = q0.clone(), torch.empty_like(q0)
        sa = B.make_stats()
        for k in range(4):
            gm.step(scheme, dt, qa, pa, k > 0, opts, sa)
        qb, pb = q0.clone(), torch.empty_like(q0)
        sb = B.make_stats()
        gm.integrate(scheme, dt, 4, qb, pb, False, opts, sb)
        assert torch.equal(qa, qb) and torch.equal(pa, pb)
        da, db = B.stats_dict(sa), B.stats_dict(sb)
        assert da["krylov_iters"] == db["krylov_iters"] and da["log"] == db["log"]


def test_integrate_rejects_missing_history():
    om, gm = euler_pair(4, 4, 2)
    with gm:
        q = dev(inputs.vortex(*om.nodes()).reshape(-1))
        with pytest.raises(B.ExpdgError) as ei:
            gm.integrate(B.EPI3, 0.01, 2, q)
        assert ei.value.code == B.EINVAL


def test_phi_zero_inputs():
    om, gm = burgers_pair(8, 2)
    with gm:
        u = dev(inputs.burgers_ic(om.nodes()[0]))
        z = torch.zeros_like(u)
        w = torch.full_like(u, 7.0)
        gm.phi_krylov(u, 0.1, [None, z], w, B.make_opts())
        assert np.all(host(w) == 0.0)
        b0 = dev(inputs.random_vector(om.n, 1))
        gm.phi_krylov(u, 0.0, [b0, z], w, B.make_opts())
        assert np.array_equal(host(w), host(b0))


# ------------------------------------------------------------------ steps
@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32, B.EXPRB42])
def test_step_burgers_c1(scheme):
    om, gm = burgers_pair(64, 2, m_max=30)
    with gm:
        x, _ = om.nodes()
        u = inputs.burgers_ic(x)
        kw = dict(tol=1e-10, m_min=5, m_max=30)
        q_o, qp_o = u, None
        q = dev(u)
        qp = torch.empty_like(q)
        have = False
        for k in range(4):
            q_o2, qp_o2, st = om.step(scheme, 0.05, q_o, qp_o, stats=True, **kw)
            gm.step(scheme, 0.05, q, qp, have, B.make_opts(forced=st["log"], **kw))
            have = True
            q_o, qp_o = q_o2, qp_o2
            assert rel(host(q), q_o) < 1e-12, k
            assert rel(host(qp), qp_o) < 1e-12, k


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32, B.EXPRB42])
def test_step_vortex_small(scheme):
    # 12 x 12 quads: the beta = 5 vortex on 8 x 8 is under-resolved and the
    # collocation scheme (oracle included) blows up there
    om, gm = euler_pair(12, 12, 3, m_max=64)
    with gm:
        x, y = om.nodes()
        q0 = inputs.vortex(x, y).reshape(-1)
        c, dx = om.max_speed(q0)
        dt = 5.0 * dx / c
        kw = dict(tol=1e-10, m_min=10, m_max=64)
        q_o, qp_o = q0, None
        q = dev(q0)
        qp = torch.empty_like(q)
        have = False
        for k in range(3):
            q_o2, qp_o2, st = om.step(scheme, dt, q_o, qp_o, stats=True, **kw)
            gm.step(scheme, dt, q, qp, have, B.make_opts(forced=st["log"], **kw))
            have = True
            q_o, qp_o = q_o2, qp_o2
            assert rel(host(q), q_o) < 1e-12, (k, rel(host(q), q_o))


def test_step_adaptive_decisions_match():
    # free adaptive runs on both sides: same schedule, results within 10 tol
    om, gm = burgers_pair(64, 2, m_max=30)
    with gm:
        x, _ = om.nodes()
        u = inputs.burgers_ic(x)
        kw = dict(tol=1e-10, m_min=5, m_max=30)
        q = dev(u)
        qp = torch.empty_like(q)
        q_o, qp_o = u, None
        for k in range(10):
            q_o, qp_o, st = om.step(B.EPI3, 1e-2, q_o, qp_o, stats=True, **kw)
            gs = B.make_stats()
            gm.step(B.EPI3, 1e-2, q, qp, k > 0, B.make_opts(**kw), gs)
            assert [m for (m, _, _) in B.stats_dict(gs)["log"]] == [m for (m, _, _) in st["log"]]
        assert rel(host(q), q_o) < 1e-9


def test_c1_full_run():
    # C1: K = 64, p = 2, EPI2, dt = 1e-2 to t = 0.5 (50 steps), forced per step
    om, gm = burgers_pair(64, 2, m_max=30)
    with gm:
        x, _ = om.nodes()
        u = inputs.burgers_ic(x)
        kw = dict(tol=1e-10, m_min=5, m_max=30)
        q = dev(u)
        q_o = u
        for k in range(50):
            q_o, _, st = om.step(B.EPI2, 1e-2, q_o, None, stats=True, **kw)
            gm.step(B.EPI2, 1e-2, q, None, False, B.make_opts(forced=st["log"], **kw))
        assert rel(host(q), q_o) < 1e-12


def test_vortex_c2_one_step():
    # the 64 x 64, p = 4 workload: one EPI3 step (EPI2 start + one EPI3) replaying
    # the oracle's schedule
    om, gm = euler_pair(64, 64, 4, m_max=64)
    with gm:
        x, y = om.nodes()
        q0 = inputs.vortex(x, y).reshape(-1)
        c, dx = om.max_speed(q0)
        dt = 5.0 * dx / c
        kw = dict(tol=1e-10, m_min=10, m_max=64)
        q = dev(q0)
        qp = torch.empty_like(q)
        q_o, qp_o = q0, None
        for k in range(2):
            q_o, qp_o, st = om.step(B.EPI3, dt, q_o, qp_o, stats=True, **kw)
            gm.step(B.EPI3, dt, q, qp, k > 0, B.make_opts(forced=st["log"], **kw))
            assert rel(host(q), q_o) < 1e-12, k


def test_step_is_deterministic():
    om, gm = euler_pair(16, 16, 4)
    with gm:
        x, y = om.nodes()
        q0 = dev(inputs.vortex(x, y).reshape(-1))
        outs = []
        for _ in range(2):
            q = q0.clone()
            gm.step(B.EPI2, 0.05, q, None, False, B.make_opts(1e-10, 10, 64))
            outs.append(host(q))
        assert np.array_equal(outs[0], outs[1])


def test_step_rejects_bad_arguments():
    with B.Mesh(B.BURGERS1D, 4, 2) as gm:
        q = dev(np.ones(gm.n))
        with pytest.raises(B.ExpdgError) as ei:
            gm.step(7, 0.1, q)
        assert ei.value.code == B.EINVAL
        with pytest.raises(B.ExpdgError):
            gm.step(B.EPI2, -1.0, q)
        with pytest.raises(B.ExpdgError):
            gm.step(B.EPI2, 0.1, q, opts=B.make_opts(m_max=99))
        assert np.all(host(q) == 1.0)
