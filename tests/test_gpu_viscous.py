"""Viscous Burgers on the GPU (Section 3.1; Appendix A; zero Dirichlet ends as
in the footnote at the start of Section 6), through the C ABI, against the
FP64 oracle.

Tolerances as for the inviscid path:
  * operators: max |gpu - oracle| <= 1e-12 max |oracle|.  The diffusion part
    adds a second (p+1)-term derivative and lift per output (the auxiliary q),
    a few more ulps relative to the largest term;
  * steps on a replayed schedule: relative l2 <= 1e-12;
  * the printed errors of Table expo-burgers-tconv-smooth (GPU EPI2 / EXPRB32
    against the oracle's RK4 reference) within 0.5 %, as for the oracle.
Shapes cover one and several 256-thread tiles, a ragged last tile, the
smallest meshes (one and two elements: the neighbours are the element itself)
and every compiled degree.
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
KAPPA = 0.03


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def maxrel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


OPTS = {
    "lf_central_dir": dict(kappa=KAPPA, bc=1),
    "ef_central_dir": dict(kappa=KAPPA, flux=1, sigma=3e-4, bc=1),
    "lf_ldg_dir": dict(kappa=KAPPA, beta=0.5, bc=1),
    "ef_ldg_per": dict(kappa=0.2, flux=1, sigma=0.01, beta=0.5),
    "lf_ldgm_per": dict(kappa=0.2, beta=-0.5),
    "ef_inviscid_dir": dict(flux=1, sigma=1e-3, bc=1),
    # the face-dependent penalty sigma = kappa/100 + h max|u^+-| (Section 5.1,
    # steep gradient)
    "eflocal_central_dir": dict(kappa=0.002, flux=2, bc=1),
    "eflocal_ldg_per": dict(kappa=0.05, flux=2, beta=0.5),
}


def pair(K, p, source=None, m_max=64, precision=B.FP64, **kw):
    okw = dict(kappa=kw.get("kappa", 0.0), flux=kw.get("flux", 0), sigma=kw.get("sigma", 0.0),
               beta=kw.get("beta", 0.0), bc=kw.get("bc", 0))
    om = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=1.0, source=source, **okw)
    gm = B.Mesh(B.BURGERS1D, K, p, x0=0.0, x1=1.0, m_max=m_max, precision=precision,
                has_source=source is not None, **okw)
    if source is not None:
        gm.set_source(dev(source))
    return om, gm


SHAPES = [(1, 1), (2, 2), (1, 4), (3, 3), (37, 4), (64, 1), (200, 4), (129, 2), (19, 5), (41, 6)]


@pytest.mark.parametrize("name", list(OPTS))
@pytest.mark.parametrize("K,p", SHAPES)
def test_viscous_operators(name, K, p):
    kw = OPTS[name]
    x = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=1.0).nodes()[0]
    g = np.random.default_rng(K * 7 + p)
    src = g.standard_normal(x.size) if kw.get("bc") == 1 else None
    om, gm = pair(K, p, source=src, **kw)
    with gm:
        u = inputs.burgers_smooth(x) + 0.3 * g.standard_normal(x.size)
        v = g.standard_normal(x.size)
        qt, vt = dev(u), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        assert maxrel(host(r), om.rhs(u)) < 1e-12, maxrel(host(r), om.rhs(u))
        assert maxrel(host(w), om.jvp(u, v)) < 1e-12, maxrel(host(w), om.jvp(u, v))


@pytest.mark.parametrize("name", ["lf_central_dir", "ef_ldg_per"])
def test_viscous_operators_fp32_bulk(name):
    # FP32 bulk on float-rounded inputs: every entry within c u32 S, with S the
    # largest term (flux derivative, diffusion derivative of q, lifts) and
    # c = 8 (p + 11) for the two chained stencils (q, then its divergence)
    kw = OPTS[name]
    K, p = 37, 4
    om, gm = pair(K, p, precision=B.FP32_BULK, **kw)
    x = om.nodes()[0]
    g = np.random.default_rng(3)
    u = (inputs.burgers_smooth(x) + 0.3 * g.standard_normal(x.size)).astype(np.float32)
    v = g.standard_normal(x.size).astype(np.float32)
    with gm:
        qt = torch.tensor(u, device=DEV)
        vt = torch.tensor(v, device=DEV)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        ud, vd = u.astype(np.float64), v.astype(np.float64)
        xi, wq, D = oracle.lgl(p)
        rh = 2.0 * K
        st = rh * (np.abs(D).sum(axis=1).max() + 1.0 / wq[0])
        fmax = max(np.abs(ud).max() ** 2, np.abs(ud).max() * np.abs(vd).max())
        qmax = max(np.abs(om.gradient(ud)).max(), np.abs(om.gradient(vd)).max())
        S = st * (fmax + kw["kappa"] * max(qmax, st * max(np.abs(ud).max(), np.abs(vd).max())))
        bound = 8 * (p + 11) * 2.0 ** -24 * S
        assert np.max(np.abs(host(r).astype(np.float64) - om.rhs(ud))) <= bound
        assert np.max(np.abs(host(w).astype(np.float64) - om.jvp(ud, vd))) <= bound


def test_source_requires_has_source():
    with B.Mesh(B.BURGERS1D, 8, 2, kappa=KAPPA) as gm:
        with pytest.raises(B.ExpdgError) as ei:
            gm.set_source(dev(np.zeros(gm.n)))
        assert ei.value.code == B.EINVAL


def test_source_is_added_once():
    K, p = 16, 3
    x = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=1.0).nodes()[0]
    _, s = inputs.burgers_mms(x, KAPPA)
    om, gm = pair(K, p, source=s, kappa=KAPPA, bc=1)
    with gm, B.Mesh(B.BURGERS1D, K, p, x0=0.0, x1=1.0, kappa=KAPPA, bc=1) as g0:
        u = dev(inputs.burgers_mms(x, KAPPA)[0])
        r1, r0 = torch.empty_like(u), torch.empty_like(u)
        gm.rhs(u, r1)
        g0.rhs(u, r0)
        assert np.max(np.abs(host(r1) - host(r0) - s)) <= 1e-12 * np.max(np.abs(s))


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32, B.EXPRB42])
@pytest.mark.parametrize("name", ["lf_central_dir", "ef_central_dir", "lf_ldg_dir"])
def test_viscous_steps_replayed(scheme, name):
    # stiff steps: k = 4, N_e = 40, dt = 0.1 (Cr_d = 161 as in the paper's table)
    kw = OPTS[name]
    om, gm = pair(40, 4, **kw)
    x = om.nodes()[0]
    u0 = inputs.burgers_smooth(x)
    ok = dict(tol=1e-10, m_min=5, m_max=64)
    with gm:
        q = dev(u0)
        qp = torch.empty_like(q)
        q_o, qp_o = u0, None
        for k in range(3):
            q_o, qp_o, st = om.step(scheme, 0.1, q_o, qp_o, stats=True, **ok)
            gm.step(scheme, 0.1, q, qp, k > 0, B.make_opts(forced=st["log"], **ok))
            assert rel(host(q), q_o) < 1e-12, (k, rel(host(q), q_o))


def test_mms_steps_with_source():
    # the manufactured solution's first EXPRB32 steps (dt = 5e-5, k = 3, N_e = 80)
    K, p = 80, 3
    x = oracle.Mesh(oracle.BURGERS1D, K, p, x0=0.0, x1=1.0).nodes()[0]
    u, s = inputs.burgers_mms(x, KAPPA)
    om, gm = pair(K, p, source=s, m_max=30, kappa=KAPPA, flux=1, sigma=3e-4, bc=1)
    ok = dict(tol=1e-12, m_min=5, m_max=30)
    with gm:
        q = dev(u)
        q_o = u
        for k in range(5):
            q_o, _, st = om.step(B.EXPRB32, 5e-5, q_o, None, stats=True, **ok)
            gm.step(B.EXPRB32, 5e-5, q, None, False, B.make_opts(forced=st["log"], **ok))
        # the increment q - u is far smaller than the residual's terms (the
        # state starts at the manufactured steady solution), so the FP64
        # target applies to the state, as for every other step
        assert rel(host(q), q_o) < 1e-12


def test_temporal_table_on_gpu():
    """Table expo-burgers-tconv-smooth (LF rows) through expdg_integrate: the
    GPU's EPI2 and EXPRB32 errors against the oracle's RK4 reference within
    0.5 % of the printed ones."""
    printed = {("epi2", 0.1): 5.411e-4, ("epi2", 0.01): 4.943e-6,
               ("exprb32", 0.1): 9.575e-05, ("exprb32", 0.01): 1.042e-7}
    om, gm = pair(40, 4, kappa=KAPPA, bc=1)
    x = om.nodes()[0]
    u0 = inputs.burgers_smooth(x)
    saved = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        ref = om.rk4(u0, 2e-5, 50000)
    finally:
        oracle.set_num_threads(saved)
    M = om.mass()
    with gm:
        for (name, dt), err_p in printed.items():
            scheme = B.EPI2 if name == "epi2" else B.EXPRB32
            q = dev(u0)
            gm.integrate(scheme, dt, int(round(1.0 / dt)), q, None, False,
                         B.make_opts(1e-12, 5, 64))
            err = math.sqrt(float(np.sum(M * (host(q) - ref) ** 2)))
            assert abs(err / err_p - 1.0) <= 5e-3, (name, dt, err, err_p)


def test_shock_temporal_table_on_gpu():
    """Table expo-burgers-tconv-shock (Section 5.1, steep gradient: kappa =
    0.002, k = 4, N_e = 160, LF and the entropy flux with the face-dependent
    penalty) through expdg_integrate: the GPU's EPI2 and EXPRB32 errors at
    t = 1 against the reference of the paper's discretization (k = 10,
    N_e = 160; tests/golden, written by the oracle) within 0.5 % of the
    printed ones (EXPRB32 at dt = 0.02 within 10 %, as for the oracle)."""
    from tests.test_oracle_shock import _error, _read, _reference
    ref = _reference()
    for r in _read("burgers_viscous_shock_tconv.txt"):
        flux = B.FLUX_LF if r[0] == "LF" else B.FLUX_EF_LOCAL
        dt = float(r[1])
        print(f"shock table: flux {r[0]} dt {dt}", flush=True)
        with B.Mesh(B.BURGERS1D, 160, 4, x0=0.0, x1=1.0, kappa=0.002, bc=B.BC_DIRICHLET,
                    flux=flux) as gm:
            x = gm.nodes()[0]
            for col, scheme in ((3, B.EPI2), (4, B.EXPRB32)):
                q = dev(np.sin(2.0 * math.pi * x))
                gm.integrate(scheme, dt, int(round(1.0 / dt)), q, None, False,
                             B.make_opts(1e-10, 5, 64))
                e = _error(host(q), 4, 160, ref)
                tolr = 0.10 if (scheme == B.EXPRB32 and dt == 0.02) else 0.005
                assert abs(e / float(r[col]) - 1.0) <= tolr, (r[0], dt, scheme, e, r[col])
