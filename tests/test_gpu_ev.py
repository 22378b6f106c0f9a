"""Entropy viscosity for 2D Euler on the GPU (Section 3.2, "Artificial
viscosity"), through the C ABI, against the oracle.

  * the nodal viscosity (entropy residual, element viscosity min(nu_max,
    nu_E), vertex averages, bilinear reconstruction) to 1e-12 of its largest
    value, with the cap branch, the residual branch and a mix of both, on
    every compiled degree, a single element (every neighbour is the element
    itself) and ragged last blocks;
  * the residual and the linear operator with a given nodal viscosity (the
    diffusion div(nu grad v) with central fluxes added to both) to 1e-12 of
    the largest output;
  * a phi combination with the viscosity, replaying the oracle's substeps, to
    1e-12 relative, and the adaptive run taking the oracle's decisions;
  * two steps of each scheme on the shear layer, the viscosity recomputed in
    each step from q^n and q^{n-1}, to 1e-12 relative at the state level;
    several steps in one call bitwise equal to one call per step;
  * FP32 bulk: one EPI2 step within 1e-6 of the FP64 oracle;
  * c_max = 0: the viscosity vanishes exactly and steps equal the inviscid
    ones to 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2011_01316_amd import binding as B
from paper_2011_01316_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
DOM = dict(x0=0.0, x1=1.0, y0=0.0, y1=1.0)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxrel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def states(m, seed):
    """The shear layer at the mesh's nodes and a perturbed earlier state."""
    x, y = m.nodes()
    q = inputs.shear_layer(x, y, seed=seed).reshape(-1)
    g = np.random.default_rng(seed + 1)
    qp = q * (1.0 + 1e-3 * g.standard_normal(q.size))
    return q, qp


SHAPES = [(1, 1, 1), (1, 1, 6), (4, 3, 2), (3, 5, 3), (6, 4, 4), (5, 3, 5), (3, 4, 6), (7, 2, 1),
          (5, 1, 3), (1, 4, 4)]


@pytest.mark.parametrize("nx,ny,p", SHAPES)
@pytest.mark.parametrize("ce", [1e-4, 1.0, 1e9])
def test_viscosity(nx, ny, p, ce):
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=ce, ev_cmax=0.1, **DOM)
    q, qp = states(om, nx * 10 + p)
    want = om.entropy_viscosity(q, qp, 0.02)
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=ce, ev_cmax=0.1, **DOM) as gm:
        nu = torch.empty(gm.K * gm.Np, dtype=torch.float64, device=DEV)
        gm.entropy_viscosity(dev(q), dev(qp), 0.02, nu)
        assert np.max(want) > 0
        assert maxrel(host(nu), want) < 1e-12, maxrel(host(nu), want)


@pytest.mark.parametrize("nx,ny,p", SHAPES)
def test_operators_with_viscosity(nx, ny, p):
    om0 = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, **DOM)
    g = np.random.default_rng(p + 10 * nx)
    nu = g.uniform(0.0, 0.02, om0.K * om0.Np)
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, nu=nu, **DOM)
    q = inputs.random_euler_state(om.K * om.Np, p).reshape(-1)
    v = g.standard_normal(om.n)
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM) as gm:
        gm.set_viscosity(dev(nu))
        qt, vt = dev(q), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        ro, wo = om.rhs(q), om.jvp(q, v)
        assert maxrel(host(r), ro) < 1e-12, maxrel(host(r), ro)
        assert maxrel(host(w), wo) < 1e-12, maxrel(host(w), wo)
        # the viscosity is active: the operator differs from the inviscid one
        # (except on one element of degree 1, periodic with itself, where the
        # central gradient of every field vanishes: g = D v + ({{v}} - v^-) / w_0 = 0)
        if (nx, ny, p) != (1, 1, 1):
            assert maxrel(om0.jvp(q, v), wo) > 1e-6


@pytest.mark.parametrize("iop", [0, 2])
def test_phi_with_viscosity(iop):
    nx, ny, p = 6, 5, 3
    om0 = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM)
    q, qp = states(om0, 3)
    nu = om0.entropy_viscosity(q, qp, 0.01)
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, nu=nu, **DOM)
    R = om.rhs(q)
    b = [None, R, 0.1 * np.random.default_rng(4).standard_normal(om.n)]
    c, dx = om.max_speed(q)
    tau = 10.0 * dx / c
    ref, st = om.phi_krylov(q, tau, b, tol=1e-10, m_min=4, m_max=16, stats=True, iop=iop)
    assert st["substeps"] > 1
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, m_max=16, **DOM) as gm:
        gm.set_viscosity(dev(nu))
        bt = [None if bb is None else dev(bb) for bb in b]
        qt = dev(q)
        w = torch.empty_like(qt)
        gm.phi_krylov(qt, tau, bt, w, B.make_opts(1e-10, 4, 16, forced=st["log"], iop=iop))
        assert rel(host(w), ref) < 1e-12, rel(host(w), ref)
        gs = B.make_stats()
        gm.phi_krylov(qt, tau, bt, w, B.make_opts(1e-10, 4, 16, iop=iop), gs)
        d = B.stats_dict(gs)
        assert d["substeps"] == st["substeps"] and d["rejects"] == st["rejects"]


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB32, B.EXPRB42])
def test_steps_shear_layer(scheme):
    nx, ny, p = 8, 8, 3
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM)
    x, y = om.nodes()
    q0 = inputs.shear_layer(x, y, seed=0).reshape(-1)
    c, dx = om.max_speed(q0)
    dt = 5.0 * dx / c
    kw = dict(tol=1e-10, m_min=10, m_max=64)
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM) as gm:
        q_o, qp_o = q0, None
        q = dev(q0)
        qp = torch.empty_like(q)
        for k in range(2):
            q_o, qp_o, st = om.step(scheme, dt, q_o, qp_o, stats=True, **kw)
            gm.step(scheme, dt, q, qp, k > 0, B.make_opts(forced=st["log"], **kw))
            assert rel(host(q), q_o) < 1e-12, (k, rel(host(q), q_o))
        # the viscosity the next step would take, from q^2 after q^1
        nu = torch.empty(gm.K * gm.Np, dtype=torch.float64, device=DEV)
        gm.entropy_viscosity(q, qp, dt, nu)
        want = om.entropy_viscosity(q_o, qp_o, dt)
        assert np.max(want) > 0 and maxrel(host(nu), want) < 1e-10


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3, B.EXPRB42])
def test_integrate_equals_steps_with_viscosity(scheme):
    # several steps in one call: bitwise the same as one call per step, each
    # step's viscosity from its own q^n and q^{n-1}
    nx, ny, p = 8, 8, 3
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM) as gm:
        x, y = gm.nodes()
        q0 = dev(inputs.shear_layer(x, y, seed=4).reshape(-1))
        dt = 5.0 * gm.dx_min / gm.max_speed(q0)
        opts = B.make_opts(1e-10, 10, 64)
        qa, pa = q0.clone(), torch.empty_like(q0)
        sa = B.make_stats()
        for k in range(3):
            gm.step(scheme, dt, qa, pa, k > 0, opts, sa)
        qb, pb = q0.clone(), torch.empty_like(q0)
        sb = B.make_stats()
        gm.integrate(scheme, dt, 3, qb, pb, False, opts, sb)
        assert torch.equal(qa, qb) and torch.equal(pa, pb)
        da, db = B.stats_dict(sa), B.stats_dict(sb)
        assert da["krylov_iters"] == db["krylov_iters"] and da["log"] == db["log"]


def test_fp32_bulk_step():
    nx, ny, p = 6, 6, 3
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.1, **DOM)
    x, y = om.nodes()
    q0 = inputs.shear_layer(x, y, seed=2).reshape(-1)
    c, dx = om.max_speed(q0)
    dt = 5.0 * dx / c
    ref = om.step(B.EPI2, dt, q0, None, tol=1e-10, m_min=10, m_max=64)[0]
    with B.Mesh(B.EULER2D, nx, p, ny=ny, precision=B.FP32_BULK, ev_ce=1.0, ev_cmax=0.1,
                **DOM) as gm:
        q = dev(q0)
        gm.step(B.EPI2, dt, q, None, False, B.make_opts(1e-7, 10, 64))
        assert rel(host(q), ref) < 1e-6, rel(host(q), ref)


def test_zero_cap_equals_inviscid():
    # c_max = 0: nu = min(nu_max, nu_E) = 0 everywhere (exactly), and steps
    # equal the inviscid ones to rounding: the viscous kernel subtracts nu g =
    # 0 exactly, but the compiler contracts products into the surrounding
    # sums differently in the two kernels, so the last bits may differ
    nx, ny, p = 6, 5, 3
    with B.Mesh(B.EULER2D, nx, p, ny=ny, ev_ce=1.0, ev_cmax=0.0, **DOM) as ge, \
            B.Mesh(B.EULER2D, nx, p, ny=ny, **DOM) as g0:
        x, y = g0.nodes()
        q0 = dev(inputs.shear_layer(x, y, seed=6).reshape(-1))
        nu = torch.empty(ge.K * ge.Np, dtype=torch.float64, device=DEV)
        ge.entropy_viscosity(q0, q0 * 1.001, 0.01, nu)
        assert torch.count_nonzero(nu).item() == 0
        dt = 5.0 * g0.dx_min / g0.max_speed(q0)
        opts = B.make_opts(1e-10, 10, 64)
        qa, qb = q0.clone(), q0.clone()
        pa, pb = torch.empty_like(q0), torch.empty_like(q0)
        for k in range(2):
            ge.step(B.EPI3, dt, qa, pa, k > 0, opts)
            g0.step(B.EPI3, dt, qb, pb, k > 0, opts)
        assert rel(host(qa), host(qb)) < 1e-12, rel(host(qa), host(qb))


def test_rejections():
    with B.Mesh(B.EULER2D, 2, 2, ny=2, **DOM) as gm:
        z = dev(np.zeros(gm.K * gm.Np))
        with pytest.raises(B.ExpdgError):
            gm.set_viscosity(z)
    with pytest.raises(B.ExpdgError):
        B.Mesh(B.BURGERS1D, 4, 2, ev_ce=1.0)
    with pytest.raises(B.ExpdgError):
        B.Mesh(B.EULER2D, 2, 2, ny=2, ev_ce=-1.0, **DOM)
