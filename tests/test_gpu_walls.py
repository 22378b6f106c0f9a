"""No-slip walls for 2D Euler on the GPU (Section 5.3: periodic in x, walls at
y0 and y1), through the C ABI, against the oracle.

  * the residual and the linear operator with walls, with and without a
    nodal entropy viscosity, to 1e-12 of the largest output, on every
    compiled degree, one and several element rows and ragged last blocks;
  * the nodal entropy viscosity with walls (wall jumps 2 |v S|, two-element
    averages at the wall vertices) to 1e-12 of its largest value;
  * EPI2 and EPI3 steps of the Kelvin-Helmholtz problem with walls and the
    entropy viscosity, replaying the oracle's schedule, to 1e-12 relative,
    and mass and energy conserved by the GPU steps to 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2011_01316_amd import binding as B
from paper_2011_01316_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
DOM = dict(x0=-1.0, x1=1.0, y0=0.0, y1=1.0)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def maxrel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


SHAPES = [(1, 1, 1), (1, 1, 6), (4, 3, 2), (3, 5, 3), (6, 4, 4), (5, 3, 5), (3, 4, 6), (7, 2, 1),
          (5, 1, 3), (1, 4, 4)]


def kh_state(m):
    x, y = m.nodes()
    return inputs.kelvin_helmholtz(5.0 * x, 5.0 * y, sigma=0.2).reshape(-1)


@pytest.mark.parametrize("nx,ny,p", SHAPES)
@pytest.mark.parametrize("visc", [False, True])
def test_operators_with_walls(nx, ny, p, visc):
    print(f"walls operators: {nx}x{ny} p={p} viscosity {visc}", flush=True)
    om0 = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, bc=oracle.BC_WALL_Y, **DOM)
    g = np.random.default_rng(p + 10 * nx + ny)
    nu = g.uniform(0.0, 0.02, om0.K * om0.Np) if visc else None
    ev = dict(ev_ce=1.0, ev_cmax=0.1) if visc else {}
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, bc=oracle.BC_WALL_Y, nu=nu, **ev, **DOM)
    q = inputs.random_euler_state(om.K * om.Np, p + 3).reshape(-1)
    v = g.standard_normal(om.n)
    with B.Mesh(B.EULER2D, nx, p, ny=ny, bc=B.BC_WALL_Y, **ev, **DOM) as gm:
        if visc:
            gm.set_viscosity(dev(nu))
        qt, vt = dev(q), dev(v)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        ro, wo = om.rhs(q), om.jvp(q, v)
        assert maxrel(host(r), ro) < 1e-12, maxrel(host(r), ro)
        assert maxrel(host(w), wo) < 1e-12, maxrel(host(w), wo)
    # the walls matter: the periodic operator differs
    per = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, nu=nu, **ev, **DOM)
    assert maxrel(per.jvp(q, v), wo) > 1e-6


@pytest.mark.parametrize("nx,ny,p", SHAPES)
@pytest.mark.parametrize("ce", [1e-4, 1.0, 1e9])
def test_viscosity_with_walls(nx, ny, p, ce):
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, bc=oracle.BC_WALL_Y, ev_ce=ce, ev_cmax=0.1,
                     **DOM)
    x, y = om.nodes()
    q = inputs.shear_layer(0.5 * (x + 1.0), y, seed=nx + p).reshape(-1)
    qp = q * (1.0 + 1e-3 * np.random.default_rng(p).standard_normal(q.size))
    want = om.entropy_viscosity(q, qp, 0.02)
    with B.Mesh(B.EULER2D, nx, p, ny=ny, bc=B.BC_WALL_Y, ev_ce=ce, ev_cmax=0.1, **DOM) as gm:
        nu = torch.empty(gm.K * gm.Np, dtype=torch.float64, device=DEV)
        gm.entropy_viscosity(dev(q), dev(qp), 0.02, nu)
        assert np.max(want) > 0
        assert maxrel(host(nu), want) < 1e-12, maxrel(host(nu), want)


@pytest.mark.parametrize("scheme", [B.EPI2, B.EPI3])
def test_kh_steps_with_walls(scheme):
    print(f"walls KH steps: scheme {scheme}", flush=True)
    nx, ny, p = 8, 4, 4
    ev = dict(ev_ce=1.0, ev_cmax=0.1)
    om = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, bc=oracle.BC_WALL_Y, **ev, **DOM)
    q0 = kh_state(om)
    c, dx = om.max_speed(q0)
    dt = 4.0 * dx / c
    npts = om.K * om.Np
    M = om.mass()
    with B.Mesh(B.EULER2D, nx, p, ny=ny, bc=B.BC_WALL_Y, **ev, **DOM) as gm:
        q = dev(q0)
        qp = torch.empty_like(q)
        oq, oqp = q0, None
        for k in range(2):
            oq, oqp, st = om.step(scheme, dt, oq, oqp, tol=1e-10, m_min=10, m_max=64, stats=True)
            gm.step(scheme, dt, q, qp, k > 0, B.make_opts(1e-10, 10, 64, forced=st["log"]))
            assert rel(host(q), oq) < 1e-12, (k, rel(host(q), oq))
        qh = host(q)
        for c_ in (0, 3):
            a, b = M @ q0[c_ * npts:(c_ + 1) * npts], M @ qh[c_ * npts:(c_ + 1) * npts]
            assert abs(a - b) <= 1e-12 * abs(a), c_


def test_served_viscosity_and_walls_bitwise():
    """Served solves with entropy viscosity and walls (grouped launches of the
    viscous operator, mixed with inviscid and periodic solves) are bitwise
    equal to expdg_step on their own meshes (history passed for EPI2 too, so
    each step's viscosity sees q^{n-1})."""
    from tests.test_gpu_serve import burgers_case, euler_case, serve_all
    print("served viscosity and walls", flush=True)
    kh = []
    for (nx, ny, p, scheme, bc) in [(8, 4, 3, B.EPI2, B.BC_WALL_Y), (6, 6, 2, B.EPI3, B.BC_WALL_Y),
                                    (8, 4, 3, B.EPI3, B.BC_PERIODIC)]:
        r = B.make_request(B.EULER2D, nx, p, ny=ny, scheme=scheme, nsteps=3, cfl=4.0, tol=1e-10,
                           m_min=10, m_max=64, bc=bc, ev_ce=1.0, ev_cmax=0.1, **DOM)
        m = B.Mesh(B.EULER2D, nx, p, ny=ny, bc=bc, ev_ce=1.0, ev_cmax=0.1, **DOM)
        q0 = kh_state(m)
        kh.append((r, q0, m))
    plain = [burgers_case(40, 2, 0.3), euler_case(10, 3, 4.0, 6.0, 3.0)]
    cases = [(r, q0) for (r, q0, _) in kh] + plain
    with B.Server(hbm_budget=1 << 30, max_active=8) as srv:
        got = serve_all(srv, cases)
    for k, (r, q0, m) in enumerate(kh):
        with m:
            q = dev(q0)
            qp = torch.empty_like(q)
            dt = r.cfl * m.dx_min / m.max_speed(q)
            for s in range(r.nsteps):
                m.step(r.scheme, dt, q, qp, s > 0, B.make_opts(1e-10, 10, 64))
            np.testing.assert_array_equal(host(q), got[k][0])
