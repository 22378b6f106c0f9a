"""Pins of the oracle's no-slip walls for 2D Euler (Section 5.3: periodic in
x, no-slip walls at y0 and y1; the exterior state at a wall is the mirror
M q = (rho, -rho u, -rho v, rho E)).

  * a fluid at rest is a steady state (R = 0): the wall flux is the pressure;
  * mass and energy are conserved exactly on any state (the mirror pair
    carries no mass or energy through a wall), x-momentum is not (wall drag);
  * on a state that is constant over the mesh the residual is the face term
    of the textbook Rusanov flux between q and M q at the wall nodes, and
    zero elsewhere;
  * reflecting the state about the channel's mid-line (y -> y0 + y1 - y,
    v -> -v) reflects the residual (the two walls are treated alike);
  * the linear operator is the complex-step derivative of the residual with
    lambda frozen (the mirror is linear);
  * the entropy-viscosity diffusion stays symmetric negative semi-definite in
    the mass inner product and conserves density and energy;
  * the entropy viscosity matches the definitions written out with numpy
    (jump 2|v S| at a wall, two-element averages at wall vertices);
  * steps with walls and entropy viscosity conserve mass and energy.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs
from tests import _textbook as T

GAMMA = 1.4
BOX = (0.0, 2.0, 0.0, 1.0)


def mesh(nx, ny, p, **kw):
    d = dict(x0=BOX[0], x1=BOX[1], y0=BOX[2], y1=BOX[3], bc=oracle.BC_WALL_Y)
    d.update(kw)
    return oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, **d)


def state(m, seed, amp=0.2):
    return inputs.random_euler_state(m.K * m.Np, seed, spread=amp).reshape(-1)


def smooth_state(m):
    x, y = m.nodes()
    rho = 1.0 + 0.2 * np.sin(math.pi * x) * np.cos(math.pi * y)
    u = 0.3 + 0.1 * np.cos(math.pi * y)
    v = 0.1 * np.sin(math.pi * x) * np.sin(math.pi * y)
    pr = 1.0 + 0.1 * np.cos(math.pi * x + math.pi * y)
    return np.concatenate([rho, rho * u, rho * v, pr / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


def test_rest_state_is_steady():
    m = mesh(4, 3, 3)
    npts = m.K * m.Np
    q = np.concatenate([np.full(npts, 1.3), np.zeros(npts), np.zeros(npts),
                        np.full(npts, 2.0 / (GAMMA - 1))])
    assert np.max(np.abs(m.rhs(q))) <= 1e-13


@pytest.mark.parametrize("p", [1, 3, 4])
def test_mass_and_energy_conserved(p):
    m = mesh(5, 4, p)
    npts = m.K * m.Np
    M = m.mass()
    R = m.rhs(state(m, p)).reshape(4, npts)
    scale = np.abs(M * R).sum()
    for c in (0, 3):
        assert abs(M @ R[c]) <= 1e-13 * scale, (c, M @ R[c])
    assert abs(M @ R[1]) > 1e-6 * scale  # x-momentum: the walls drag


def test_constant_state_wall_flux_is_textbook_rusanov():
    p = 3
    m = mesh(3, 2, p)
    npts, n1 = m.K * m.Np, p + 1
    q1 = np.array([1.2, 1.2 * 0.4, 1.2 * 0.25, 2.6])
    q = np.repeat(q1, npts)
    R = m.rhs(q).reshape(4, 2, 3, n1, n1)  # [c, ey, ex, j, i]
    _, w, _ = T.lgl_textbook(p)
    hy = (BOX[3] - BOX[2]) / 2
    mq = q1 * np.array([1.0, -1.0, -1.0, 1.0])
    for side, ey, j, sn in (("bottom", 0, 0, -1.0), ("top", 1, p, 1.0)):
        fstar = T.rusanov(q1, mq, 1, GAMMA) if sn > 0 else T.rusanov(mq, q1, 1, GAMMA)
        f = T.euler_flux(q1, 1, GAMMA)
        want = -(2.0 / hy) / w[j] * (sn * fstar - sn * f)
        got = R[:, ey, :, j, :]  # every node on that wall
        assert np.max(np.abs(got - want[:, None, None])) <= 1e-12 * np.max(np.abs(want)), side
    # nowhere else: the interior of the wall rows and the whole interior
    inner = R.copy()
    inner[:, 0, :, 0, :] = 0.0
    inner[:, 1, :, p, :] = 0.0
    assert np.max(np.abs(inner)) <= 1e-12


def reflect(m, f):
    """f(x, y0 + y1 - y) with the y-momentum reversed, in the library layout."""
    n1 = m.p + 1
    a = f.reshape(4, m.ny, m.nx, n1, n1)[:, ::-1, :, ::-1, :].copy()
    a[2] *= -1.0
    return a.reshape(-1)


@pytest.mark.parametrize("p", [2, 4])
def test_reflection_about_the_mid_line(p):
    m = mesh(4, 5, p)
    q = state(m, 10 + p)
    R = m.rhs(q)
    Rr = m.rhs(reflect(m, q))
    assert np.max(np.abs(Rr - reflect(m, R))) <= 1e-12 * np.max(np.abs(R))


@pytest.mark.parametrize("p", [2, 3])
def test_jvp_complex_step(p):
    m = mesh(3, 4, p)
    q = state(m, 20 + p)
    v = np.random.default_rng(p).standard_normal(m.n)
    w = m.jvp(q, v)
    assert np.max(np.abs(w - m.jvp_complex_step(q, v))) <= 1e-12 * np.max(np.abs(w))


@pytest.mark.parametrize("p", [1, 3])
def test_diffusion_with_walls_symmetric_negative(p):
    m0 = mesh(4, 3, p)
    g = np.random.default_rng(p)
    nu = g.uniform(0.01, 0.2, m0.K * m0.Np)
    m = mesh(4, 3, p, nu=nu)
    M = np.tile(m.mass(), 4)
    u, v = g.standard_normal(m.n), g.standard_normal(m.n)
    Du, Dv = m.ev_diffusion(u), m.ev_diffusion(v)
    a, b = u @ (M * Dv), v @ (M * Du)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert v @ (M * Dv) < 0 and u @ (M * Du) < 0
    npts = m.K * m.Np
    Mv = m.mass()
    for c in (0, 3):
        assert abs(Mv @ Dv[c * npts:(c + 1) * npts]) <= 1e-12 * np.abs(M * Dv).sum()


@pytest.mark.parametrize("ce,cmax", [(0.05, 1e9), (0.5, 0.1)])
def test_entropy_viscosity_with_walls_textbook(ce, cmax):
    nx, ny, p, dt = 5, 4, 3, 0.05
    m = mesh(nx, ny, p, ev_ce=ce, ev_cmax=cmax)
    x, y = m.nodes()
    g = np.random.default_rng(4)
    off = np.repeat(g.uniform(-1.0, 1.0, nx * ny), (p + 1) ** 2)

    def st(ph):
        rho = 1.0 + 0.2 * np.sin(math.pi * (x + ph)) * np.cos(2 * math.pi * y)
        u = 0.3 + 0.1 * np.cos(2 * math.pi * (y - ph))
        v = 0.1 * np.sin(math.pi * x) + 0.05  # nonzero at the walls: wall jumps 2 |v S|
        pr = 1.0 + 0.1 * np.cos(math.pi * x + 2 * math.pi * (y + ph)) + 0.3 * off
        return np.concatenate([rho, rho * u, rho * v, pr / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])

    q, qp = st(0.0), st(0.05)
    want = T.entropy_viscosity_2d(q, qp, dt, nx, ny, p, BOX, ce, cmax, walls=True)
    got = m.entropy_viscosity(q, qp, dt)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(want)
    periodic = T.entropy_viscosity_2d(q, qp, dt, nx, ny, p, BOX, ce, cmax, walls=False)
    assert np.max(np.abs(got - periodic)) > 1e-6 * np.max(want)  # the walls matter here


def test_steps_with_walls_and_viscosity_conserve_mass_energy():
    m = mesh(8, 6, 3, x0=-1.0, x1=1.0, y0=0.0, y1=1.0, ev_ce=1.0, ev_cmax=0.1)
    x, y = m.nodes()
    q0 = inputs.kelvin_helmholtz(x * 5.0, y * 5.0).reshape(-1)
    c, dx = m.max_speed(q0)
    dt = 5.0 * dx / c
    Mv = m.mass()
    npts = m.K * m.Np
    q, qp = q0, None
    for _ in range(3):
        q, qp = m.step(oracle.EPI2, dt, q, qp, tol=1e-10, m_min=10, m_max=64)
    for cidx in (0, 3):
        a = Mv @ q0[cidx * npts:(cidx + 1) * npts]
        b = Mv @ q[cidx * npts:(cidx + 1) * npts]
        assert abs(a - b) <= 1e-11 * abs(a), cidx
