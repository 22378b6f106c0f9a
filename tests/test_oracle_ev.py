"""Pins of the oracle's entropy viscosity for 2D Euler (Section 3.2,
"Artificial viscosity"; c_E = 1 and c_max = 0.1 as in Section 5.3's runs).

The diffusion div(nu grad v) with central fluxes:
  * is symmetric and negative semi-definite in the LGL mass inner product,
    u^T M D(v) = v^T M D(u) and v^T M D(v) <= 0, for any positive nodal nu
    (summation by parts: D = -M^-1 G^T M nu G with G the discrete gradient);
  * annihilates constants and conserves each variable (periodic);
  * converges to nu Laplace(v) for constant nu and smooth v (order > 2.5 in
    the maximum norm at p = 4).
The viscosity:
  * vanishes for constant and for isentropic states (S = 0 when p = rho^gamma,
    the vortex among them);
  * with a large c_E it is the cap c_max h max(|u.e_d| + a) averaged to the
    vertices and interpolated bilinearly (equal caps give a constant nu);
  * only the time-derivative term depends on dt.
The linear operator with a frozen nu is the complex-step derivative of the
residual with the same nu; steps with entropy viscosity conserve mass.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs

GAMMA = 1.4


def mesh(nx, ny, p, **kw):
    d = dict(x0=0.0, x1=1.0, y0=0.0, y1=1.0)
    d.update(kw)
    return oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, **d)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_diffusion_symmetric_negative(p):
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
    # constants are annihilated; each variable's mass is conserved
    assert np.max(np.abs(m.ev_diffusion(np.ones(m.n)))) <= 1e-11
    Mv = m.mass()
    for c in range(4):
        assert abs(Mv @ Dv[c * m.K * m.Np:(c + 1) * m.K * m.Np]) <= 1e-12 * (np.abs(M * Dv).sum())


def test_diffusion_converges_to_laplacian():
    errs = []
    for n in (4, 8):
        m0 = mesh(n, n, 4)
        x, y = m0.nodes()
        nu0 = 0.05
        m = mesh(n, n, 4, nu=np.full(x.size, nu0))
        f = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
        v = np.concatenate([f, 2 * f, -f, 0.5 * f])
        lap = -8 * math.pi ** 2 * nu0 * v
        errs.append(np.max(np.abs(m.ev_diffusion(v) - lap)) / np.max(np.abs(lap)))
    # central (BR1) fluxes lose orders on a second derivative: at p = 4 the
    # maximum error falls by 6.6 from h to h/2 (order > 2.5)
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 5.5, errs


def test_viscosity_vanishes_for_constant_and_isentropic_states():
    m = mesh(6, 5, 3, x1=10.0, y1=10.0, ev_ce=1.0, ev_cmax=0.1)
    npts = m.K * m.Np
    const = np.concatenate([np.full(npts, c) for c in (1.2, 0.3, -0.2, 3.0)])
    # (rounding only: the derivative of a constant flux is ~1e-16 of it)
    assert np.max(np.abs(m.entropy_viscosity(const, const, 0.1))) <= 1e-14
    x, y = m.nodes()
    q = inputs.vortex(x, y, beta=5.0).reshape(-1)       # p = rho^gamma: S = 0
    qp = inputs.vortex(x, y, t=0.3, beta=5.0).reshape(-1)
    nu = m.entropy_viscosity(q, qp, 0.3)
    assert np.max(np.abs(nu)) <= 1e-12


def element_caps(m, q, cmax):
    """c_max h max over the element of (|u.e_d| + a), h = sqrt(hx^2+hy^2)/p."""
    npts = m.K * m.Np
    rho, mu, mv, E = q.reshape(4, npts)
    u, v = mu / rho, mv / rho
    pr = (GAMMA - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    a = np.sqrt(GAMMA * pr / rho)
    lam = np.maximum(np.abs(u) + a, np.abs(v) + a).reshape(m.K, m.Np).max(axis=1)
    hx, hy = (m.x1 - m.x0) / m.nx, (m.y1 - m.y0) / m.ny
    return cmax * math.sqrt(hx * hx + hy * hy) / m.p * lam


@pytest.mark.parametrize("p", [2, 4])
def test_cap_and_bilinear_smoothing(p):
    nx, ny = 5, 4
    m = mesh(nx, ny, p, ev_ce=1e9, ev_cmax=0.1)
    g = np.random.default_rng(7)
    npts = m.K * m.Np
    rho = 1.0 + 0.3 * g.uniform(0, 1, npts)
    u, v = 0.4 * g.uniform(-1, 1, npts), 0.4 * g.uniform(-1, 1, npts)
    pr = 1.0 + 0.3 * g.uniform(0, 1, npts)
    q = np.concatenate([rho, rho * u, rho * v, pr / 0.4 + 0.5 * rho * (u * u + v * v)])
    nu = m.entropy_viscosity(q, q, 0.05).reshape(ny, nx, p + 1, p + 1)
    cap = element_caps(m, q, 0.1).reshape(ny, nx)
    vert = 0.25 * (cap + np.roll(cap, 1, axis=1) + np.roll(cap, 1, axis=0) +
                   np.roll(np.roll(cap, 1, axis=0), 1, axis=1))
    xi, _, _ = oracle.lgl(p)
    r = 0.5 * (xi + 1.0)
    for ey in range(ny):
        for ex in range(nx):
            v00, v10 = vert[ey, ex], vert[ey, (ex + 1) % nx]
            v01, v11 = vert[(ey + 1) % ny, ex], vert[(ey + 1) % ny, (ex + 1) % nx]
            want = (np.outer(1 - r, 1 - r) * v00 + np.outer(1 - r, r) * v10 +
                    np.outer(r, 1 - r) * v01 + np.outer(r, r) * v11)  # [j, i]
            assert np.max(np.abs(nu[ey, ex] - want)) <= 1e-14 * np.max(cap)
    # the same state in every element: equal caps, a constant viscosity
    rep = np.tile(q.reshape(4, m.K, m.Np)[:, :1, :], (1, m.K, 1)).reshape(-1)
    nu2 = m.entropy_viscosity(rep, rep, 0.05)
    assert np.max(np.abs(nu2 - nu2[0])) <= 1e-15 * nu2[0] and nu2[0] > 0


def test_time_derivative_term():
    m = mesh(4, 4, 3, ev_ce=1.0, ev_cmax=1e9)
    x, y = m.nodes()
    q = inputs.shear_layer(x, y, seed=1).reshape(-1)
    qp = q * (1.0 + 1e-3 * np.random.default_rng(2).standard_normal(q.size))
    a, b = m.entropy_viscosity(q, q, 0.01), m.entropy_viscosity(q, q, 1.0)
    assert np.array_equal(a, b)  # no time-derivative term when q_prev = q
    c, d = m.entropy_viscosity(q, qp, 0.01), m.entropy_viscosity(q, qp, 1.0)
    assert np.max(c) > np.max(d)


def test_jvp_complex_step_with_viscosity():
    m0 = mesh(4, 3, 3)
    g = np.random.default_rng(3)
    nu = g.uniform(0.0, 0.05, m0.K * m0.Np)
    m = mesh(4, 3, 3, nu=nu)
    x, y = m.nodes()
    q = inputs.shear_layer(x, y, seed=0).reshape(-1)
    v = g.standard_normal(m.n)
    w = m.jvp(q, v)
    assert np.max(np.abs(w - m.jvp_complex_step(q, v))) <= 1e-12 * np.max(np.abs(w))
    # the viscous part is exactly the diffusion operator
    w0 = mesh(4, 3, 3).jvp(q, v)
    assert np.max(np.abs((w - w0) - m.ev_diffusion(v))) <= 1e-12 * np.max(np.abs(w))


def test_steps_with_viscosity_conserve_mass():
    m = mesh(8, 8, 3, ev_ce=1.0, ev_cmax=0.1)
    x, y = m.nodes()
    q0 = inputs.shear_layer(x, y, seed=0).reshape(-1)
    c, dx = m.max_speed(q0)
    dt = 5.0 * dx / c
    Mv = m.mass()
    npts = m.K * m.Np
    q, qp = q0, None
    for _ in range(3):
        q, qp = m.step(oracle.EPI2, dt, q, qp, tol=1e-10, m_min=10, m_max=64)
    for cidx in (0, 1, 2, 3):
        a = Mv @ q0[cidx * npts:(cidx + 1) * npts]
        b = Mv @ q[cidx * npts:(cidx + 1) * npts]
        assert abs(a - b) <= 1e-11 * max(1.0, abs(a))
    # the viscosity is active (the steps differ from the inviscid ones)
    m2 = mesh(8, 8, 3)
    q2, qp2 = q0, None
    for _ in range(3):
        q2, qp2 = m2.step(oracle.EPI2, dt, q2, qp2, tol=1e-10, m_min=10, m_max=64)
    assert np.linalg.norm(q - q2) > 1e-8 * np.linalg.norm(q)


# ---- nu_E against the paper's definitions written out with numpy -------------
from tests import _textbook as T  # noqa: E402

BOX = (0.0, 2.0, 0.0, 1.0)  # hx != hy: h = sqrt(hx^2 + hy^2)/p is neither hx/p nor hy/p


def node_xy(nx, ny, p, box):
    """Node coordinates in the library's layout from the textbook LGL nodes."""
    xi = T.lgl_textbook(p)[0]
    x0, x1, y0, y1 = box
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    ex = np.arange(nx)[None, :, None, None]
    ey = np.arange(ny)[:, None, None, None]
    X = x0 + hx * (ex + 0.5 * (xi[None, None, None, :] + 1.0)) + 0.0 * ey
    Y = y0 + hy * (ey + 0.5 * (xi[None, None, :, None] + 1.0)) + 0.0 * ex
    return np.broadcast_to(X, (ny, nx, p + 1, p + 1)).reshape(-1), \
        np.broadcast_to(Y, (ny, nx, p + 1, p + 1)).reshape(-1)


def conservative(rho, u, v, pr):
    return np.concatenate([rho, rho * u, rho * v, pr / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def test_nu_E_polynomial_entropy_closed_form():
    """rho = 1, constant velocity (u0, v0), p = exp(s) with s quadratic: S =
    s/(gamma-1) and u S are polynomials of degree 2 <= p, so the nodal
    divergence is exact and Res has a closed form.  The periodic seams make
    [[u S . n]] nonzero on the boundary elements (the jump branch of the max)
    and zero inside (the residual branch)."""
    nx, ny, p, dt = 6, 4, 3, 0.1
    u0, v0, gm1 = 0.3, -0.2, GAMMA - 1.0
    x, y = node_xy(nx, ny, p, BOX)
    s = 0.1 + 0.2 * x + 0.3 * y * y
    s_prev = s - dt * 0.01 * (1.0 + x)
    one = np.ones_like(x)
    q = conservative(one, u0 * one, v0 * one, np.exp(s))
    qp = conservative(one, u0 * one, v0 * one, np.exp(s_prev))
    res_exact = (0.01 * (1.0 + x) + 0.5 * (u0 * (0.2 + 0.2 - 0.01 * dt) + 2.0 * v0 * 0.6 * y)) / gm1
    nu_tb, parts = T.entropy_viscosity_2d(q, qp, dt, nx, ny, p, BOX, 1.0, 1e9, parts=True)
    assert np.max(np.abs(parts["res"].reshape(-1) - res_exact)) <= 1e-12 * np.max(np.abs(res_exact))
    # both branches of max(|Res|, |[[uS.n]]|/h) are taken
    jump_wins = parts["jmax"] / parts["h"] > parts["rmax"]
    assert jump_wins[0, 0] and not jump_wins[1, 2] and 0 < jump_wins.sum() < nx * ny
    m = mesh(nx, ny, p, x0=BOX[0], x1=BOX[1], y0=BOX[2], y1=BOX[3], ev_ce=1.0, ev_cmax=1e9)
    ox, oy = m.nodes()
    assert np.max(np.abs(ox - x)) <= 1e-14 and np.max(np.abs(oy - y)) <= 1e-14
    nu = m.entropy_viscosity(q, qp, dt)
    assert np.max(np.abs(nu - nu_tb)) <= 1e-12 * np.max(nu_tb), np.max(np.abs(nu - nu_tb))


@pytest.mark.parametrize("ce,cmax", [(0.05, 1e9), (0.5, 0.1)])
def test_nu_E_smooth_state_with_element_jumps(ce, cmax):
    """A smooth non-isentropic state with a per-element pressure offset
    (nonzero face jumps everywhere), the previous state shifted in phase:
    the oracle's viscosity against the definitions written out with numpy,
    with nu_E alone (c_max large) and with c_E = 0.5, c_max = 0.1 (the min
    takes both branches; so does the max inside nu_E)."""
    nx, ny, p, dt = 5, 4, 4, 0.05
    x, y = node_xy(nx, ny, p, BOX)
    g = np.random.default_rng(11)
    off = np.repeat(g.uniform(-1.0, 1.0, nx * ny), (p + 1) ** 2)

    def state(ph):
        rho = 1.0 + 0.2 * np.sin(math.pi * (x + ph)) * np.cos(2 * math.pi * y)
        u = 0.3 + 0.1 * np.cos(2 * math.pi * (y - ph))
        v = 0.1 * np.sin(math.pi * x)
        pr = 1.0 + 0.1 * np.cos(math.pi * x + 2 * math.pi * (y + ph)) + 0.3 * off
        return conservative(rho, u, v, pr)

    q, qp = state(0.0), state(0.05)
    nu_tb, parts = T.entropy_viscosity_2d(q, qp, dt, nx, ny, p, BOX, ce, cmax, parts=True)
    m = mesh(nx, ny, p, x0=BOX[0], x1=BOX[1], y0=BOX[2], y1=BOX[3], ev_ce=ce, ev_cmax=cmax)
    nu = m.entropy_viscosity(q, qp, dt)
    assert np.max(np.abs(nu - nu_tb)) <= 1e-12 * np.max(nu_tb), np.max(np.abs(nu - nu_tb))
    nu_E = ce * parts["h"] ** 2 * np.maximum(parts["rmax"], parts["jmax"] / parts["h"])
    jump_wins = parts["jmax"] / parts["h"] > parts["rmax"]
    assert 0 < jump_wins.sum() < nx * ny, jump_wins.sum()
    if cmax > 1.0:
        assert np.all(nu_E < cmax * parts["h"] * parts["lam"])
    else:
        capped = cmax * parts["h"] * parts["lam"] < nu_E
        assert 0 < capped.sum() < nx * ny, capped.sum()
