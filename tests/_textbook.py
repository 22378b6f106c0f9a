"""Textbook formulas used by the oracle pin tests (test-side only).

These are written from the governing equations (paper Section 3), not from
the oracle: the physical Euler flux, the Rusanov flux between two constant
states, and the Burgers characteristic solution.  Nothing here is imported by
the product path.
"""
import numpy as np


def euler_flux(q, dirn, gamma=1.4):
    """Physical Euler flux F . e_dir for conservative q of shape (4, ...)."""
    rho, mx, my, E = q
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    un = u if dirn == 0 else v
    return np.stack([rho * un, mx * un + (p if dirn == 0 else 0.0 * p),
                     my * un + (p if dirn == 1 else 0.0 * p), (E + p) * un])


def euler_speed(q, dirn, gamma=1.4):
    rho, mx, my, E = q
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    return np.abs(u if dirn == 0 else v) + np.sqrt(gamma * p / rho)


def flux_jacobian_cs(q, dirn, gamma=1.4, h=1e-30):
    """dF_dir/dq at a single state q (4,), by complex step on euler_flux."""
    A = np.zeros((4, 4))
    for k in range(4):
        qc = q.astype(np.complex128)
        qc[k] += 1j * h
        A[:, k] = euler_flux(qc, dirn, gamma).imag / h
    return A


def rusanov(qL, qR, dirn, gamma=1.4):
    """Rusanov flux F* . e_dir between a left state qL and a right state qR."""
    lam = max(euler_speed(qL, dirn, gamma), euler_speed(qR, dirn, gamma))
    return 0.5 * (euler_flux(qL, dirn, gamma) + euler_flux(qR, dirn, gamma)) - 0.5 * lam * (qR - qL)


def burgers_characteristic(x, t, u0, du0, iters=60):
    """Smooth solution of u_t + (u^2/2)_x = 0: u = u0(xi), x = xi + u0(xi) t."""
    xi = x - u0(x) * t
    for _ in range(iters):
        f = xi + u0(xi) * t - x
        xi = xi - f / (1.0 + du0(xi) * t)
    return u0(xi)


def lgl_textbook(p):
    """LGL nodes (the endpoints and the roots of P_p'), weights
    2 / (p (p+1) P_p(x)^2) and differentiation matrix D = V' V^-1 from the
    Legendre Vandermonde matrix, all through numpy's Legendre module."""
    from numpy.polynomial import legendre as leg
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(leg.legroots(leg.legder(c)).real) if p > 1 else np.zeros(0)
    xi = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1.0) * leg.legval(xi, c) ** 2)
    V = leg.legvander(xi, p)
    Vx = np.stack([leg.legval(xi, leg.legder(np.eye(p + 1)[k])) for k in range(p + 1)], axis=1)
    return xi, w, Vx @ np.linalg.inv(V)


def entropy_viscosity_2d(q, q_prev, dt, nx, ny, p, box, ce, cmax, gamma=1.4, parts=False,
                         walls=False):
    """Entropy viscosity of Section 3.2 ("Artificial viscosity" and its
    footnotes) on a periodic nx x ny mesh of box = (x0, x1, y0, y1), written
    out from the definitions with numpy:
      S = rho/(gamma-1) log(p/rho^gamma), entropy flux u S;
      Res = (S(q) - S(q_prev))/dt + (div(u S)(q) + div(u S)(q_prev))/2 at the
      nodes, the divergence from each element's own LGL interpolant;
      h = 2r/k with r the circumradius of the element (an hx x hy rectangle:
      r = sqrt(hx^2 + hy^2)/2) and k = p;
      nu_E = c_E h^2 max(max|Res|, max|[[u S . n]]|/h) per element, the jump
      over the nodes of its four faces;
      nu_max = c_max h max(|f'(q)|) = c_max h max over its nodes of |u.e_d| + a;
      Smooth: vertex averages of min(nu_max, nu_E), then the bilinear
      interpolant on each element.
    With walls (no-slip at y0 and y1, periodic in x): the face beyond a wall
    carries the mirror state (v reversed), so its jump is 2 |v S|, and a wall
    vertex averages the two elements it belongs to.
    Returns the nodal viscosity in the library's layout (and, with parts, the
    per-element maxima rmax, jmax, the wave speed and h)."""
    x0, x1, y0, y1 = box
    n1 = p + 1
    _, _, D = lgl_textbook(p)
    xi = lgl_textbook(p)[0]
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    h = 2.0 * (0.5 * np.sqrt(hx * hx + hy * hy)) / p

    def fields(qq):
        rho, mu, mv, E = np.asarray(qq, dtype=np.float64).reshape(4, ny, nx, n1, n1)
        u, v = mu / rho, mv / rho
        pr = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
        S = rho / (gamma - 1.0) * np.log(pr / rho ** gamma)
        a = np.sqrt(gamma * pr / rho)
        return S, u * S, v * S, np.maximum(np.abs(u) + a, np.abs(v) + a)

    def div(F, G):
        # [ey, ex, j, i]: i runs along x, j along y
        return ((2.0 / hx) * np.einsum("il,abjl->abji", D, F) +
                (2.0 / hy) * np.einsum("jl,abli->abji", D, G))

    S1, F1, G1, lam = fields(q)
    S0, F0, G0, _ = fields(q_prev)
    res = (S1 - S0) / dt + 0.5 * (div(F1, G1) + div(F0, G0))
    rmax = np.abs(res).max(axis=(2, 3))
    # x faces: the right face of element ex against the left face of ex+1
    jx = np.abs(F1[:, :, :, p] - np.roll(F1, -1, axis=1)[:, :, :, 0]).max(axis=2)
    jy = np.abs(G1[:, :, p, :] - np.roll(G1, -1, axis=0)[:, :, 0, :]).max(axis=2)
    jy_below = np.roll(jy, 1, axis=0)
    if walls:
        jy[-1] = np.abs(2.0 * G1[-1, :, p, :]).max(axis=1)     # top wall
        jy_below[0] = np.abs(2.0 * G1[0, :, 0, :]).max(axis=1)  # bottom wall
    jmax = np.maximum(np.maximum(jx, np.roll(jx, 1, axis=1)), np.maximum(jy, jy_below))
    nu_E = ce * h * h * np.maximum(rmax, jmax / h)
    nu_max = cmax * h * lam.max(axis=(2, 3))
    nue = np.minimum(nu_max, nu_E)
    # vertex (vy, vx): lower-left corner of element (vy, vx)
    row = 0.5 * (nue + np.roll(nue, 1, axis=1))  # the two elements left/right of a vertex
    if walls:
        vert = np.empty((ny + 1, nx))
        vert[1:ny] = 0.5 * (row[1:] + row[:-1])
        vert[0], vert[ny] = row[0], row[ny - 1]
        up = vert[1:]
    else:
        vert = 0.5 * (row + np.roll(row, 1, axis=0))
        up = np.roll(vert, -1, axis=0)
    r = 0.5 * (xi + 1.0)
    v00 = vert[:ny, :, None, None]
    v10 = np.roll(vert[:ny], -1, axis=1)[:, :, None, None]
    v01 = up[:, :, None, None]
    v11 = np.roll(up, -1, axis=1)[:, :, None, None]
    R, T = r[None, None, None, :], r[None, None, :, None]  # [j, i]: x weight r_i, y weight r_j
    nu = ((1 - R) * (1 - T) * v00 + R * (1 - T) * v10 + (1 - R) * T * v01 + R * T * v11)
    nu = nu.reshape(-1)
    if parts:
        return nu, dict(rmax=rmax, jmax=jmax, lam=lam.max(axis=(2, 3)), h=h, res=res)
    return nu
