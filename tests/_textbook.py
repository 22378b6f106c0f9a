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
