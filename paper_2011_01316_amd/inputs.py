"""Seeded synthetic inputs for the exponential-DG workloads.

This module holds only the workloads: initial states sampled at given node
coordinates, random fields and request mixes.  It holds none of the method's
arithmetic (no DG operator, no quadrature, no Krylov or stepping), so both
the GPU path and the CPU oracle may be fed from it.  Coordinates always come
from the caller.

Conservative Euler variables are returned stacked as an array of shape
(4, npts): (rho, rho u, rho v, rho E).

Workloads (paper, Section 5):
  * Burgers: u0 = 0.5 + sin(x + theta) on [0, 2 pi] (smooth, pre-shock until
    t = 1 for theta = 0).
  * Viscous Burgers on [0, 1] with u = 0 at both ends (Section 5.1): the
    time-independent manufactured solution u = sin(x^2) x (x - 1) with its
    source term, and the smooth initial state sin^3(2 pi x) (1 - x)^{3/2}.
  * Isentropic vortex translating in a uniform mean flow (Section 5.2; in 3D
    extruded along z with w = 0; after
    Zhou & Wei): velocity perturbation (lambda / 2 pi) e^{alpha (1 - r^2)/2}
    (-y~, x~), temperature T = T_inf - (lambda/2 pi)^2 e^{alpha (1-r^2)} /
    (2 alpha c_p), c_p = gamma / (gamma - 1), density from the isentropic
    relation rho = T^{1/(gamma-1)}, p = rho T.  On a periodic box the centre is
    taken at the nearest periodic image.
  * Shear layer (Kelvin-Helmholtz, Section 5.3) rescaled to the periodic unit
    square with two layers at y = 1/4 and 3/4 and a seeded multi-mode
    transverse-velocity perturbation.
"""
from __future__ import annotations

import math

import numpy as np


def burgers_ic(x: np.ndarray, theta: float = 0.0) -> np.ndarray:
    """u0(x) = 0.5 + sin(x + theta)."""
    return 0.5 + np.sin(np.asarray(x, dtype=np.float64) + theta)


def burgers_mms(x: np.ndarray, kappa: float):
    """Manufactured steady solution u = sin(x^2) x (x - 1) of u_t + (u^2/2)_x =
    kappa u_xx + s, and its source s = u u_x - kappa u_xx.  Returns (u, s)."""
    x = np.asarray(x, dtype=np.float64)
    sn, cs = np.sin(x * x), np.cos(x * x)
    u = sn * x * (x - 1.0)
    ux = (2.0 * x - 1.0) * sn + 2.0 * x * x * (x - 1.0) * cs
    uxx = (2.0 + 4.0 * x ** 3 - 4.0 * x ** 4) * sn + (10.0 * x * x - 6.0 * x) * cs
    return u, u * ux - kappa * uxx


def burgers_smooth(x: np.ndarray) -> np.ndarray:
    """Smooth viscous Burgers initial state sin^3(2 pi x) (1 - x)^{3/2} on [0, 1]."""
    x = np.asarray(x, dtype=np.float64)
    return np.sin(2.0 * math.pi * x) ** 3 * np.clip(1.0 - x, 0.0, None) ** 1.5


def primitive_to_conservative(rho, u, v, p, gamma=1.4) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E + 0.0 * rho])


def _wrap(d: np.ndarray, period: float) -> np.ndarray:
    """Nearest periodic image of a displacement."""
    return d - period * np.round(d / period)


def vortex(x, y, t: float = 0.0, beta: float = 5.0, alpha: float = 2.0, xc: float = 5.0,
           yc: float = 5.0, uinf: float = 0.2, vinf: float = 0.0, gamma: float = 1.4,
           Lx: float = 10.0, Ly: float = 10.0) -> np.ndarray:
    """Translating isentropic vortex of strength beta at time t (conservative)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xt = _wrap(x - xc - uinf * t, Lx)
    yt = _wrap(y - yc - vinf * t, Ly)
    r2 = xt * xt + yt * yt
    amp = beta / (2.0 * math.pi)
    g = np.exp(alpha * (1.0 - r2) / 2.0)
    u = uinf - amp * yt * g
    v = vinf + amp * xt * g
    cp = gamma / (gamma - 1.0)
    T = 1.0 - amp * amp * np.exp(alpha * (1.0 - r2)) / (2.0 * alpha * cp)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return primitive_to_conservative(rho, u, v, p, gamma)


def vortex3d(x, y, z, t: float = 0.0, beta: float = 5.0, xc: float = 5.0, yc: float = 0.0,
             Lx: float = 10.0, Ly: float = 10.0, **kw) -> np.ndarray:
    """The vortex extruded along z with zero vertical velocity (Section 5.2's
    three-dimensional case on (0, 10) x (-5, 5) x (0, 1)): conservative
    (rho, rho u, rho v, rho w, rho E), shape (5, npts)."""
    del z  # the state does not depend on z
    q = vortex(x, y, t=t, beta=beta, xc=xc, yc=yc, Lx=Lx, Ly=Ly, **kw)
    return np.stack([q[0], q[1], q[2], np.zeros_like(q[0]), q[3]])


def shear_layer(x, y, seed: int = 0, a: float = 0.01, sigma: float = 0.04, amp: float = 1e-2,
                s1: float = 0.25, s2: float = 0.75, modes: int = 4,
                gamma: float = 1.4) -> np.ndarray:
    """Kelvin-Helmholtz-type shear layer on the periodic unit square.

    rho = 1 + (tanh((y-s1)/a) - tanh((y-s2)/a))/2 (density 2:1),
    u = 0.1 + tanh((y-s1)/a) - tanh((y-s2)/a) - 1, p = 1/gamma, and
    v = amp sum_k a_k sin(2 pi k x + theta_k) (e^{-(y-s1)^2/sigma^2} +
    e^{-(y-s2)^2/sigma^2}) with seeded a_k (normalised to sum 1), theta_k.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rng = np.random.default_rng(seed)
    ak = rng.uniform(0.0, 1.0, modes)
    ak /= ak.sum()
    th = rng.uniform(0.0, 2.0 * math.pi, modes)
    t = np.tanh((y - s1) / a) - np.tanh((y - s2) / a)
    rho = 1.0 + 0.5 * t
    u = 0.1 + t - 1.0
    env = np.exp(-((y - s1) ** 2) / sigma ** 2) + np.exp(-((y - s2) ** 2) / sigma ** 2)
    v = np.zeros_like(x)
    for k in range(modes):
        v += ak[k] * np.sin(2.0 * math.pi * (k + 1) * x + th[k])
    v *= amp * env
    p = np.full_like(x, 1.0 / gamma)
    return primitive_to_conservative(rho, u, v, p, gamma)


def kelvin_helmholtz(x, y, a: float = 0.05, amp: float = 0.01, sigma: float = 0.2,
                     s1: float = 2.0, s2: float = 3.0, gamma: float = 1.4) -> np.ndarray:
    """The Kelvin-Helmholtz initial state of Section 5.3 on (-5, 5) x (0, 5).

    rho = 1 + (tanh((y-s1)/a) - tanh((y-s2)/a))/2, u = 0.1 + tanh((y-s1)/a) -
    tanh((y-s2)/a) - 1, v = amp sin(2 pi x)(e^{-(y-s1)^2/sigma^2} +
    e^{-(y-s2)^2/sigma^2}), p = 1/gamma.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    t = np.tanh((y - s1) / a) - np.tanh((y - s2) / a)
    rho = 1.0 + 0.5 * t
    u = 0.1 + t - 1.0
    env = np.exp(-((y - s1) ** 2) / sigma ** 2) + np.exp(-((y - s2) ** 2) / sigma ** 2)
    v = amp * np.sin(2.0 * math.pi * x) * env
    p = np.full_like(x, 1.0 / gamma)
    return primitive_to_conservative(rho, u, v, p, gamma)


def random_euler_state(npts: int, seed: int, gamma: float = 1.4, spread: float = 0.2) -> np.ndarray:
    """Pointwise random admissible Euler state (positive density and pressure)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + spread * rng.uniform(-1.0, 1.0, npts)
    u = 0.3 + spread * rng.uniform(-1.0, 1.0, npts)
    v = -0.2 + spread * rng.uniform(-1.0, 1.0, npts)
    p = 1.0 + spread * rng.uniform(-1.0, 1.0, npts)
    return primitive_to_conservative(rho, u, v, p, gamma)


def random_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Uniform random direction vector in [-scale, scale]^n."""
    rng = np.random.default_rng(seed)
    return scale * rng.uniform(-1.0, 1.0, n)


def bloch_mode_plus_noise(K: int, p: int, wavenumber: int, eps: float, seed: int) -> np.ndarray:
    """A 1D nodal vector (K elements of p+1 nodes) of the form
    Re(exp(2 pi i k e / K) phi_i) with random complex phi, scaled to unit
    length, plus eps times a random unit vector.  On a periodic mesh with a
    constant reference state every element applies the same operator, so the
    first part spans an invariant subspace of dimension 2(p+1) of the linear
    operator (a nearly invariant one for small eps)."""
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal(p + 1) + 1j * rng.standard_normal(p + 1)
    e = np.arange(K)
    base = (np.exp(2j * math.pi * wavenumber * e / K)[:, None] * phi[None, :]).real.reshape(-1)
    base /= np.linalg.norm(base)
    r = rng.standard_normal(K * (p + 1))
    return base + eps * r / np.linalg.norm(r)


def served_mix(n_requests: int = 2000, rate: float = 200.0, seed: int = 0,
               burgers_k=(32, 4096), burgers_p=(1, 4), euler_n=(16, 128), euler_p=(2, 4),
               steps: int = 20):
    """Poisson arrivals of mixed Burgers / Euler solves (served workload).

    Returns a list of dicts with arrival time (s), equation, mesh size,
    degree and the seeded initial-condition parameters.  Sizes are drawn
    log-uniformly, degrees uniformly, 50/50 equation mix.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(n_requests):
        if rng.uniform() < 0.5:
            K = int(round(math.exp(rng.uniform(math.log(burgers_k[0]), math.log(burgers_k[1])))))
            p = int(rng.integers(burgers_p[0], burgers_p[1] + 1))
            reqs.append(dict(arrival=float(t[i]), equation="burgers1d", nx=K, ny=1, p=p,
                             theta=float(rng.uniform(0.0, 2.0 * math.pi)), dt=1e-2,
                             steps=steps))
        else:
            n = int(round(math.exp(rng.uniform(math.log(euler_n[0]), math.log(euler_n[1])))))
            p = int(rng.integers(euler_p[0], euler_p[1] + 1))
            reqs.append(dict(arrival=float(t[i]), equation="euler2d", nx=n, ny=n, p=p,
                             xc=float(rng.uniform(0.0, 10.0)), yc=float(rng.uniform(0.0, 10.0)),
                             beta=float(rng.uniform(1.0, 5.0)), cr=5.0, steps=steps))
    return reqs
