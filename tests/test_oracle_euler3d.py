"""Pins of the oracle's three-dimensional Euler operators (the system of
Section 3.2 written for three velocity components; the extruded vortex of
Section 5.2, periodic in every direction).

  * extrusion: for a state that does not depend on z and has w = 0, the 3D
    residual and linear operator equal the (separately pinned) 2D ones node by
    node, and their w components vanish;
  * axis permutation: relabelling x -> y -> z -> x (state, velocity
    components and mesh) permutes the residual and the linear operator, so the
    y and z code paths are pinned to the x one;
  * free stream, discrete conservation, the complex-step derivative of the
    frozen-dissipation residual equals L, and L(q) q = R(q) (the Euler flux is
    homogeneous of degree one and both use the same lambda);
  * the translating vortex is followed to its exact position with the
    expected temporal order of EPI2 (2) on a resolved mesh.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs

DOM = dict(x0=0.0, x1=10.0, y0=-5.0, y1=5.0, z0=0.0, z1=1.0)


def mesh3(nx, ny, nz, p, **kw):
    d = dict(DOM)
    d.update(kw)
    return oracle.Mesh(oracle.EULER3D, nx, p, ny=ny, nz=nz, **d)


def random_state(npts, seed, nvar=5):
    g = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * g.uniform(-1, 1, npts)
    vel = [0.3 * g.uniform(-1, 1, npts) for _ in range(nvar - 2)]
    p = 1.0 + 0.2 * g.uniform(-1, 1, npts)
    E = p / 0.4 + 0.5 * rho * sum(v * v for v in vel)
    return np.concatenate([rho] + [rho * v for v in vel] + [E])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_extrusion_equals_2d(p):
    nx, ny = 4, 3
    m2 = oracle.Mesh(oracle.EULER2D, nx, p, ny=ny, x0=0.0, x1=10.0, y0=-5.0, y1=5.0)
    m3 = mesh3(nx, ny, 2, p)
    n1 = p + 1
    q2 = random_state(m2.K * m2.Np, p, nvar=4).reshape(4, m2.K, n1, n1)
    v2 = np.random.default_rng(p + 9).standard_normal((4, m2.K, n1, n1))
    # extrude: element e3 = ez nx ny + e2, node (k, j, i)
    def ext(a2, w):
        out = np.zeros((5, 2 * m2.K, n1, n1, n1))
        for ez in range(2):
            for c3, c2 in ((0, 0), (1, 1), (2, 2), (4, 3)):
                out[c3, ez * m2.K:(ez + 1) * m2.K] = a2[c2][:, None, :, :]
            out[3, ez * m2.K:(ez + 1) * m2.K] = w
        return out.reshape(-1)
    q3 = ext(q2, 0.0)
    v3 = ext(v2, 0.0)
    r2 = m2.rhs(q2.reshape(-1)).reshape(4, m2.K, n1, n1)
    r3 = m3.rhs(q3).reshape(5, 2, m2.K, n1, n1, n1)
    w2 = m2.jvp(q2.reshape(-1), v2.reshape(-1)).reshape(4, m2.K, n1, n1)
    w3 = m3.jvp(q3, v3).reshape(5, 2, m2.K, n1, n1, n1)
    scale = max(np.abs(r2).max(), np.abs(w2).max())
    for c3, c2 in ((0, 0), (1, 1), (2, 2), (4, 3)):
        for ez in range(2):
            for k in range(n1):
                assert np.max(np.abs(r3[c3, ez, :, k] - r2[c2])) <= 1e-13 * scale
                assert np.max(np.abs(w3[c3, ez, :, k] - w2[c2])) <= 1e-13 * scale
    assert np.max(np.abs(r3[3])) <= 1e-13 * scale and np.max(np.abs(w3[3])) <= 1e-13 * scale


@pytest.mark.parametrize("p", [1, 2, 3])
def test_axis_permutation(p):
    n = 3
    L = dict(x0=0.0, x1=2.0, y0=0.0, y1=2.0, z0=0.0, z1=2.0)
    m = mesh3(n, n, n, p, **L)
    n1 = p + 1
    q = random_state(m.K * m.Np, 20 + p).reshape(5, n, n, n, n1, n1, n1)  # c, ez, ey, ex, k, j, i
    v = np.random.default_rng(p).standard_normal(q.shape)
    # relabel axes: new x = old z, new y = old x, new z = old y
    def rot(a):
        # element and node axes: (ez, ey, ex, k, j, i) -> new (ez', ey', ex') = (ey, ex, ez)
        b = np.transpose(a, (0, 2, 3, 1, 5, 6, 4))
        # velocity components: new (u', v', w') = (w, u, v)
        return b[[0, 3, 1, 2, 4]]
    R = m.rhs(q.reshape(-1)).reshape(q.shape)
    W = m.jvp(q.reshape(-1), v.reshape(-1)).reshape(q.shape)
    Rr = m.rhs(rot(q).reshape(-1)).reshape(q.shape)
    Wr = m.jvp(rot(q).reshape(-1), rot(v).reshape(-1)).reshape(q.shape)
    scale = max(np.abs(R).max(), np.abs(W).max())
    assert np.max(np.abs(Rr - rot(R))) <= 1e-13 * scale
    assert np.max(np.abs(Wr - rot(W))) <= 1e-13 * scale


@pytest.mark.parametrize("p", [1, 2, 4])
def test_free_stream_and_conservation(p):
    m = mesh3(3, 2, 2, p)
    npts = m.K * m.Np
    const = np.concatenate([np.full(npts, c) for c in (1.2, 0.3, -0.2, 0.1, 3.0)])
    assert np.max(np.abs(m.rhs(const))) <= 1e-12
    assert np.max(np.abs(m.jvp(const, const))) <= 1e-12
    q = random_state(npts, p)
    r = m.rhs(q).reshape(5, npts)
    M = m.mass()
    for c in range(5):
        assert abs(M @ r[c]) <= 1e-13 * (M @ np.abs(r[c])) + 1e-15


@pytest.mark.parametrize("p", [1, 3])
def test_jvp_complex_step_and_homogeneity(p):
    m = mesh3(2, 3, 2, p)
    npts = m.K * m.Np
    q = random_state(npts, 5 + p)
    v = np.random.default_rng(p).standard_normal(q.size)
    w = m.jvp(q, v)
    assert np.max(np.abs(w - m.jvp_complex_step(q, v))) <= 1e-12 * np.max(np.abs(w))
    r = m.rhs(q)
    assert np.max(np.abs(m.jvp(q, q) - r)) <= 1e-12 * np.max(np.abs(r))


def test_extruded_vortex_temporal_order():
    m = mesh3(10, 10, 1, 3)
    x, y, z = m.nodes()
    q0 = inputs.vortex3d(x, y, z, beta=2.0).reshape(-1)
    c, dx = m.max_speed(q0)
    T = 0.5
    ref = None
    errs = []
    # the reference is the oracle's own solution with a small step (the time
    # error, not the spatial one, is measured)
    for n in (2, 4, 8, 32):
        q = q0.copy()
        for _ in range(n):
            q, _ = m.step(oracle.EPI2, T / n, q, tol=1e-12, m_min=10, m_max=64)
        if n == 32:
            ref = q
        else:
            errs.append(q)
    e = [np.linalg.norm(a - ref) for a in errs]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.7 < o < 2.4 for o in orders), orders
    # and the vortex has moved to its exact position within the spatial error
    ex = inputs.vortex3d(x, y, z, t=T, beta=2.0).reshape(-1)
    assert np.linalg.norm(ref - ex) / np.linalg.norm(ex) < 2e-3
