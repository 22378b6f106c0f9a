"""Pins for the oracle's matrix exponential and phi-function evaluation (CPU).

  * expm against scipy.linalg.expm (a different algorithm, called not
    copied), diagonal and Jordan-block closed forms, exp(X) exp(-X) = I;
  * phi_k scalar closed forms (phi_1 = (e^z - 1)/z, ...) and the recurrence
    phi_{k+1}(z) = (phi_k(z) - 1/k!)/z (Section 2.3) on diagonal matrices;
  * A = 0: sum tau^k b_k / k!;
  * Krylov with the augmented matrix against the dense augmented exponential
    (whose top block identity is independent of the eta scaling);
  * full Krylov space (m = n + p) is exact (happy breakdown);
  * adaptive error within the requested tolerance, and a replayed schedule
    reproduces the adaptive run bit for bit.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2011_01316_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------- expm
@pytest.mark.parametrize("n,scale", [(1, 0.3), (5, 0.1), (12, 1.0), (30, 10.0), (65, 3.0), (20, 1e3)])
def test_expm_vs_scipy(n, scale):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) * scale / math.sqrt(n)
    # keep the matrix well-conditioned for exp: shift the spectrum left
    A -= np.eye(n) * max(0.0, np.max(np.linalg.eigvals(A).real))
    E = oracle.expm(A)
    Es = scipy.linalg.expm(A)
    assert np.linalg.norm(E - Es) <= 1e-12 * max(1.0, np.linalg.norm(Es)) * max(1.0, scale / 10)


def test_expm_closed_forms():
    d = np.array([-50.0, -3.0, 0.0, 0.5, 2.0])
    # s = 7 squarings for ||A|| = 50 amplify rounding by about 2^7
    np.testing.assert_allclose(oracle.expm(np.diag(d)), np.diag(np.exp(d)), rtol=1e-12, atol=1e-300)
    lam, n = -1.7, 6
    J = lam * np.eye(n) + np.diag(np.ones(n - 1), 1)
    E = oracle.expm(J)
    expect = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            expect[i, j] = math.exp(lam) / math.factorial(j - i)
    np.testing.assert_allclose(E, expect, rtol=1e-13, atol=1e-16)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((9, 9))
    np.testing.assert_allclose(oracle.expm(X) @ oracle.expm(-X), np.eye(9), atol=1e-12)


# --------------------------------------------------------------------- phi closed forms
def phi_scalar(k, z):
    """phi_k(z) from its definition, by series for small |z|."""
    if abs(z) < 1e-2:
        return sum(z ** j / math.factorial(j + k) for j in range(25))
    # closed form: (e^z - sum_{j<k} z^j/j!) / z^k
    return (math.exp(z) - sum(z ** j / math.factorial(j) for j in range(k))) / z ** k


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_phi_dense_diagonal(p):
    lam = np.array([-40.0, -5.0, -0.3, -1e-4, 0.0, 1e-3, 0.7, 2.0])
    n = lam.size
    tau = 0.37
    rng = np.random.default_rng(p)
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    out = oracle.phi_dense(np.diag(lam), tau, bs)
    expect = np.zeros(n)
    for k in range(p + 1):
        expect += tau ** k * np.array([phi_scalar(k, tau * l) for l in lam]) * bs[k]
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-14)


def test_phi_recurrence():
    # phi_{k+1}(tA) b = (phi_k(tA) b - b/k!) (tA)^{-1}, checked via A phi_{k+1} = ...
    rng = np.random.default_rng(5)
    n = 7
    A = rng.standard_normal((n, n)) - 3 * np.eye(n)
    b = rng.standard_normal(n)
    tau = 0.6
    z = np.zeros(n)
    for k in range(1, 4):
        bk = [z] * k + [b]        # tau^k phi_k(tau A) b
        bk1 = [z] * (k + 1) + [b]  # tau^{k+1} phi_{k+1}(tau A) b
        pk = oracle.phi_dense(A, tau, bk) / tau ** k
        pk1 = oracle.phi_dense(A, tau, bk1) / tau ** (k + 1)
        lhs = tau * A @ pk1
        rhs = pk - b / math.factorial(k)
        assert rel(lhs, rhs) < 1e-12


def test_phi_zero_matrix():
    n = 5
    rng = np.random.default_rng(9)
    bs = [rng.standard_normal(n) for _ in range(4)]
    tau = 1.7
    out = oracle.phi_dense(np.zeros((n, n)), tau, bs)
    expect = sum(tau ** k / math.factorial(k) * bs[k] for k in range(4))
    np.testing.assert_allclose(out, expect, rtol=1e-13)
    out = oracle.phi_krylov_dense(np.zeros((n, n)), tau, bs, tol=1e-12, m_min=1)
    np.testing.assert_allclose(out, expect, rtol=1e-12)


# --------------------------------------------------------------------- Krylov vs dense
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_krylov_dense_random(p):
    n = 60
    rng = np.random.default_rng(100 + p)
    A = rng.standard_normal((n, n)) / math.sqrt(n) * 4 - 2 * np.eye(n)
    bs = [rng.standard_normal(n) * 10.0 ** (k - 1) for k in range(p + 1)]
    tau = 0.9
    ref = oracle.phi_dense(A, tau, bs)
    out, st = oracle.phi_krylov_dense(A, tau, bs, tol=1e-12, m_min=5, m_max=40, stats=True)
    nu = sum(tau ** k * np.linalg.norm(bs[k]) / math.factorial(k) for k in range(p + 1))
    assert np.linalg.norm(out - ref) <= 10 * 1e-12 * nu
    assert st["substeps"] >= 1


def test_krylov_full_space_exact():
    n, p = 9, 2
    rng = np.random.default_rng(1)
    A = rng.standard_normal((n, n))
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    tau = 0.8
    ref = oracle.phi_dense(A, tau, bs)
    out, st = oracle.phi_krylov_dense(A, tau, bs, tol=1e-30, m_min=n + p, m_max=n + p + 2,
                                      stats=True)
    assert st["breakdown"] == 1 and st["substeps"] == 1
    assert rel(out, ref) < 1e-12


def test_krylov_substepping():
    # a stiff operator with a small m_max forces rejections and substeps
    n = 80
    lam = -np.linspace(0.0, 400.0, n)
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(lam) @ Q.T
    bs = [rng.standard_normal(n), rng.standard_normal(n)]
    tau = 0.5
    ref = oracle.phi_dense(A, tau, bs)
    out, st = oracle.phi_krylov_dense(A, tau, bs, tol=1e-10, m_min=5, m_max=15, stats=True)
    nu = np.linalg.norm(bs[0]) + tau * np.linalg.norm(bs[1])
    assert st["substeps"] > 1 and st["rejects"] >= 1
    assert np.linalg.norm(out - ref) <= 20 * 1e-10 * nu
    # the schedule sums to tau and its last substep is flagged
    assert abs(sum(d for (_, d, _) in st["log"]) - tau) < 1e-12
    assert [l for (_, _, l) in st["log"]] == [0] * (st["substeps"] - 1) + [1]
    # replay reproduces the adaptive result bit for bit
    out2 = oracle.phi_krylov_dense(A, tau, bs, tol=1e-10, m_min=5, m_max=15, forced=st["log"])
    assert np.array_equal(out, out2)


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10, 1e-12])
def test_krylov_tolerance_sweep(tol):
    n = 50
    rng = np.random.default_rng(4)
    # stable (dissipative) spectrum, like the DG operators: radius ~6 about -4
    A = rng.standard_normal((n, n)) * 6 / math.sqrt(n) - 4 * np.eye(n)
    A -= np.eye(n) * max(0.0, np.max(np.linalg.eigvals(A).real))
    bs = [rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)]
    tau = 0.7
    ref = oracle.phi_dense(A, tau, bs)
    out = oracle.phi_krylov_dense(A, tau, bs, tol=tol, m_min=3, m_max=30)
    nu = sum(tau ** k * np.linalg.norm(bs[k]) / math.factorial(k) for k in range(3))
    assert np.linalg.norm(out - ref) <= 10 * tol * nu


# --------------------------------------------------------------------- DG operator
def test_krylov_dg_burgers_vs_dense():
    m = oracle.Mesh(oracle.BURGERS1D, 64, 2, x0=0.0, x1=2 * math.pi)
    x, _ = m.nodes()
    u = inputs.burgers_ic(x)
    L = m.assemble_jvp(u)
    # the assembled matrix reproduces the operator
    v = inputs.random_vector(m.n, 1)
    assert rel(L @ v, m.jvp(u, v)) < 1e-14
    R = m.rhs(u)
    for dt in [1e-2, 0.1]:
        ref = oracle.phi_dense(L, dt, [None, R])
        out = m.phi_krylov(u, dt, [None, R], tol=1e-12, m_min=5, m_max=30)
        assert np.linalg.norm(out - ref) <= 10 * 1e-12 * dt * np.linalg.norm(R)


def test_krylov_dg_euler_tiny_vs_dense():
    m = oracle.Mesh(oracle.EULER2D, 2, 2, ny=2, x0=0.0, x1=1.0, y0=0.0, y1=1.0)
    q = inputs.random_euler_state(m.K * m.Np, 3).reshape(-1)
    L = m.assemble_jvp(q)
    R = m.rhs(q)
    b2 = inputs.random_vector(m.n, 4)
    tau = 0.05
    ref = oracle.phi_dense(L, tau, [q, R, b2])
    out = m.phi_krylov(q, tau, [q, R, b2], tol=1e-12, m_min=5, m_max=60)
    nu = np.linalg.norm(q) + tau * np.linalg.norm(R) + tau ** 2 / 2 * np.linalg.norm(b2)
    assert np.linalg.norm(out - ref) <= 10 * 1e-12 * nu
