"""The oracle's Arnoldi (classical Gram-Schmidt applied twice, explicit norms)
near a breakdown (Section 2.3, Arnoldi projection of the augmented matrix).

On a periodic Burgers mesh with a constant reference state, a Bloch mode of
one wavenumber spans an invariant subspace of dimension 2(p+1) of the linear
operator; adding eps times a random vector makes it nearly invariant, so the
subdiagonal entry h_{6,5} (p = 2) falls to about 17 eps while the vector it
normalizes has a norm of about 10.  Across eps = 1e-4 .. 1e-10 (beta / ||x||
from about 1e-4 to 1e-10):
  * the basis stays orthonormal to 1e-14 and the Arnoldi relation
    A V_m = V_{m+1} H holds to 1e-13 ||A||;
  * h_{6,5} scales with eps (the near breakdown is where it is expected);
  * exp(tau A) b from 30 Arnoldi vectors (through the near-invariant
    dimension) equals the dense exponential to 1e-12, and the adaptive run
    is within 10 tol of it;
  * eps = 0 is an exact breakdown at dimension 6 (h_{6,5} at rounding level).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2011_01316_amd import inputs

K, P, WAVE = 16, 2, 3


def operator():
    om = oracle.Mesh(oracle.BURGERS1D, K, P, x0=0.0, x1=2 * math.pi)
    ut = np.full(om.n, 0.7)
    return om, ut, om.assemble_jvp(ut)


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8, 1e-10, 0.0])
def test_arnoldi_near_breakdown(eps):
    om, ut, A = operator()
    b = inputs.bloch_mode_plus_noise(K, P, WAVE, eps, seed=5)
    V, H = oracle.arnoldi_dense(A, b, 12)
    d = 2 * (P + 1)
    nA = np.linalg.norm(A, 2)
    if eps > 0:
        m = V.shape[0] - 1
        assert m == 12
        assert np.max(np.abs(V @ V.T - np.eye(m + 1))) <= 1e-14
        res = A @ V[:m].T - V.T @ H
        assert np.max(np.abs(res)) <= 1e-13 * nA
        assert 5.0 * eps <= H[d, d - 1] <= 50.0 * eps, H[d, d - 1]
        assert np.min(np.diag(H, -1)[: d - 1]) > 0.1
    else:
        # exact breakdown: the space is exhausted at dimension 6
        assert V.shape[0] == d + 1 or H[d, d - 1] <= 1e-12 * np.linalg.norm(H)
    # exp(tau A) b from 30 vectors, through the near-invariant dimension
    tau = 0.5
    dense = oracle.phi_dense(A, tau, [b])
    forced = [(30, tau, 1)] if eps > 0 else [(d, tau, 1)]
    got = om.phi_krylov(ut, tau, [b], tol=1e-10, forced=forced)
    assert np.linalg.norm(got - dense) <= 1e-12 * np.linalg.norm(dense)
    ad, st = om.phi_krylov(ut, tau, [b], tol=1e-10, m_min=2, m_max=30, stats=True)
    assert np.linalg.norm(ad - dense) <= 10 * 1e-10 * np.linalg.norm(b)
