"""Pins of the oracle's steep-gradient viscous Burgers case (Section 5.1, "A
solution with steep gradient": u(x, 0) = sin(2 pi x), zero Dirichlet ends,
kappa = 0.002, and the entropy flux with the face-dependent penalty
sigma = kappa/100 + h max|u^+-|).

  * on piecewise-constant periodic states the residual's energy is
    u^T M R(u) = -sum_faces (2 kappa/(100 h_e) + max|u^+-|) [[u]]^2
    - kappa q^T M q (the entropy-conservative part drops out; the penalty is
    read per face; the diffusion gives its energy identity);
  * Table expo-burgers-tconv-shock (tests/golden): EPI2 and EXPRB32 with LF
    and EF on k = 4, N_e = 160 against the reference of the paper's
    discretization (k = 10, N_e = 160, LF; tests/golden/
    burgers_shock_reference_k10_ne160.txt, written by the oracle's own
    script there), every entry within 0.5 % except EXPRB32 at dt = 0.02,
    where the error approaches the spatial difference between the two
    discretizations (within 10 %);
  * Table expo-burgers-sconv-shock (LF and EF, N_e = 40 and 80): the errors
    within a factor 0.85 .. 2.3 of the printed ones (the band of the smooth
    tables, reading 20).
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KAPPA = 0.002


def _read(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def _lagrange(xi, pts):
    L = np.ones((pts.size, xi.size))
    for j in range(xi.size):
        for l in range(xi.size):
            if l != j:
                L[:, j] *= (pts - xi[l]) / (xi[j] - xi[l])
    return L


@pytest.mark.parametrize("kappa", [0.0, 0.03])
def test_local_penalty_piecewise_constant(kappa):
    ne, p = 11, 3
    m = oracle.Mesh(oracle.BURGERS1D, ne, p, x0=0.0, x1=1.0, kappa=kappa,
                    flux=oracle.FLUX_EF_LOCAL)
    g = np.random.default_rng(5)
    ue = g.uniform(-1.5, 2.0, ne)
    u = np.repeat(ue, p + 1)
    M = m.mass()
    ur = np.roll(ue, -1)
    jumps = ue - ur  # u_L - u_R at the right face of each element
    pen = 2.0 * kappa / (100.0 / ne) + np.maximum(np.abs(ue), np.abs(ur))
    expect = -np.sum(pen * jumps ** 2)
    if kappa > 0:
        q = m.gradient(u)
        expect -= kappa * (q @ (M * q))
    got = u @ (M * m.rhs(u))
    assert abs(got - expect) <= 1e-12 * (1.0 + abs(expect) + np.sum(np.abs(ue) ** 3)), (got, expect)
    # with the constant-sigma entropy flux the same state gives another energy
    mc = oracle.Mesh(oracle.BURGERS1D, ne, p, x0=0.0, x1=1.0, kappa=kappa, flux=oracle.FLUX_EF,
                     sigma=3e-4)
    assert abs(u @ (M * mc.rhs(u)) - got) > 1e-3 * abs(got)


def _reference():
    ref = np.array([float(r[0]) for r in _read("burgers_shock_reference_k10_ne160.txt")])
    assert ref.size == 160 * 11
    return ref


def _error(q, k, ne, ref):
    """L2 distance at t = 1 to the reference, 16-point Gauss on its mesh."""
    pr, nr = 10, 160
    xir, _, _ = oracle.lgl(pr)
    xi, _, _ = oracle.lgl(k)
    gx, gw = np.polynomial.legendre.leggauss(16)
    Lr = _lagrange(xir, gx)
    hf, r = 1.0 / nr, nr // ne
    err2 = 0.0
    for ef in range(nr):
        ec = ef // r
        xc = 2.0 * ((ef + 0.5 * (gx + 1.0)) * hf - ec / ne) * ne - 1.0
        d = _lagrange(xi, xc) @ q[ec * (k + 1):(ec + 1) * (k + 1)] - Lr @ ref[ef * (pr + 1):(ef + 1) * (pr + 1)]
        err2 += np.sum(gw * 0.5 * hf * d * d)
    return math.sqrt(err2)


def _run(k, ne, flux, scheme, dt, tol):
    m = oracle.Mesh(oracle.BURGERS1D, ne, k, x0=0.0, x1=1.0, kappa=KAPPA, bc=oracle.BC_DIRICHLET,
                    flux=flux)
    q = np.sin(2.0 * math.pi * m.nodes()[0])
    for _ in range(int(round(1.0 / dt))):
        q, _ = m.step(scheme, dt, q, tol=tol, m_min=5, m_max=64)
    return q


def test_shock_temporal_table():
    """Table expo-burgers-tconv-shock."""
    ref = _reference()
    for r in _read("burgers_viscous_shock_tconv.txt"):
        flux = oracle.FLUX_LF if r[0] == "LF" else oracle.FLUX_EF_LOCAL
        dt = float(r[1])
        for col, scheme in ((3, oracle.EPI2), (4, oracle.EXPRB32)):
            e = _error(_run(4, 160, flux, scheme, dt, 1e-10), 4, 160, ref)
            tolr = 0.10 if (scheme == oracle.EXPRB32 and dt == 0.02) else 0.005
            assert abs(e / float(r[col]) - 1.0) <= tolr, (r[0], dt, scheme, e, r[col])


def test_shock_spatial_table():
    """Table expo-burgers-sconv-shock, N_e = 40 and 80 (EXPRB32 at dt = 2e-3,
    whose temporal error is far below these)."""
    ref = _reference()
    for r in _read("burgers_viscous_shock_sconv.txt"):
        k, ne = int(r[0]), int(r[1])
        if ne == 160:
            continue
        for col, flux in ((2, oracle.FLUX_LF), (3, oracle.FLUX_EF_LOCAL)):
            e = _error(_run(k, ne, flux, oracle.EXPRB32, 2e-3, 1e-12), k, ne, ref)
            assert 0.85 <= e / float(r[col]) <= 2.3, (k, ne, col, e, r[col])
