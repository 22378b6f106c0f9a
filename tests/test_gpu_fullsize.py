"""GPU checks at the full sizes of the large workloads, in FP64 and FP32 bulk.

Workloads:
  * the 256 x 256, p = 3 isentropic vortex on [0, 10]^2 (4,194,304 DOF);
  * the 512 x 512, p = 4 shear layer on the periodic unit square (26,214,400
    DOF).

Checks:
  * Operators, every entry, against the oracle: in FP32 bulk on the same
    float-rounded inputs, so input rounding cancels and only the arithmetic
    remains.  Each output is a sum of at most 2 (p + 1) + 4 derivative, face
    and lift terms.  Each term is at most S = (2/h)(max_i sum_l |D_il| + 1/w_0)
    max |F| and carries a few roundings.  Hence |err| <= c u S, with u the
    unit roundoff of the arithmetic (2^-53 or 2^-24) and c = 4 (p + 11).  F is
    the physical flux (residual) or A(q) v (linear operator), taken from the
    data.  At these resolutions the outputs are far smaller than their terms
    (the 256^2 vortex residual peaks near 0.55 against S near 1.5e3), so the
    bound is absolute in S, not relative to the output.
  * One EPI2 step in both precisions (FP64 tol 1e-10, FP32 bulk tol 1e-7):
    - the increment w = dt phi_1(dt L) R inherits the operators' rounding,
      every entry within about dt c u S of exact, and the Krylov combination
      adds at most a few such contributions.  Hence
      max |w32 - w64| <= 4 c u32 dt S.  The near-steady shear layer shows why
      the bound is absolute: its residual is far smaller than its terms, so
      relative to the increment the FP32 difference is 2e-3 (measured).
      Relative to the state it is far smaller; that state-level L2 difference
      is checked below 1e-6.
    - both conserve the discrete mass sum_e (h_x h_y / 4) sum_ij w_i w_j rho.
      The linear operator's density flux is the momentum perturbation, and its
      frozen Rusanov term has the same speed on both sides of a face, so the
      mass of every operator output cancels exactly in exact arithmetic.
      Rounding leaves each entry of the increment within about dt u S of
      exact, and the Krylov combination of up to m vectors multiplies that.
      Hence |mass of the increment| <= 2048 u dt S area, with u the unit
      roundoff of the bulk type (2^-53 or 2^-24).
  * Entropy viscosity on the shear layer at 512 x 512, p = 4 (the size its
    measurement runs at): the nodal viscosity and both operators with it
    against the oracle within bounds of the same kind (stated with the
    tests), and one FP32-bulk EPI3 step with the viscosity against the FP64
    one.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2011_01316_amd import binding as B
from paper_2011_01316_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
U32 = 2.0 ** -24
GAMMA = 1.4

CASES = {
    "vortex256_p3": dict(n=256, p=3, L=10.0),
    "shear512_p4": dict(n=512, p=4, L=1.0),
}


def setup(case, precision=B.FP64):
    c = CASES[case]
    n, p, L = c["n"], c["p"], c["L"]
    om = oracle.Mesh(oracle.EULER2D, n, p, ny=n, x0=0.0, x1=L, y0=0.0, y1=L)
    gm = B.Mesh(B.EULER2D, n, p, ny=n, x0=0.0, x1=L, y0=0.0, y1=L, precision=precision)
    x, y = om.nodes()
    if case.startswith("vortex"):
        q = inputs.vortex(x, y).reshape(-1)
    else:
        q = inputs.shear_layer(x, y, seed=0).reshape(-1)
    return om, gm, q


def flux_np(q, npts):
    """Euler fluxes F_x, F_y (4 x npts each) of a conservative state."""
    r, m, nn, E = q.reshape(4, npts)
    u, v = m / r, nn / r
    pr = (GAMMA - 1.0) * (E - 0.5 * (m * u + nn * v))
    fx = np.stack([m, m * u + pr, nn * u, (E + pr) * u])
    fy = np.stack([nn, m * v, nn * v + pr, (E + pr) * v])
    return fx, fy


def stencil_bound(om, p, fmax):
    xi, w, D = oracle.lgl(p)
    h = min(om.x1 - om.x0, om.y1 - om.y0) / om.nx
    return (2.0 / h) * (np.abs(D).sum(axis=1).max() + 1.0 / w[0]) * fmax


def operator_bounds(om, p, qd, vd, u):
    """c u S for the residual at qd and the linear operator at qd applied to vd."""
    npts = qd.size // 4
    c = 4 * (p + 11)
    fx, fy = flux_np(qd, npts)
    bound_r = c * u * stencil_bound(om, p, max(np.abs(fx).max(), np.abs(fy).max()))
    # A(q) v by a central difference of the flux (only its size is needed)
    eps = 1e-4 * max(1.0, np.abs(qd).max()) / max(np.abs(vd).max(), 1e-300)
    fxp, fyp = flux_np(qd + eps * vd, npts)
    fxm, fym = flux_np(qd - eps * vd, npts)
    amax = max(np.abs(fxp - fxm).max(), np.abs(fyp - fym).max()) / (2 * eps)
    # the Rusanov term adds lambda |v| <= (|u| + a) |v|, at most a few times |A v|
    bound_w = c * u * stencil_bound(om, p, 4.0 * max(amax, np.abs(vd).max()))
    return bound_r, bound_w


@pytest.mark.parametrize("case", list(CASES))
def test_operators_full_size_fp64(case):
    om, gm, q = setup(case)
    p = CASES[case]["p"]
    with gm:
        g = np.random.default_rng(3)
        v = q * (1.0 + 0.1 * g.standard_normal(q.size))
        qt = torch.tensor(q, device=DEV)
        vt = torch.tensor(v, device=DEV)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        torch.cuda.synchronize()
        ro, wo = om.rhs(q), om.jvp(q, v)
        bound_r, bound_w = operator_bounds(om, p, q, v, 2.0 ** -53)
        er = np.max(np.abs(r.cpu().numpy() - ro))
        ew = np.max(np.abs(w.cpu().numpy() - wo))
        assert er <= bound_r, (er, bound_r)
        assert ew <= bound_w, (ew, bound_w)


@pytest.mark.parametrize("case", list(CASES))
def test_operators_full_size_fp32_bulk(case):
    om, gm, q = setup(case, B.FP32_BULK)
    p = CASES[case]["p"]
    with gm:
        g = np.random.default_rng(4)
        # a direction of the state's size and shape, as in the Krylov basis
        v = (q * (1.0 + 0.1 * g.standard_normal(q.size))).astype(np.float32)
        q32 = q.astype(np.float32)
        qt = torch.tensor(q32, device=DEV)
        vt = torch.tensor(v, device=DEV)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        torch.cuda.synchronize()
        qd, vd = q32.astype(np.float64), v.astype(np.float64)
        ro, wo = om.rhs(qd), om.jvp(qd, vd)
        bound_r, bound_w = operator_bounds(om, p, qd, vd, U32)
        er = np.max(np.abs(r.cpu().numpy().astype(np.float64) - ro))
        ew = np.max(np.abs(w.cpu().numpy().astype(np.float64) - wo))
        assert er <= bound_r, (er, bound_r)
        assert ew <= bound_w, (ew, bound_w)
        # FP32 storage, FP64 arithmetic: the stored residual is the FP64 value
        # rounded once to FP32 (the FP64 arithmetic's own c u64 S on top)
        r64 = r.cpu().numpy().astype(np.float64)
        tight = U32 * np.abs(ro) + operator_bounds(om, p, qd, vd, 2.0 ** -53)[0]
        assert np.all(np.abs(r64 - ro) <= tight), np.max(np.abs(r64 - ro) - tight)


def discrete_mass(om, q, p):
    _, w, _ = oracle.lgl(p)
    hx = (om.x1 - om.x0) / om.nx
    hy = (om.y1 - om.y0) / om.ny
    np1 = p + 1
    rho = q[: q.size // 4].reshape(-1, np1, np1)  # [e][j][i]
    wq = np.outer(w, w) * (hx * hy / 4.0)
    return float(np.sum(rho * wq)), float(np.sum(np.abs(rho) * wq))


@pytest.mark.parametrize("case", list(CASES))
def test_fp32_bulk_step_full_size(case):
    p = CASES[case]["p"]
    om, g64, q = setup(case)
    with g64:
        q0 = torch.tensor(q, device=DEV)
        dt = 5.0 * g64.dx_min / g64.max_speed(q0)
        q64 = q0.clone()
        g64.step(B.EPI2, dt, q64, None, False, B.make_opts(1e-10, 10, 64, 1))
        w64 = (q64 - q0).cpu().numpy()
    g32 = B.Mesh(B.EULER2D, om.nx, p, ny=om.ny, x0=om.x0, x1=om.x1, y0=om.y0, y1=om.y1,
                 precision=B.FP32_BULK)
    with g32:
        q32 = q0.clone()
        g32.step(B.EPI2, dt, q32, None, False, B.make_opts(1e-7, 10, 64, 1))
        w32 = (q32 - q0).cpu().numpy()
    fx, fy = flux_np(q, q.size // 4)
    S = stencil_bound(om, p, max(np.abs(fx).max(), np.abs(fy).max()))
    c = 4 * (p + 11)
    dmax = np.max(np.abs(w32 - w64))
    assert dmax <= 4 * c * U32 * dt * S, (dmax, 4 * c * U32 * dt * S)
    state_diff = np.linalg.norm(w32 - w64) / np.linalg.norm(q + w64)
    assert state_diff <= 1e-6, state_diff
    area = (om.x1 - om.x0) * (om.y1 - om.y0)
    m64, _ = discrete_mass(om, w64, p)
    m32, _ = discrete_mass(om, w32, p)
    assert abs(m64) <= 2048 * 2.0 ** -53 * dt * S * area, (m64, dt * S * area)
    assert abs(m32) <= 2048 * U32 * dt * S * area, (m32, dt * S * area)


# ---- entropy viscosity at the size of its measurement (512 x 512, p = 4) ----
# The viscosity: Res at a node sums the two entropy time terms and the 2(p+1)
# terms of the two element-local divergences, each at most
# T = 2 max|S| / dt + (2/h) max_i sum_l |D_il| max|uS| in size, so its error is
# at most c u T; a face jump |[[uS . n]]| is off by at most 2 u max|uS|; the
# element viscosity scales these by c_E h_e^2 (at most h_e^2 T c_E when the cap
# is not taken, at most the cap's own rounding otherwise) and the smoothing
# only averages.  Hence |nu_gpu - nu_oracle| <= c u c_E h_e^2 (T + max|uS|/h_e)
# + c u max(nu), c = 4 (p + 11).
# The operators with a viscosity nu: the viscous terms are a second stencil
# applied to nu g, g itself a stencil of v: each entry within
# c u (S + 2 S_v) with S_v = (2/h)^2 (max_i sum_l |D_il| + 1/w_0)^2 max(nu) max|v|.

def entropy_fields(q, npts):
    r, m, nn, E = q.reshape(4, npts)
    u, v = m / r, nn / r
    pr = (GAMMA - 1.0) * (E - 0.5 * (m * u + nn * v))
    S = r / (GAMMA - 1.0) * np.log(pr / r ** GAMMA)
    return S, np.abs(u * S).max() + np.abs(v * S).max()


def ev_setup(precision=B.FP64):
    n, p = 512, 4
    om = oracle.Mesh(oracle.EULER2D, n, p, ny=n, ev_ce=1.0, ev_cmax=0.1)
    gm = B.Mesh(B.EULER2D, n, p, ny=n, precision=precision, ev_ce=1.0, ev_cmax=0.1)
    x, y = om.nodes()
    q = inputs.shear_layer(x, y, seed=0).reshape(-1)
    qp = q * (1.0 + 1e-3 * np.random.default_rng(5).standard_normal(q.size))
    return om, gm, q, qp


def test_entropy_viscosity_full_size():
    om, gm, q, qp = ev_setup()
    p, dt = 4, 0.02
    with gm:
        nu = torch.empty(gm.K * gm.Np, dtype=torch.float64, device=DEV)
        gm.entropy_viscosity(torch.tensor(q, device=DEV), torch.tensor(qp, device=DEV), dt, nu)
        got = nu.cpu().numpy()
    want = om.entropy_viscosity(q, qp, dt)
    npts = q.size // 4
    S, us = entropy_fields(q, npts)
    Sp, usp = entropy_fields(qp, npts)
    xi, w, D = oracle.lgl(p)
    h = 1.0 / 512
    he = math.sqrt(2.0) * h / p
    T = 2 * max(np.abs(S).max(), np.abs(Sp).max()) / dt + \
        (2.0 / h) * np.abs(D).sum(axis=1).max() * max(us, usp)
    c = 4 * (p + 11)
    u = 2.0 ** -53
    bound = c * u * (he * he * (T + max(us, usp) / he) + want.max())
    err = np.max(np.abs(got - want))
    assert want.max() > 0 and err <= bound, (err, bound, want.max())


def test_operators_with_viscosity_full_size():
    om0, gm, q, qp = ev_setup()
    p = 4
    nu = om0.entropy_viscosity(q, qp, 0.02)
    om = oracle.Mesh(oracle.EULER2D, 512, p, ny=512, ev_ce=1.0, ev_cmax=0.1, nu=nu)
    with gm:
        gm.set_viscosity(torch.tensor(nu, device=DEV))
        v = q * (1.0 + 0.1 * np.random.default_rng(6).standard_normal(q.size))
        qt = torch.tensor(q, device=DEV)
        vt = torch.tensor(v, device=DEV)
        r = torch.empty_like(qt)
        w = torch.empty_like(qt)
        gm.rhs(qt, r)
        gm.jvp(qt, vt, w)
        torch.cuda.synchronize()
        rg, wg = r.cpu().numpy(), w.cpu().numpy()
    ro, wo = om.rhs(q), om.jvp(q, v)
    bound_r, bound_w = operator_bounds(om, p, q, v, 2.0 ** -53)
    xi, wq, D = oracle.lgl(p)
    k2 = ((2.0 * 512) * (np.abs(D).sum(axis=1).max() + 1.0 / wq[0])) ** 2
    c = 4 * (p + 11)
    sv_r = 2 * c * 2.0 ** -53 * k2 * nu.max() * np.abs(q).max()
    sv_w = 2 * c * 2.0 ** -53 * k2 * nu.max() * np.abs(v).max()
    er, ew = np.max(np.abs(rg - ro)), np.max(np.abs(wg - wo))
    assert er <= bound_r + sv_r, (er, bound_r, sv_r)
    assert ew <= bound_w + sv_w, (ew, bound_w, sv_w)
    # the viscosity is active at this size
    assert np.max(np.abs(wo - om0.jvp(q, v))) > 1e3 * (bound_w + sv_w)


def test_fp32_bulk_step_with_viscosity_full_size():
    # one EPI3 step (first step: EPI2 form) as the bench times it, FP32 bulk at
    # tol 1e-7 against FP64 at tol 1e-10, both recomputing the viscosity from
    # the state: state-level l2 difference <= 1e-6, discrete mass of both
    # increments as in the inviscid check (the diffusion conserves mass)
    p = 4
    om, g64, q, _ = ev_setup()
    with g64:
        q0 = torch.tensor(q, device=DEV)
        dt = 5.0 * g64.dx_min / g64.max_speed(q0)
        q64 = q0.clone()
        qp = torch.empty_like(q0)
        g64.step(B.EPI3, dt, q64, qp, False, B.make_opts(1e-10, 10, 64, 1))
        w64 = (q64 - q0).cpu().numpy()
    g32 = B.Mesh(B.EULER2D, 512, p, ny=512, precision=B.FP32_BULK, ev_ce=1.0, ev_cmax=0.1)
    with g32:
        q32 = q0.clone()
        g32.step(B.EPI3, dt, q32, qp, False, B.make_opts(1e-7, 10, 64, 1))
        w32 = (q32 - q0).cpu().numpy()
    state_diff = np.linalg.norm(w32 - w64) / np.linalg.norm(q + w64)
    assert state_diff <= 1e-6, state_diff
    fx, fy = flux_np(q, q.size // 4)
    S = stencil_bound(om, p, max(np.abs(fx).max(), np.abs(fy).max()))
    m64, _ = discrete_mass(om, w64, p)
    m32, _ = discrete_mass(om, w32, p)
    assert abs(m64) <= 2048 * 2.0 ** -53 * dt * S, (m64, dt * S)
    assert abs(m32) <= 2048 * U32 * dt * S, (m32, dt * S)
