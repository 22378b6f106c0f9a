"""The allocation-free linear operator (expdg_jvp_noalloc) against expdg_jvp.

expdg_jvp_noalloc runs the same kernels as expdg_jvp on a mesh created from
the same description, with the frozen fields of the Euler operators in the
library's static device scratch instead of the mesh workspace, so the two
results must be bitwise equal.  Two calls in a row, the second on a smaller
mesh (the scratch then holds the first call's larger contents), and one
operator per equation and precision.  The FP64 results are also held to the
oracle's linear operator at the parity bound of the operators (1e-12 of the
largest entry).
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


def case_state(eq, nx, ny, nz, p, precision, seed):
    """Mesh (created the usual way), reference state and direction on it."""
    L = dict(x0=0.0, x1=10.0, y0=0.0, y1=10.0, z0=0.0, z1=2.0)
    if eq == B.BURGERS1D:
        L = dict(x0=0.0, x1=2 * math.pi)
    gm = B.Mesh(eq, nx, p, ny=ny, nz=nz, precision=precision, **L)
    npts = gm.K * gm.Np
    if eq == B.BURGERS1D:
        x, _ = gm.nodes()
        q0 = inputs.burgers_ic(x)
    else:
        q0 = inputs.random_euler_state(npts, seed, gamma=1.4)
        if eq == B.EULER3D:
            # five variables: insert a w momentum plane beside rho u, rho v
            q4 = q0.reshape(4, npts)
            rho = q4[0]
            mw = 0.1 * rho * np.sin(np.arange(npts) * 0.37)
            E = q4[3] + 0.5 * mw * mw / rho
            q0 = np.concatenate([q4[0], q4[1], q4[2], mw, E])
    v0 = inputs.random_vector(gm.n, seed + 1)
    dt = gm.dtype
    q = torch.tensor(q0.reshape(-1), dtype=dt, device=DEV)
    v = torch.tensor(v0, dtype=dt, device=DEV)
    return gm, q, v, L


def oracle_jvp(eq, nx, ny, nz, p, L, q, v):
    om = oracle.Mesh(eq, nx, p, ny=ny, nz=nz, **L)
    return om.jvp(q.double().cpu().numpy(), v.double().cpu().numpy())


CASES = [
    # (equation, (nx, ny, nz, p) first call, second call smaller, precision)
    (B.EULER2D, (24, 20, 1, 4), (6, 5, 1, 3), B.FP64),
    (B.EULER2D, (17, 9, 1, 3), (3, 2, 1, 2), B.FP32_BULK),
    (B.EULER3D, (6, 5, 4, 3), (3, 2, 2, 2), B.FP64),
    (B.BURGERS1D, (300, 1, 1, 4), (7, 1, 1, 2), B.FP64),
]


@pytest.mark.parametrize("eq,big,small,precision", CASES)
def test_noalloc_jvp_matches_mesh_jvp(eq, big, small, precision):
    print(f"noalloc jvp: equation {eq}, {big} then {small}, precision {precision}", flush=True)
    for call, (nx, ny, nz, p) in enumerate((big, small)):
        gm, q, v, L = case_state(eq, nx, ny, nz, p, precision, seed=10 + call)
        with gm:
            w_mesh = torch.full_like(v, float("nan"))
            w_free = torch.full_like(v, float("nan"))
            gm.jvp(q, v, w_mesh)
            B.expdg_jvp_noalloc(gm.desc, q, v, w_free)
            torch.cuda.synchronize()
            a = w_mesh.cpu().numpy()
            b = w_free.cpu().numpy()
        assert np.all(np.isfinite(b)), (call, nx, ny, nz, p)
        assert np.array_equal(a, b), (call, float(np.max(np.abs(a - b))))
        if precision == B.FP64:
            ref = oracle_jvp(eq, nx, ny, nz, p, L, q, v)
            err = np.max(np.abs(b - ref)) / np.max(np.abs(ref))
            assert err < 1e-12, (call, err)


def test_noalloc_jvp_rejects_oversize_and_viscosity():
    # 400 x 400 quadrilaterals of degree 4 in FP64: 13.6M frozen-field values
    # (109 MB) do not fit the 64 MiB scratch
    d = B.MeshDesc(B.EULER2D, 400, 400, 4, B.FP64, 0, 0.0, 1.0, 0.0, 1.0, 1.4, 64, 0.0,
                   B.FLUX_LF, 0.0, 0.0, B.BC_PERIODIC, 0, 1, 0.0, 1.0, 0.0, 0.0)
    x = torch.zeros(16, dtype=torch.float64, device=DEV)
    w = torch.full((16,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(B.ExpdgError) as ei:
        B.expdg_jvp_noalloc(d, x, x, w)
    assert ei.value.code == B.EINVAL and "scratch" in str(ei.value)
    d.nx = d.ny = 8
    d.ev_ce, d.ev_cmax = 1.0, 0.1
    with pytest.raises(B.ExpdgError) as ei:
        B.expdg_jvp_noalloc(d, x, x, w)
    assert ei.value.code == B.EINVAL
    torch.cuda.synchronize()
    assert torch.all(w == 7.0)  # outputs untouched on EINVAL
