"""FP64 CPU oracle for the exponential-DG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its binding) never imports, links or calls it, and the
two share no code.

This is a ctypes wrapper around ``liboracle.so`` built from the C++ sources in
this directory by :func:`build` (g++, -O3, OpenMP over elements).  Every
function works on numpy float64 arrays in the nodal layout
``idx = (c*K + e)*Np + n``.

Paper: Kang & Bui-Thanh, "A scalable exponential-DG approach for nonlinear
conservation laws: with application to Burger and Euler equations".  Each C++
source cites the section/equation it implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["refelem.cpp", "dg.cpp", "expm.cpp", "krylov.cpp", "steppers.cpp"]

BURGERS1D = 1
EULER2D = 2
EULER3D = 3
EPI2, EPI3, EXPRB32, EXPRB42 = 2, 3, 32, 42
FLUX_LF, FLUX_EF, FLUX_EF_LOCAL = 0, 1, 2
BC_PERIODIC, BC_DIRICHLET, BC_WALL_Y = 0, 1, 2


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (always recompiles)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-std=c++17", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Mesh(C.Structure):
    _fields_ = [("equation", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("p", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("kappa", C.c_double), ("flux", C.c_int),
                ("sigma", C.c_double), ("beta", C.c_double), ("bc", C.c_int),
                ("source", C.POINTER(C.c_double)), ("nz", C.c_int), ("z0", C.c_double),
                ("z1", C.c_double), ("ev_ce", C.c_double), ("ev_cmax", C.c_double),
                ("nu", C.POINTER(C.c_double))]


class Substep(C.Structure):
    _fields_ = [("m", C.c_int), ("last", C.c_int), ("dtau", C.c_double)]


class _KOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("m_min", C.c_int), ("m_max", C.c_int),
                ("check_every", C.c_int), ("forced", C.POINTER(Substep)), ("n_forced", C.c_int),
                ("iop", C.c_int), ("adapt", C.c_int), ("m_init", C.c_int)]


class _KStats(C.Structure):
    _fields_ = [("substeps", C.c_int), ("rejects", C.c_int), ("krylov_iters", C.c_int),
                ("jvps", C.c_int), ("breakdown", C.c_int), ("phi_calls", C.c_int),
                ("rhs_calls", C.c_int), ("err_est", C.c_double),
                ("log", C.POINTER(Substep)), ("log_cap", C.c_int), ("log_len", C.c_int),
                ("checks", C.c_int), ("m_next", C.c_int)]


_lib = None


def build_at(src_dir: str, out_path: str) -> str:
    """Compile the oracle sources found in src_dir into out_path."""
    srcs = [os.path.join(src_dir, s) for s in SOURCES]
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", out_path] + srcs
    subprocess.run(cmd, check=True)
    return out_path


def load(path: str):
    """Load an oracle library and declare its C signatures."""
    L = C.CDLL(path)
    _declare(L)
    return L


class use_library:
    """Context manager: route every wrapper call to another oracle build."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def _declare(L):
    dp = C.POINTER(C.c_double)
    mp = C.POINTER(_Mesh)
    L.orc_lgl.argtypes = [C.c_int, dp, dp, dp]
    L.orc_ndof.argtypes = [mp]
    L.orc_nodes.argtypes = [mp, dp, dp, dp]
    L.orc_mass.argtypes = [mp, dp]
    L.orc_rhs.argtypes = [mp, dp, dp]
    L.orc_jvp.argtypes = [mp, dp, dp, dp]
    L.orc_gradient.argtypes = [mp, dp, dp]
    L.orc_ev_diffusion.argtypes = [mp, dp, dp]
    L.orc_entropy_viscosity.argtypes = [mp, dp, dp, C.c_double, dp]
    L.orc_jvp_complex_step.argtypes = [mp, dp, dp, C.c_double, dp]
    L.orc_assemble_jvp.argtypes = [mp, dp, dp]
    L.orc_max_speed.argtypes = [mp, dp, dp, dp]
    L.orc_expm.argtypes = [C.c_int, dp, dp]
    L.orc_phi_dense.argtypes = [C.c_int, dp, C.c_double, C.c_int, C.POINTER(dp), dp]
    L.orc_phi_krylov_dense.argtypes = [C.c_int, dp, C.c_double, C.c_int, C.POINTER(dp), dp,
                                       C.POINTER(_KOpts), C.POINTER(_KStats)]
    L.orc_phi_krylov_dg.argtypes = [mp, dp, C.c_double, C.c_int, C.POINTER(dp), dp,
                                    C.POINTER(_KOpts), C.POINTER(_KStats)]
    L.orc_step.argtypes = [mp, C.c_int, C.c_double, dp, dp, C.c_int, C.POINTER(_KOpts),
                           C.POINTER(_KStats)]
    L.orc_rk4.argtypes = [mp, C.c_double, C.c_int, dp]
    L.orc_arnoldi_dense.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int, dp, dp]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


class Mesh:
    """Uniform mesh: Burgers 1D (nx intervals) or Euler 2D (nx x ny periodic quads).

    Burgers options (Section 3.1): viscosity kappa, nonlinear flux FLUX_LF or
    FLUX_EF (jump coefficient sigma), diffusion fluxes beta (0 central, 0.5
    LDG), boundaries BC_PERIODIC or BC_DIRICHLET (u = 0 at both ends), and a
    nodal source added to the residual.
    """

    def __init__(self, equation: int, nx: int, p: int, ny: int = 1, x0: float = 0.0,
                 x1: float = 1.0, y0: float = 0.0, y1: float = 1.0, gamma: float = 1.4,
                 kappa: float = 0.0, flux: int = FLUX_LF, sigma: float = 0.0,
                 beta: float = 0.0, bc: int = BC_PERIODIC, source=None, nz: int = 1,
                 z0: float = 0.0, z1: float = 1.0, ev_ce: float = 0.0, ev_cmax: float = 0.0,
                 nu=None):
        self.equation, self.nx, self.ny, self.nz, self.p = equation, nx, ny, nz, p
        self.z0, self.z1 = z0, z1
        self.x0, self.x1, self.y0, self.y1, self.gamma = x0, x1, y0, y1, gamma
        self.kappa, self.flux, self.sigma, self.beta, self.bc = kappa, flux, sigma, beta, bc
        self.source = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
        sp = _dp(self.source) if self.source is not None else C.POINTER(C.c_double)()
        self.ev_ce, self.ev_cmax = ev_ce, ev_cmax
        self.nu = None if nu is None else np.ascontiguousarray(nu, dtype=np.float64)
        nup = _dp(self.nu) if self.nu is not None else C.POINTER(C.c_double)()
        self._m = _Mesh(equation, nx, ny, p, x0, x1, y0, y1, gamma, kappa, flux, sigma, beta,
                        bc, sp, nz, z0, z1, ev_ce, ev_cmax, nup)
        dim = {BURGERS1D: 1, EULER2D: 2, EULER3D: 3}.get(equation, 1)
        self.dim = dim
        self.nvar = 1 if equation == BURGERS1D else dim + 2
        self.Np = (p + 1) ** dim
        self.K = nx * ny * (nz if equation == EULER3D else 1)
        self.n = lib().orc_ndof(C.byref(self._m))
        if self.n < 0:
            raise ValueError("invalid oracle mesh")
        if self.source is not None and self.source.size != self.n:
            raise ValueError("source must have one entry per degree of freedom")

    # geometry ------------------------------------------------------------
    def nodes(self):
        """(x, y) node coordinates, (x, y, z) for Euler 3D."""
        x = np.zeros(self.K * self.Np)
        y = np.zeros(self.K * self.Np)
        z = np.zeros(self.K * self.Np)
        _check(lib().orc_nodes(C.byref(self._m), _dp(x), _dp(y), _dp(z)), "nodes")
        return (x, y, z) if self.dim == 3 else (x, y)

    def mass(self):
        w = np.zeros(self.K * self.Np)
        _check(lib().orc_mass(C.byref(self._m), _dp(w)), "mass")
        return w

    def max_speed(self, q):
        c, d = C.c_double(), C.c_double()
        _check(lib().orc_max_speed(C.byref(self._m), _dp(q), C.byref(c), C.byref(d)), "speed")
        return c.value, d.value

    # operators -----------------------------------------------------------
    def rhs(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        r = np.zeros(self.n)
        _check(lib().orc_rhs(C.byref(self._m), _dp(q), _dp(r)), "rhs")
        return r

    def jvp(self, qref, v):
        qref = np.ascontiguousarray(qref, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.zeros(self.n)
        _check(lib().orc_jvp(C.byref(self._m), _dp(qref), _dp(v), _dp(w)), "jvp")
        return w

    def entropy_viscosity(self, q, q_prev, dt):
        """Nodal entropy viscosity (K*Np values) of q after q_prev, step dt."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        q_prev = np.ascontiguousarray(q_prev, dtype=np.float64)
        nu = np.zeros(self.K * self.Np)
        _check(lib().orc_entropy_viscosity(C.byref(self._m), _dp(q), _dp(q_prev), dt, _dp(nu)),
               "entropy viscosity")
        return nu

    def ev_diffusion(self, v):
        """div(nu grad v) with the mesh's nodal viscosity."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.zeros(self.n)
        _check(lib().orc_ev_diffusion(C.byref(self._m), _dp(v), _dp(out)), "ev diffusion")
        return out

    def gradient(self, u):
        """Auxiliary variable q(u) of viscous Burgers (eq. gov-burgers1d-gradu)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        q = np.zeros(self.n)
        _check(lib().orc_gradient(C.byref(self._m), _dp(u), _dp(q)), "gradient")
        return q

    def jvp_complex_step(self, qref, v, h=1e-30):
        qref = np.ascontiguousarray(qref, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.zeros(self.n)
        _check(lib().orc_jvp_complex_step(C.byref(self._m), _dp(qref), _dp(v), h, _dp(w)),
               "complex step")
        return w

    def assemble_jvp(self, qref):
        qref = np.ascontiguousarray(qref, dtype=np.float64)
        L = np.zeros((self.n, self.n))  # filled column by column (column-major)
        _check(lib().orc_assemble_jvp(C.byref(self._m), _dp(qref), _dp(L)), "assemble")
        return np.ascontiguousarray(L.T)

    def phi_krylov(self, qref, tau, bs, tol=1e-10, m_min=10, m_max=64, check_every=1,
                   forced=None, stats=False, iop=0, adapt=0, m_init=0):
        qref = np.ascontiguousarray(qref, dtype=np.float64)
        out = np.zeros(self.n)
        opts, st, keep = _kopts(tol, m_min, m_max, check_every, forced, iop=iop, adapt=adapt,
                                m_init=m_init)
        barr, keep2 = _bvec(bs)
        rc = lib().orc_phi_krylov_dg(C.byref(self._m), _dp(qref), tau, len(bs) - 1, barr,
                                     _dp(out), C.byref(opts), C.byref(st))
        _check(rc, "phi_krylov")
        return (out, _stats(st)) if stats else out

    def step(self, scheme, dt, q, q_prev=None, tol=1e-10, m_min=10, m_max=64, check_every=1,
             forced=None, stats=False, iop=0, adapt=0, m_init=0):
        """One step; returns (q_new, q_prev_new[, stats]).  Inputs are not modified."""
        q = np.array(q, dtype=np.float64, copy=True)
        have_prev = q_prev is not None
        qp = (np.array(q_prev, dtype=np.float64, copy=True) if have_prev else np.zeros(self.n))
        opts, st, keep = _kopts(tol, m_min, m_max, check_every, forced, iop=iop, adapt=adapt,
                                m_init=m_init)
        rc = lib().orc_step(C.byref(self._m), scheme, dt, _dp(q), _dp(qp), int(have_prev),
                            C.byref(opts), C.byref(st))
        _check(rc, "step")
        return (q, qp, _stats(st)) if stats else (q, qp)

    def rk4(self, q, dt, nsteps):
        q = np.array(q, dtype=np.float64, copy=True)
        _check(lib().orc_rk4(C.byref(self._m), dt, nsteps, _dp(q)), "rk4")
        return q


def _bvec(bs):
    arrs = [None if b is None else np.ascontiguousarray(b, dtype=np.float64) for b in bs]
    barr = (C.POINTER(C.c_double) * len(arrs))()
    for i, a in enumerate(arrs):
        barr[i] = _dp(a) if a is not None else C.POINTER(C.c_double)()
    return barr, arrs


def _kopts(tol, m_min, m_max, check_every, forced, log_cap=4096, iop=0, adapt=0, m_init=0):
    if forced:
        fa = (Substep * len(forced))(*[Substep(int(m), int(last), float(dt))
                                       for (m, dt, last) in forced])
        fp, nf = fa, len(forced)
    else:
        fa, fp, nf = None, None, 0
    opts = _KOpts(tol, m_min, m_max, check_every, fp, nf, iop, adapt, m_init)
    log = (Substep * log_cap)()
    st = _KStats(0, 0, 0, 0, 0, 0, 0, 0.0, log, log_cap, 0, 0, 0)
    return opts, st, (fa, log)


def _stats(st):
    n = min(st.log_len, st.log_cap)
    return {
        "substeps": st.substeps, "rejects": st.rejects, "krylov_iters": st.krylov_iters,
        "jvps": st.jvps, "breakdown": st.breakdown, "phi_calls": st.phi_calls,
        "rhs_calls": st.rhs_calls, "err_est": st.err_est,
        "log": [(st.log[i].m, st.log[i].dtau, st.log[i].last) for i in range(n)],
        "checks": st.checks, "m_next": st.m_next,
    }


def lgl(p: int):
    """LGL nodes, weights and differentiation matrix D[i, j] = l_j'(xi_i)."""
    xi, w, D = np.zeros(p + 1), np.zeros(p + 1), np.zeros((p + 1) * (p + 1))
    _check(lib().orc_lgl(p, _dp(xi), _dp(w), _dp(D)), "lgl")
    return xi, w, D.reshape(p + 1, p + 1)


def expm(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    E = np.zeros_like(A)
    _check(lib().orc_expm(n, _dp(A), _dp(E)), "expm")
    return E


def phi_dense(A, tau, bs):
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros(A.shape[0])
    barr, keep = _bvec(bs)
    _check(lib().orc_phi_dense(A.shape[0], _dp(A), tau, len(bs) - 1, barr, _dp(out)),
           "phi_dense")
    return out


def phi_krylov_dense(A, tau, bs, tol=1e-10, m_min=10, m_max=64, check_every=1, forced=None,
                     stats=False, iop=0, adapt=0, m_init=0):
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros(A.shape[0])
    opts, st, keep = _kopts(tol, m_min, m_max, check_every, forced, iop=iop, adapt=adapt,
                                m_init=m_init)
    barr, keep2 = _bvec(bs)
    rc = lib().orc_phi_krylov_dense(A.shape[0], _dp(A), tau, len(bs) - 1, barr, _dp(out),
                                    C.byref(opts), C.byref(st))
    _check(rc, "phi_krylov_dense")
    return (out, _stats(st)) if stats else out


def arnoldi_dense(A, b, m, iop=0):
    """m Arnoldi steps of the phi evaluations' orthogonalization: (V, H), V of
    shape (m+1, n) (rows are basis vectors), H of shape (m+1, m)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = A.shape[0]
    V, H = np.zeros((m + 1, n)), np.zeros((m + 1, m))
    _check(lib().orc_arnoldi_dense(n, _dp(A), _dp(b), m, iop, _dp(V), _dp(H)), "arnoldi")
    return V, H


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(n)
