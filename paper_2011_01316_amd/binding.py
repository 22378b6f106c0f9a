"""Thin ctypes binding of ``libexpdg.so`` (C ABI in ``include/expdg.h``).

Argument marshalling only: every entry point forwards device pointers (torch
tensors' ``data_ptr()``), sizes and the current HIP stream to the library,
where all the work runs in HIP kernels.  The module-level functions carry the
C names (``expdg_mesh_create``, ``expdg_rhs``, ``expdg_jvp``,
``expdg_phi_krylov``, ``expdg_step``, ...); :class:`Mesh` wraps a handle for
convenience.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexpdg.so")

BURGERS1D, EULER2D, EULER3D = 1, 2, 3
FP64, FP32_BULK = 0, 1
EPI2, EPI3, EXPRB32, EXPRB42 = 2, 3, 32, 42
FLUX_LF, FLUX_EF, FLUX_EF_LOCAL = 0, 1, 2
BC_PERIODIC, BC_DIRICHLET, BC_WALL_Y = 0, 1, 2
OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5


class ExpdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"expdg error {code}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("equation", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("p", C.c_int),
                ("precision", C.c_int), ("device", C.c_int), ("x0", C.c_double),
                ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("m_max", C.c_int), ("kappa", C.c_double),
                ("flux", C.c_int), ("sigma", C.c_double), ("beta", C.c_double),
                ("bc", C.c_int), ("has_source", C.c_int), ("nz", C.c_int), ("z0", C.c_double),
                ("z1", C.c_double), ("ev_ce", C.c_double), ("ev_cmax", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [("ndof", C.c_size_t), ("nvar", C.c_int), ("K", C.c_int), ("Np", C.c_int),
                ("elem_bytes", C.c_int), ("hx", C.c_double), ("hy", C.c_double),
                ("dx_min", C.c_double), ("hz", C.c_double)]


class Substep(C.Structure):
    _fields_ = [("m", C.c_int), ("last", C.c_int), ("dtau", C.c_double)]


class KrylovOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("m_min", C.c_int), ("m_max", C.c_int),
                ("check_every", C.c_int), ("forced", C.POINTER(Substep)), ("n_forced", C.c_int),
                ("iop", C.c_int), ("adapt", C.c_int), ("m_init", C.c_int)]


class KrylovStats(C.Structure):
    _fields_ = [("substeps", C.c_int), ("rejects", C.c_int), ("krylov_iters", C.c_int),
                ("jvps", C.c_int), ("breakdown", C.c_int), ("phi_calls", C.c_int),
                ("rhs_calls", C.c_int), ("err_est", C.c_double),
                ("log", C.POINTER(Substep)), ("log_cap", C.c_int), ("log_len", C.c_int),
                ("checks", C.c_int), ("m_next", C.c_int)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("total_ms", C.c_double), ("bytes", C.c_double)]


class Request(C.Structure):
    _fields_ = [("mesh", MeshDesc), ("scheme", C.c_int), ("nsteps", C.c_int),
                ("dt", C.c_double), ("cfl", C.c_double), ("tol", C.c_double),
                ("m_min", C.c_int), ("m_max", C.c_int), ("check_every", C.c_int),
                ("iop", C.c_int), ("adapt", C.c_int)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int), ("error", C.c_int), ("steps_done", C.c_int),
                ("dt", C.c_double), ("stats", KrylovStats), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("bytes", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("ticks", C.c_longlong), ("grouped_launches", C.c_longlong),
                ("batched_checks", C.c_longlong), ("arnoldi_items", C.c_longlong),
                ("check_items", C.c_longlong), ("active", C.c_int), ("queued", C.c_int),
                ("done", C.c_int), ("arena_bytes", C.c_size_t), ("arena_used", C.c_size_t),
                ("arena_peak", C.c_size_t)]


REQ_QUEUED, REQ_ACTIVE, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

K_RESIDUAL, K_LINEAR, K_GS_DOTS, K_SMALLEXPM, K_COMBINE = 0, 1, 2, 3, 4
K_GS_UPDATE, K_GS_NORM, K_GS_FINISH = 5, 6, 7
K_EV_VISC = 8
K_GS_FOLD = 9
KERNEL_CLASSES = {K_RESIDUAL: "residual", K_LINEAR: "linear_operator", K_GS_DOTS: "gs_dots",
                  K_SMALLEXPM: "small_expm", K_COMBINE: "combine", K_GS_UPDATE: "gs_update",
                  K_GS_NORM: "gs_norm", K_GS_FINISH: "gs_finish", K_EV_VISC: "ev_visc",
                  K_GS_FOLD: "gs_fold"}
# kernel symbol of each class, as rocprofv3 names it
# kernels of the 64x64 p=4 vortex (410 operator blocks: the linear operator
# runs as 512-thread blocks there; larger grids launch euler_op<p, T, true, false>)
KERNEL_SYMBOLS = {"residual": "euler_op<4, double, false, false>",
                  "linear_operator": "euler_op_halves<4, double>",
                  "gs_dots": "gs_dots2_kernel<double>", "small_expm": "hess_expm_kernel",
                  "combine": "combine_kernel<double>", "gs_update": "dcgs_update_kernel<double>",
                  "gs_norm": "gs_norm_kernel<double>",
                  "gs_finish": "dcgs_finish_kernel / finish_norm_kernel",
                  "ev_visc": "ev_element_kernel<4> / ev_smooth_kernel<4, double>",
                  "gs_fold": "fold_kernel"}

# name -> (restype, argtypes)
_SIGS = {
    "expdg_mesh_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(C.c_void_p)]),
    "expdg_mesh_destroy": (C.c_int, [C.c_void_p]),
    "expdg_workspace_bytes": (C.c_size_t, [C.POINTER(MeshDesc)]),
    "expdg_mesh_get_info": (C.c_int, [C.c_void_p, C.POINTER(MeshInfo)]),
    "expdg_mesh_nodes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_mesh_set_source": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_mesh_set_viscosity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_entropy_viscosity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_void_p, C.c_void_p]),
    "expdg_lgl": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_jvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_jvp_noalloc": (C.c_int, [C.POINTER(MeshDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "expdg_max_speed": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "expdg_phi_krylov": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                   C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(KrylovOpts),
                                   C.POINTER(KrylovStats), C.c_void_p]),
    "expdg_step": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int,
                             C.POINTER(KrylovOpts), C.POINTER(KrylovStats), C.c_void_p]),
    "expdg_integrate": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_void_p,
                                  C.c_void_p, C.c_int, C.POINTER(KrylovOpts),
                                  C.POINTER(KrylovStats), C.c_void_p]),
    "expdg_small_expm": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "expdg_profile_enable": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "expdg_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(KernelProfile)]),
    "expdg_request_bytes": (C.c_size_t, [C.POINTER(Request)]),
    "expdg_server_create": (C.c_int, [C.c_int, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    "expdg_server_destroy": (C.c_int, [C.c_void_p]),
    "expdg_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.c_void_p,
                                      C.POINTER(C.c_longlong)]),
    "expdg_server_tick": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "expdg_server_finished": (C.c_int, [C.c_void_p, C.POINTER(C.c_longlong), C.c_int]),
    "expdg_server_poll": (C.c_int, [C.c_void_p, C.c_longlong, C.POINTER(RequestInfo)]),
    "expdg_server_fetch": (C.c_int, [C.c_void_p, C.c_longlong, C.c_void_p]),
    "expdg_server_cancel": (C.c_int, [C.c_void_p, C.c_longlong]),
    "expdg_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "expdg_server_sync": (C.c_int, [C.c_void_p]),
    "expdg_server_clock": (C.c_double, [C.c_void_p]),
    "expdg_last_error": (C.c_char_p, []),
    "expdg_version": (C.c_int, []),
}

_lib = None


def lib():
    """Load libexpdg.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ExpdgError(EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int):
    if rc != OK:
        raise ExpdgError(rc, lib().expdg_last_error().decode(errors="replace"))


def _ptr(x):
    """Device pointer of a tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---- C names ---------------------------------------------------------------
def expdg_mesh_create(desc: MeshDesc) -> int:
    h = C.c_void_p()
    _check(lib().expdg_mesh_create(C.byref(desc), C.byref(h)))
    return h.value


def expdg_mesh_destroy(handle: int) -> None:
    _check(lib().expdg_mesh_destroy(handle))


def expdg_workspace_bytes(desc: MeshDesc) -> int:
    return lib().expdg_workspace_bytes(C.byref(desc))


def expdg_mesh_set_source(handle, s, stream=None):
    import torch
    if not (isinstance(s, torch.Tensor) and s.dtype == torch.float64 and s.is_contiguous()):
        raise ExpdgError(EINVAL, "the source must be a contiguous float64 device tensor")
    _check(lib().expdg_mesh_set_source(handle, _ptr(s), _stream(stream)))


def _f64_dev(x, what):
    import torch
    if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_contiguous()):
        raise ExpdgError(EINVAL, what + " must be a contiguous float64 device tensor")
    return _ptr(x)


def expdg_mesh_set_viscosity(handle, nu, stream=None):
    _check(lib().expdg_mesh_set_viscosity(handle, _f64_dev(nu, "nu"), _stream(stream)))


def expdg_entropy_viscosity(handle, q, q_prev, dt, nu=None, stream=None):
    _check(lib().expdg_entropy_viscosity(handle, _f64_dev(q, "q"), _f64_dev(q_prev, "q_prev"),
                                         float(dt), None if nu is None else _f64_dev(nu, "nu"),
                                         _stream(stream)))


def expdg_rhs(handle, q, r, stream=None):
    _check(lib().expdg_rhs(handle, _ptr(q), _ptr(r), _stream(stream)))


def expdg_jvp(handle, qref, v, w, stream=None):
    _check(lib().expdg_jvp(handle, _ptr(qref), _ptr(v), _ptr(w), _stream(stream)))


def expdg_jvp_noalloc(desc: MeshDesc, qref, v, w, stream=None):
    _check(lib().expdg_jvp_noalloc(C.byref(desc), _ptr(qref), _ptr(v), _ptr(w), _stream(stream)))


def expdg_max_speed(handle, q, stream=None) -> float:
    c = C.c_double()
    _check(lib().expdg_max_speed(handle, _ptr(q), C.byref(c), _stream(stream)))
    return c.value


def make_opts(tol=1e-10, m_min=10, m_max=64, check_every=1, forced=None, iop=0, adapt=0,
              m_init=0):
    """Krylov options; forced is a list of (m, dtau, last); iop > 0 selects
    incomplete orthogonalization against the iop most recent vectors; adapt = 1
    the cost-based choice of the Krylov size and the substep."""
    keep = None
    if forced:
        keep = (Substep * len(forced))(*[Substep(int(m), int(last), float(dt))
                                         for (m, dt, last) in forced])
        o = KrylovOpts(tol, m_min, m_max, check_every, keep, len(forced), iop, adapt, m_init)
    else:
        o = KrylovOpts(tol, m_min, m_max, check_every, None, 0, iop, adapt, m_init)
    o._keep = keep
    return o


def make_stats(log_cap=4096):
    log = (Substep * log_cap)()
    s = KrylovStats(0, 0, 0, 0, 0, 0, 0, 0.0, log, log_cap, 0, 0, 0)
    s._keep = log
    return s


def stats_dict(s: KrylovStats):
    n = min(s.log_len, s.log_cap)
    return {"substeps": s.substeps, "rejects": s.rejects, "krylov_iters": s.krylov_iters,
            "jvps": s.jvps, "breakdown": s.breakdown, "phi_calls": s.phi_calls,
            "rhs_calls": s.rhs_calls, "err_est": s.err_est,
            "log": [(s.log[i].m, s.log[i].dtau, s.log[i].last) for i in range(n)],
            "checks": s.checks, "m_next": s.m_next}


def expdg_phi_krylov(handle, qref, tau, bs, w, opts, stats=None, stream=None):
    arr = (C.c_void_p * len(bs))(*[_ptr(b) for b in bs])
    _check(lib().expdg_phi_krylov(handle, _ptr(qref), tau, len(bs) - 1, arr, _ptr(w),
                                  C.byref(opts), C.byref(stats) if stats is not None else None,
                                  _stream(stream)))


def expdg_step(handle, scheme, dt, q, q_prev, have_prev, opts, stats=None, stream=None):
    _check(lib().expdg_step(handle, scheme, dt, _ptr(q), _ptr(q_prev), int(have_prev),
                            C.byref(opts), C.byref(stats) if stats is not None else None,
                            _stream(stream)))


def expdg_integrate(handle, scheme, dt, nsteps, q, q_prev, have_prev, opts, stats=None,
                    stream=None):
    _check(lib().expdg_integrate(handle, scheme, dt, int(nsteps), _ptr(q), _ptr(q_prev),
                                 int(have_prev), C.byref(opts),
                                 C.byref(stats) if stats is not None else None, _stream(stream)))


def expdg_small_expm(n, A, E, stream=None):
    _check(lib().expdg_small_expm(n, _ptr(A), _ptr(E), _stream(stream)))


def expdg_profile_enable(handle, kernel_class, enable=True):
    _check(lib().expdg_profile_enable(handle, kernel_class, int(enable)))


def expdg_profile_read(handle, kernel_class):
    out = KernelProfile()
    _check(lib().expdg_profile_read(handle, kernel_class, C.byref(out)))
    return {"launches": out.launches, "total_ms": out.total_ms, "bytes": out.bytes}


def expdg_lgl(p):
    import numpy as np
    xi, w, D = np.zeros(p + 1), np.zeros(p + 1), np.zeros((p + 1) * (p + 1))
    _check(lib().expdg_lgl(p, xi.ctypes.data, w.ctypes.data, D.ctypes.data))
    return xi, w, D.reshape(p + 1, p + 1)


# ---- convenience wrapper ------------------------------------------------------
class Mesh:
    """Owns an expdg mesh handle; methods forward to the C entry points."""

    def __init__(self, equation, nx, p, ny=1, precision=FP64, device=0, x0=0.0, x1=1.0,
                 y0=0.0, y1=1.0, gamma=1.4, m_max=64, kappa=0.0, flux=FLUX_LF, sigma=0.0,
                 beta=0.0, bc=BC_PERIODIC, has_source=False, nz=1, z0=0.0, z1=1.0, ev_ce=0.0,
                 ev_cmax=0.0):
        self.desc = MeshDesc(equation, nx, ny, p, precision, device, x0, x1, y0, y1, gamma,
                             m_max, kappa, flux, sigma, beta, bc, int(bool(has_source)), nz, z0,
                             z1, ev_ce, ev_cmax)
        self.handle = expdg_mesh_create(self.desc)
        info = MeshInfo()
        _check(lib().expdg_mesh_get_info(self.handle, C.byref(info)))
        self.n, self.nvar, self.K, self.Np = info.ndof, info.nvar, info.K, info.Np
        self.hx, self.hy, self.hz, self.dx_min = info.hx, info.hy, info.hz, info.dx_min
        self.elem_bytes = info.elem_bytes
        self.p, self.equation, self.precision = p, equation, precision

    def close(self):
        if self.handle:
            expdg_mesh_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    def nodes(self):
        """(x, y) node coordinates, (x, y, z) for Euler 3D."""
        import numpy as np
        x = np.zeros(self.K * self.Np)
        y = np.zeros(self.K * self.Np)
        z = np.zeros(self.K * self.Np)
        _check(lib().expdg_mesh_nodes(self.handle, x.ctypes.data, y.ctypes.data, z.ctypes.data))
        return (x, y, z) if self.equation == EULER3D else (x, y)

    def set_source(self, s, stream=None):
        """s: float64 device tensor of ndof entries (copied into the mesh)."""
        expdg_mesh_set_source(self.handle, s, stream)

    def set_viscosity(self, nu, stream=None):
        """nu: float64 device tensor of K*Np nodal viscosities (copied into the mesh)."""
        expdg_mesh_set_viscosity(self.handle, nu, stream)

    def entropy_viscosity(self, q, q_prev, dt, nu=None, stream=None):
        """Sets the mesh's viscosity from q after q_prev (float64 device tensors);
        also writes it to nu (float64, K*Np) when given."""
        expdg_entropy_viscosity(self.handle, q, q_prev, dt, nu, stream)

    def rhs(self, q, r, stream=None):
        expdg_rhs(self.handle, q, r, stream)

    def jvp(self, qref, v, w, stream=None):
        expdg_jvp(self.handle, qref, v, w, stream)

    def max_speed(self, q, stream=None):
        return expdg_max_speed(self.handle, q, stream)

    def phi_krylov(self, qref, tau, bs, w, opts, stats=None, stream=None):
        expdg_phi_krylov(self.handle, qref, tau, bs, w, opts, stats, stream)

    def step(self, scheme, dt, q, q_prev=None, have_prev=False, opts=None, stats=None,
             stream=None):
        expdg_step(self.handle, scheme, dt, q, q_prev, have_prev, opts or make_opts(), stats,
                   stream)

    def integrate(self, scheme, dt, nsteps, q, q_prev=None, have_prev=False, opts=None,
                  stats=None, stream=None):
        expdg_integrate(self.handle, scheme, dt, nsteps, q, q_prev, have_prev,
                        opts or make_opts(), stats, stream)


# ---- solve server -------------------------------------------------------------
def make_request(equation, nx, p, ny=1, scheme=EPI3, nsteps=20, dt=0.0, cfl=0.0, tol=1e-10,
                 m_min=10, m_max=64, check_every=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                 gamma=1.4, mesh_m_max=64, kappa=0.0, flux=FLUX_LF, sigma=0.0, beta=0.0,
                 bc=BC_PERIODIC, iop=0, adapt=0, ev_ce=0.0, ev_cmax=0.0):
    return Request(MeshDesc(equation, nx, ny, p, FP64, 0, x0, x1, y0, y1, gamma, mesh_m_max,
                            kappa, flux, sigma, beta, bc, 0, 1, 0.0, 1.0, ev_ce, ev_cmax),
                   scheme, nsteps, dt, cfl, tol, m_min, m_max, check_every, iop, adapt)


def expdg_request_bytes(req: Request) -> int:
    return lib().expdg_request_bytes(C.byref(req))


def expdg_server_create(device: int, hbm_budget: int, max_active: int) -> int:
    h = C.c_void_p()
    _check(lib().expdg_server_create(device, hbm_budget, max_active, C.byref(h)))
    return h.value


def expdg_server_destroy(handle: int) -> None:
    _check(lib().expdg_server_destroy(handle))


def expdg_server_submit(handle, req: Request, q0) -> int:
    """q0: contiguous float64 numpy array on the host (copied)."""
    import numpy as np
    q0 = np.ascontiguousarray(q0, dtype=np.float64)
    rid = C.c_longlong()
    _check(lib().expdg_server_submit(handle, C.byref(req), q0.ctypes.data, C.byref(rid)))
    return rid.value


def expdg_server_tick(handle, block=True) -> int:
    n = C.c_int()
    _check(lib().expdg_server_tick(handle, int(block), C.byref(n)))
    return n.value


def expdg_server_finished(handle, cap=4096):
    ids = (C.c_longlong * cap)()
    k = lib().expdg_server_finished(handle, ids, cap)
    if k < 0:
        _check(k)
    return [ids[i] for i in range(k)]


def expdg_server_poll(handle, rid):
    info = RequestInfo()
    _check(lib().expdg_server_poll(handle, rid, C.byref(info)))
    st = info.stats
    return {"state": info.state, "error": info.error, "steps_done": info.steps_done,
            "dt": info.dt, "t_submit": info.t_submit, "t_admit": info.t_admit,
            "t_done": info.t_done, "bytes": info.bytes,
            "stats": {"substeps": st.substeps, "rejects": st.rejects,
                      "krylov_iters": st.krylov_iters, "jvps": st.jvps,
                      "breakdown": st.breakdown, "phi_calls": st.phi_calls,
                      "rhs_calls": st.rhs_calls, "err_est": st.err_est}}


def expdg_server_fetch(handle, rid, n):
    import numpy as np
    out = np.empty(n, dtype=np.float64)
    _check(lib().expdg_server_fetch(handle, rid, out.ctypes.data))
    return out


def expdg_server_cancel(handle, rid):
    _check(lib().expdg_server_cancel(handle, rid))


def expdg_server_get_stats(handle):
    s = ServerStats()
    _check(lib().expdg_server_get_stats(handle, C.byref(s)))
    return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def expdg_server_sync(handle):
    _check(lib().expdg_server_sync(handle))


def expdg_server_clock(handle) -> float:
    return lib().expdg_server_clock(handle)


class Server:
    """Owns an expdg solve server; methods forward to the C entry points."""

    def __init__(self, hbm_budget=64 << 30, max_active=256, device=0):
        self.handle = expdg_server_create(device, hbm_budget, max_active)
        self._ndof = {}

    def close(self):
        if self.handle:
            expdg_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req: Request, q0) -> int:
        rid = expdg_server_submit(self.handle, req, q0)
        self._ndof[rid] = len(q0)
        return rid

    def tick(self, block=True) -> int:
        return expdg_server_tick(self.handle, block)

    def finished(self):
        return expdg_server_finished(self.handle)

    def poll(self, rid):
        return expdg_server_poll(self.handle, rid)

    def fetch(self, rid):
        out = expdg_server_fetch(self.handle, rid, self._ndof[rid])
        self._ndof.pop(rid, None)
        return out

    def cancel(self, rid):
        expdg_server_cancel(self.handle, rid)
        self._ndof.pop(rid, None)

    def stats(self):
        return expdg_server_get_stats(self.handle)

    def sync(self):
        expdg_server_sync(self.handle)

    def clock(self) -> float:
        return expdg_server_clock(self.handle)
