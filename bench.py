#!/usr/bin/env python3
"""Benchmark of the exponential-DG hot path on one MI355X.

Workload (the value): 2D compressible Euler (gamma = 1.4), isentropic vortex
(strength 5, alpha = 2, centre (5, 5), mean flow (0.2, 0)) on the periodic
square [0, 10]^2, 64 x 64 quadrilaterals, tensor LGL degree 4 (409,600 DOF),
Rusanov flux, EPI3 steps with adaptive Krylov (tol 1e-10, m_min 10, m_max
64), Courant number 5, FP64.  One "step" is one expdg_step call: the
residuals, the linear-operator applications, the Arnoldi passes, the small
exponentials and the combines of one EPI3 step.  Inputs are synthetic and
resident in HBM before timing.

value = DOF-stage updates/s = ndof * (residual + linear-operator applications
in the timed steps) / wall time of the timed steps.

Then: the same steps again with live HIP-event timing of every kernel class
(roofline of the dominant main-stream kernel and of the linear operator), the
FP32-bulk variant of the same workload, the FP64 / FP32-bulk comparison on the
256 x 256, p = 3 vortex (4,194,304 DOF), the served workload (2000 solves of
20 EPI3 steps arriving as a Poisson stream at 200/s, 50/50 Burgers / Euler,
sizes log-uniform; p50 / p99 arrival-to-completion latency and solves/s
through the solve server, and the same first requests run one after another
through expdg_step for comparison), and the FP64 oracle on the host cores
over a bounded sample.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-stage updates/s, 2D Euler p=4 exp-DG (FP32 vs FP64); served p50/p99 latency"
UNIT = "DOF-stage updates/s"
HBM_PEAK_GBS = 8000.0
C2 = dict(nx=64, ny=64, p=4, beta=5.0, cr=5.0, tol=1e-10, m_min=10, m_max=64,
          name="2D Euler isentropic vortex, 64x64 quads, LGL p=4 (409,600 DOF), Rusanov flux, "
               "EPI3, adaptive Krylov tol 1e-10 m<=64, Courant 5")
C3 = dict(nx=256, ny=256, p=3, beta=5.0, cr=5.0, tol=1e-10, m_min=10, m_max=64,
          name="2D Euler isentropic vortex, 256x256 quads, LGL p=3 (4,194,304 DOF), EPI3, "
               "tol 1e-10, Courant 5")
# single streaming kernels eligible as "the dominant kernel" (the finishing
# class holds two different small kernels)
MAIN_STREAM = ("linear_operator", "gs_dots", "gs_update", "gs_norm", "residual", "combine")
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2011_01316_amd", "csrc", f)
                  for f in ("dg_kernels.hip", "krylov_kernels.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(symbol, workload="vortex64_p4"):
    """HBM bytes per launch of a kernel in a workload from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if that summary was taken on
    other kernel sources (the kernels changed since the counters were read)."""
    try:
        d = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("workloads", {}).get(workload, {}).get("kernels", {}).get(symbol)
    return None if k is None else k.get("bytes_per_launch")


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


class Case:
    def __init__(self, B, inputs, torch, w, precision, scheme=None, iop=0, adapt=0):
        self.B, self.torch, self.w = B, torch, w
        self.scheme = B.EPI3 if scheme is None else scheme
        self.mesh = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=0.0, x1=10.0, y0=0.0,
                           y1=10.0, m_max=w["m_max"], precision=precision)
        self.x, self.y = self.mesh.nodes()
        self.q = torch.tensor(inputs.vortex(self.x, self.y, beta=w["beta"]).reshape(-1),
                              dtype=torch.float64, device="cuda:0")
        self.qp = torch.empty_like(self.q)
        self.dt = w["cr"] * self.mesh.dx_min / self.mesh.max_speed(self.q)
        self.opts = B.make_opts(w["tol"], w["m_min"], w["m_max"], iop=iop, adapt=adapt)
        self.have = False
        self.nsteps = 0

    def run(self, steps):
        B, torch = self.B, self.torch
        st = B.make_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the K steps in one library call (the host waits for the device at the end)
        self.mesh.integrate(self.scheme, self.dt, steps, self.q, self.qp, self.have, self.opts,
                            st)
        self.have = True
        torch.cuda.synchronize()
        self.nsteps += steps
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        apps = d["rhs_calls"] + d["jvps"]
        return dict(seconds=secs, ms_per_step=secs / steps * 1e3, stats=d, applications=apps,
                    value=self.mesh.n * apps / secs, krylov_iters_per_step=d["krylov_iters"] / steps)

    def profile(self, steps):
        B = self.B
        for c in B.KERNEL_CLASSES:
            B.expdg_profile_enable(self.mesh.handle, c, True)
        r = self.run(steps)
        prof = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(self.mesh.handle, c)
                for c in B.KERNEL_CLASSES}
        for c in B.KERNEL_CLASSES:
            B.expdg_profile_enable(self.mesh.handle, c, False)
        r["profile"] = prof
        return r

    def exact_error(self, inputs, np):
        t = self.nsteps * self.dt
        ex = inputs.vortex(self.x, self.y, t=t, beta=self.w["beta"]).reshape(-1)
        qh = self.q.cpu().numpy()
        return float(np.linalg.norm(qh - ex) / np.linalg.norm(ex)), qh


# Viscous Burgers (Section 5.1): the paper's stiff runs on k = 4, N_e = 40 (u0 =
# sin^3(2 pi x)(1 - x)^{3/2}, kappa = 0.03, zero Dirichlet ends, entropy flux
# sigma = 3e-4) with EPI2 to t = 1 at Cr_d = 161 (dt = 0.1) and Cr_d = 805
# (dt = 0.5), and a large mesh of the same problem for throughput.
VB = dict(K=40, p=4, kappa=0.03, sigma=3e-4, t_end=1.0, dts=(0.1, 0.5), tol=1e-10,
          name="viscous Burgers, u0 = sin^3(2 pi x)(1-x)^1.5 on [0,1], kappa 0.03, zero "
               "Dirichlet, LGL p=4, 40 elements, entropy flux sigma 3e-4, EPI2 to t = 1")
VB_LARGE = dict(K=131072, p=4, kappa=0.03, crd=161.0, steps=10, tol=1e-10,
                name="viscous Burgers, same problem on 131,072 elements, LGL p=4 (655,360 DOF), "
                     "Lax-Friedrichs + central diffusion fluxes, EXPRB32 at Cr_d = 161")


def run_viscous(args):
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    out = {}
    w = VB
    m = B.Mesh(B.BURGERS1D, w["K"], w["p"], x0=0.0, x1=1.0, kappa=w["kappa"], flux=B.FLUX_EF,
               sigma=w["sigma"], bc=B.BC_DIRICHLET)
    x, _ = m.nodes()
    u0 = torch.tensor(inputs.burgers_smooth(x), dtype=torch.float64, device="cuda:0")
    opts = B.make_opts(w["tol"], 5, 64)
    runs = []
    for dt in w["dts"]:
        nsteps = int(round(w["t_end"] / dt))
        times = []
        for rep in range(6):
            q = u0.clone()
            st = B.make_stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.integrate(B.EPI2, dt, nsteps, q, None, False, opts, st)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        d = B.stats_dict(st)
        runs.append(dict(dt=dt, cr_d=round(w["kappa"] * dt / m.dx_min ** 2, 1), steps=nsteps,
                         seconds_to_t1=round(sorted(times[1:])[len(times[1:]) // 2], 6),
                         krylov_iters=d["krylov_iters"], substeps=d["substeps"]))
        log(f"viscous Burgers EPI2 dt={dt}: {runs[-1]['seconds_to_t1'] * 1e3:.2f} ms to t = 1")
    m.close()
    out["paper_case"] = dict(workload=w["name"], epi2=runs)

    w = VB_LARGE
    m = B.Mesh(B.BURGERS1D, w["K"], w["p"], x0=0.0, x1=1.0, kappa=w["kappa"],
               bc=B.BC_DIRICHLET, m_max=64)
    x, _ = m.nodes()
    q = torch.tensor(inputs.burgers_smooth(x), dtype=torch.float64, device="cuda:0")
    dt = w["crd"] * m.dx_min ** 2 / w["kappa"]
    opts = B.make_opts(w["tol"], 5, 64)
    m.integrate(B.EXPRB32, dt, 2, q, None, False, opts, B.make_stats())
    res = {}
    for prof in (False, True):
        for c in B.KERNEL_CLASSES:
            B.expdg_profile_enable(m.handle, c, prof)
        st = B.make_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate(B.EXPRB32, dt, w["steps"], q, None, False, opts, st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        if not prof:
            res = dict(workload=w["name"], dt=dt, steps=w["steps"],
                       ms_per_step=round(secs / w["steps"] * 1e3, 4),
                       value=round(m.n * (d["rhs_calls"] + d["jvps"]) / secs, 1), unit=UNIT,
                       krylov_iters_per_step=d["krylov_iters"] / w["steps"])
        else:
            pr = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(m.handle, c) for c in B.KERNEL_CLASSES}
            wl = "viscous_burgers_131072_p4"
            for cls, sym in (("linear_operator", "burgers_op<4, double, true, true>"),
                             ("residual", "burgers_op<4, double, false, true>"),
                             ("gs_dots", B.KERNEL_SYMBOLS["gs_dots"]),
                             ("gs_update", B.KERNEL_SYMBOLS["gs_update"])):
                res[cls + "_roofline"] = roof(pr[cls], cls, sym, measured_traffic(sym, wl))
            tot = sum(v["total_ms"] for v in pr.values())
            res["kernel_time_share"] = {k: round(v["total_ms"] / tot, 4) for k, v in pr.items()}
    for c in B.KERNEL_CLASSES:
        B.expdg_profile_enable(m.handle, c, False)
    # the same steps with incomplete orthogonalization (window of 2) and with
    # the cost-based adaptivity (errors checked at the target sizes only)
    for key, oi in (("iop2", B.make_opts(w["tol"], 5, 64, iop=2)),
                    ("adapt", B.make_opts(w["tol"], 5, 64, adapt=1)),
                    ("iop2_adapt", B.make_opts(w["tol"], 5, 64, iop=2, adapt=1))):
        q2 = torch.tensor(inputs.burgers_smooth(x), dtype=torch.float64, device="cuda:0")
        m.integrate(B.EXPRB32, dt, 2, q2, None, False, oi, B.make_stats())
        for prof in (False, True):
            for c in B.KERNEL_CLASSES:
                B.expdg_profile_enable(m.handle, c, prof)
            st = B.make_stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.integrate(B.EXPRB32, dt, w["steps"], q2, None, False, oi, st)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            d = B.stats_dict(st)
            if not prof:
                res[key] = dict(ms_per_step=round(secs / w["steps"] * 1e3, 4),
                                value=round(m.n * (d["rhs_calls"] + d["jvps"]) / secs, 1),
                                krylov_iters_per_step=d["krylov_iters"] / w["steps"],
                                checks_per_step=d["checks"] / w["steps"])
            else:
                pr = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(m.handle, c)
                      for c in B.KERNEL_CLASSES}
                tot = sum(v["total_ms"] for v in pr.values())
                res[key]["kernel_time_share"] = {k: round(v["total_ms"] / tot, 4)
                                                 for k, v in pr.items()}
        for c in B.KERNEL_CLASSES:
            B.expdg_profile_enable(m.handle, c, False)
    log(f"viscous Burgers 131072 x p4: {res['ms_per_step']:.3f} ms/step, "
        f"iop2 {res['iop2']['ms_per_step']:.3f}")
    m.close()
    out["large"] = res
    return out


# Three-dimensional Euler (Section 5.2): the paper's strong-scaling run, the
# extruded vortex on (0,10) x (-5,5) x (0,1), 80 x 80 x 8 = 51,200 elements of
# degree 6 (87.8M DOF), EPI2 with dt = 0.125 to t = 1 (8 steps).  The paper
# reports 2346 s on 32 and 33.72 s on 4096 Skylake cores for this run (its
# Table expo-euler-strongscale-isentropic-varyCr), with 561 Krylov iterations.
E3 = dict(nx=80, ny=80, nz=8, p=6, dt=0.125, steps=8, tol=1e-10, m_min=10, m_max=64,
          name="3D Euler extruded isentropic vortex on (0,10)x(-5,5)x(0,1), 80x80x8 hexahedra, "
               "LGL p=6 (87,808,000 DOF), Rusanov flux, EPI2 dt=0.125 to t=1")
E3_PAPER_SECONDS = {32: 2346.0, 4096: 33.72}


def run_euler3d(args):
    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = E3
    out = dict(workload=w["name"])
    m = B.Mesh(B.EULER3D, w["nx"], w["p"], ny=w["ny"], nz=w["nz"], x0=0.0, x1=10.0, y0=-5.0,
               y1=5.0, z0=0.0, z1=1.0, m_max=w["m_max"])
    x, y, z = m.nodes()
    # the paper's vortex strength in this experiment is not stated; its
    # Courant number 16.49 at dt = 0.125 matches a weak vortex (0.05)
    q0h = inputs.vortex3d(x, y, z, beta=0.05).reshape(-1)
    del x, y, z
    q0 = torch.tensor(q0h, dtype=torch.float64, device="cuda:0")
    out["ndof"] = m.n
    out["courant"] = round(w["dt"] * m.max_speed(q0) / m.dx_min, 2)
    for iop, adapt in ((0, 0), (2, 0), (0, 1), (2, 1)):
        q = q0.clone()
        st = B.make_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate(B.EPI2, w["dt"], w["steps"], q, None, False,
                    B.make_opts(w["tol"], w["m_min"], w["m_max"], iop=iop, adapt=adapt), st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        ex = inputs.vortex3d(*m.nodes(), t=w["dt"] * w["steps"], beta=0.05).reshape(-1)
        err = float(np.linalg.norm(q.cpu().numpy() - ex) / np.linalg.norm(ex))
        key = ("full_orthogonalization" if iop == 0 else "iop2") + ("_adapt" if adapt else "")
        out[key] = dict(seconds_to_t1=round(secs, 4), krylov_iters=d["krylov_iters"],
                        substeps=d["substeps"], checks=d["checks"],
                        value=round(m.n * (d["rhs_calls"] + d["jvps"]) / secs, 1), unit=UNIT,
                        l2_rel_err_vs_exact=err,
                        vs_paper_4096_cores=round(E3_PAPER_SECONDS[4096] / secs, 2),
                        vs_paper_32_cores=round(E3_PAPER_SECONDS[32] / secs, 1))
        log(f"3D Euler 80x80x8 p=6 ({key}): {secs:.3f} s to t = 1, "
            f"{d['krylov_iters']} Krylov iterations")
    out["paper_seconds"] = {str(k): v for k, v in E3_PAPER_SECONDS.items()}
    out["paper_krylov_iters"] = 561
    # one more step with live kernel timing (linear operator, update sweep)
    for c in B.KERNEL_CLASSES:
        B.expdg_profile_enable(m.handle, c, True)
    q = q0.clone()
    m.integrate(B.EPI2, w["dt"], 1, q, None, False,
                B.make_opts(w["tol"], w["m_min"], w["m_max"]), B.make_stats())
    pr = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(m.handle, c) for c in B.KERNEL_CLASSES}
    for c in B.KERNEL_CLASSES:
        B.expdg_profile_enable(m.handle, c, False)
    wl = "euler3d_80x80x8_p6"
    for cls, sym in (("linear_operator", "euler3_op<6, double, true>"),
                     ("residual", "euler3_op<6, double, false>"),
                     ("gs_update", B.KERNEL_SYMBOLS["gs_update"])):
        out[cls + "_roofline"] = roof(pr[cls], cls, sym, measured_traffic(sym, wl))
    out["kernel_avg_us"] = {k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                            for k, v in pr.items()}
    m.close()
    return out


# Entropy viscosity (Section 3.2, "Artificial viscosity"): the paper's
# Kelvin-Helmholtz run of Section 5.3 (N_e = 722 = 38 x 19 elements of degree 6
# on (-5, 5) x (0, 5), periodic in x with no-slip walls at y = 0 and 5,
# c_E = 1, c_max = 0.1, EPI2 to t = 100 at dt = 0.5 and 0.04; quadrilaterals
# where the paper's footnote on h speaks of triangles), and the 512 x 512,
# p = 4 shear layer with and without the viscosity.
KH = dict(nx=38, ny=19, p=6, ce=1.0, cmax=0.1, t_end=100.0, dts=(0.5, 0.04), tol=1e-10,
          m_min=10, m_max=64,
          name="Kelvin-Helmholtz, (-5,5)x(0,5) periodic in x, no-slip walls at y = 0 and 5, "
               "38x19 quads (N_e = 722), LGL p=6 (141,512 DOF), entropy viscosity c_E = 1, "
               "c_max = 0.1, EPI2 to t = 100, FP64")
KH_PAPER_SECONDS = {"rk4_dt0.005": 8729.0, "epi2_dt0.04": 3505.0, "epi2_dt0.5": 2656.0}
SL = dict(nx=512, ny=512, p=4, cr=5.0, steps=20, tol=1e-7, m_min=10, m_max=64, ce=1.0, cmax=0.1,
          name="shear layer, periodic [0,1]^2, 512x512 quads, LGL p=4 (26,214,400 DOF), density "
               "2:1, seeded 1e-2 perturbation, EPI3 FP32-bulk at Courant 5, tol 1e-7")


def run_ev(args):
    out = {}
    if not args.no_kh:
        out["kelvin_helmholtz"] = run_kh(args)
    out["shear_layer_512_p4"] = run_shear_ev(args)
    return out


def run_kh(args):
    import math

    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = KH
    m = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=-5.0, x1=5.0, y0=0.0, y1=5.0,
               m_max=w["m_max"], ev_ce=w["ce"], ev_cmax=w["cmax"], bc=B.BC_WALL_Y)
    x, y = m.nodes()
    q0 = torch.tensor(inputs.kelvin_helmholtz(x, y).reshape(-1), dtype=torch.float64,
                      device="cuda:0")
    _, wq, _ = B.expdg_lgl(w["p"])
    wn = np.outer(wq, wq).reshape(-1) * (m.hx * m.hy / 4.0)
    mass = np.tile(wn, m.K)
    npts = m.K * m.Np
    m0 = [float(mass @ q0.cpu().numpy()[c * npts:(c + 1) * npts]) for c in range(4)]
    runs = {}

    def run_one(m, dt, iop, tag=""):
        nsteps = int(round(w["t_end"] / dt))
        q = q0.clone()
        qp = torch.empty_like(q)
        st = B.make_stats()
        opts = B.make_opts(w["tol"], w["m_min"], w["m_max"], iop=iop)
        # chunks of `chunk` steps, so that a run that loses positivity is
        # reported with the time it reached (one library call per chunk)
        chunk = nsteps if dt < 0.1 else 2
        done, failed = 0, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < nsteps and failed is None:
            k = min(chunk, nsteps - done)
            try:
                m.integrate(B.EPI2, dt, k, q, qp, done > 0, opts, st)
                done += k
            except B.ExpdgError as e:
                failed = str(e)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        paper_key = f"epi2_dt{dt:g}"
        key = paper_key + ("_iop2" if iop else "") + tag
        r = dict(dt=dt, iop=iop, steps=nsteps, steps_done=done, t_reached=round(done * dt, 3),
                 seconds=round(secs, 3), ms_per_step=round(secs / max(1, done) * 1e3, 4),
                 krylov_iters=d["krylov_iters"], substeps=d["substeps"], rejects=d["rejects"],
                 courant=round(dt * m.max_speed(q0) / m.dx_min, 2))
        if failed is None:
            qh = q.cpu().numpy()
            rho = qh[:npts]
            vel2 = (qh[npts:2 * npts] ** 2 + qh[2 * npts:3 * npts] ** 2) / rho
            pr = 0.4 * (qh[3 * npts:] - 0.5 * vel2)
            nu = torch.empty(npts, dtype=torch.float64, device="cuda:0")
            m.entropy_viscosity(q, qp, dt, nu)
            r.update(seconds_to_t100=round(secs, 3),
                     vs_paper=round(KH_PAPER_SECONDS[paper_key] / secs, 1),
                     min_density=float(rho.min()), min_pressure=float(pr.min()),
                     max_nu_final=float(nu.max().item()),
                     mass_energy_drift=max(abs(float(mass @ qh[c * npts:(c + 1) * npts]) -
                                               m0[c]) / max(1.0, abs(m0[c])) for c in (0, 3)))
            log(f"KH EPI2 dt={dt} iop={iop}{tag}: {secs:.3f} s to t = 100 ({nsteps} steps, "
                f"{d['krylov_iters']} Krylov iterations)")
        else:
            r["diverged"] = failed
            log(f"KH EPI2 dt={dt}{tag}: diverged after t = {done * dt:g} ({failed})")
        runs[key] = r

    # both of the paper's steps, and the smaller one again with incomplete
    # orthogonalization (L = 2)
    for dt, iop in [(dt, 0) for dt in w["dts"]] + [(min(w["dts"]), 2)]:
        run_one(m, dt, iop)
    # sensitivity of the larger step to the amount of viscosity: the same run
    # with the cap constant c_max raised by sqrt(2)
    ms = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=-5.0, x1=5.0, y0=0.0, y1=5.0,
                m_max=w["m_max"], ev_ce=w["ce"], ev_cmax=w["cmax"] * math.sqrt(2.0),
                bc=B.BC_WALL_Y)
    run_one(ms, max(w["dts"]), 0, "_cmax_x1.414")
    runs[f"epi2_dt{max(w['dts']):g}_cmax_x1.414"]["note"] = "c_max = 0.1 sqrt(2) (not the paper's)"
    ms.close()
    m.close()
    return dict(workload=w["name"], ndof=m.n, runs=runs, paper_seconds=KH_PAPER_SECONDS)


C5 = dict(nx=512, ny=512, p=4, cr=5.0, steps=100, tol=1e-7, m_min=10, m_max=64,
          name="shear layer, periodic [0,1]^2, 512x512 quads, LGL p=4 (26,214,400 DOF), density "
               "2:1, seeded 1e-2 velocity perturbation, EPI3 at Courant 5, 100 steps, tol 1e-7")


def run_c5(args):
    """The shear layer as configured: 100 EPI3 steps in FP32 bulk (FP64
    Arnoldi), and the same 100 steps in FP64 for the difference; finiteness,
    mass and energy drift."""
    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = C5
    out = dict(workload=w["name"], steps=w["steps"])
    states = {}
    for name, prec in (("fp32_bulk", B.FP32_BULK), ("fp64", B.FP64)):
        m = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], m_max=w["m_max"], precision=prec)
        x, y = m.nodes()
        q0h = inputs.shear_layer(x, y, seed=0).reshape(-1)
        del x, y
        _, wq, _ = B.expdg_lgl(w["p"])
        wn = np.tile(np.outer(wq, wq).reshape(-1) * (m.hx * m.hy / 4.0), m.K)
        npts = m.K * m.Np
        q = torch.tensor(q0h, dtype=torch.float64, device="cuda:0")
        qp = torch.empty_like(q)
        dt = w["cr"] * m.dx_min / m.max_speed(q)
        st = B.make_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate(B.EPI3, dt, w["steps"], q, qp, False,
                    B.make_opts(w["tol"], w["m_min"], w["m_max"]), st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        qh = q.cpu().numpy()
        drift = max(abs(float(wn @ (qh[c * npts:(c + 1) * npts] - q0h[c * npts:(c + 1) * npts]))) /
                    abs(float(wn @ q0h[c * npts:(c + 1) * npts])) for c in (0, 3))
        out[name] = dict(ms_per_step=round(secs / w["steps"] * 1e3, 3), dt=dt,
                         value=round(m.n * (d["rhs_calls"] + d["jvps"]) / secs, 1), unit=UNIT,
                         krylov_iters_per_step=d["krylov_iters"] / w["steps"],
                         finite=bool(np.all(np.isfinite(qh))), mass_energy_drift=drift,
                         min_density=float(qh[:npts].min()))
        states[name] = qh
        log(f"512^2 p=4 shear layer, 100 EPI3 steps, {name}: {out[name]['ms_per_step']} ms/step")
        m.close()
        del q, qp
    a, b = states["fp32_bulk"], states["fp64"]
    out["fp32_l2_rel_diff_vs_fp64"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["step_time_ratio_fp64_over_fp32"] = round(out["fp64"]["ms_per_step"] /
                                                  out["fp32_bulk"]["ms_per_step"], 3)
    return out


def run_shear_ev(args):
    """The 512 x 512 shear layer: EPI3 steps with and without the viscosity,
    then two instrumented steps with it."""
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = SL
    res = {}
    for ev in (False, True):
        kw = dict(ev_ce=w["ce"], ev_cmax=w["cmax"]) if ev else {}
        m = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], m_max=w["m_max"],
                   precision=B.FP32_BULK, **kw)
        x, y = m.nodes()
        q = torch.tensor(inputs.shear_layer(x, y, seed=0).reshape(-1), dtype=torch.float64,
                         device="cuda:0")
        del x, y
        qp = torch.empty_like(q)
        dt = w["cr"] * m.dx_min / m.max_speed(q)
        opts = B.make_opts(w["tol"], w["m_min"], w["m_max"])
        m.integrate(B.EPI3, dt, 2, q, qp, False, opts, B.make_stats())
        st = B.make_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate(B.EPI3, dt, w["steps"], q, qp, True, opts, st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = B.stats_dict(st)
        r = dict(ms_per_step=round(secs / w["steps"] * 1e3, 3),
                 value=round(m.n * (d["rhs_calls"] + d["jvps"]) / secs, 1), unit=UNIT,
                 krylov_iters_per_step=d["krylov_iters"] / w["steps"],
                 finite=bool(torch.isfinite(q).all().item()))
        if ev:
            for c in B.KERNEL_CLASSES:
                B.expdg_profile_enable(m.handle, c, True)
            m.integrate(B.EPI3, dt, 2, q, qp, True, opts, B.make_stats())
            pr = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(m.handle, c) for c in B.KERNEL_CLASSES}
            for c in B.KERNEL_CLASSES:
                B.expdg_profile_enable(m.handle, c, False)
            wl = "shear512_p4_ev"
            r["linear_operator_roofline"] = roof(
                pr["linear_operator"], "linear_operator", "euler_op<4, float, true, true>",
                measured_traffic("euler_op<4, float, true, true>", wl))
            r["ev_visc_roofline"] = roof(pr["ev_visc"], "ev_visc",
                                         "ev_element_kernel<4> / ev_smooth_kernel<4, float>")
            tot = sum(v["total_ms"] for v in pr.values())
            r["kernel_time_share"] = {k: round(v["total_ms"] / tot, 4) for k, v in pr.items()}
            r["kernel_avg_us"] = {k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                                  for k, v in pr.items()}
        res["with_ev" if ev else "without_ev"] = r
        log(f"shear layer 512^2 p=4 ev={ev}: {r['ms_per_step']:.3f} ms/step")
        m.close()
        del q, qp
    res["ev_step_cost_ratio"] = round(res["with_ev"]["ms_per_step"] /
                                      res["without_ev"]["ms_per_step"], 3)
    return dict(workload=w["name"], steps=w["steps"], **res)


def roof(p, name, symbol, traffic=None):
    if not p or not p["launches"] or p["total_ms"] <= 0:
        return None
    achieved = p["bytes"] / (p["total_ms"] * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=symbol,
                kernel_class=name, launches=p["launches"],
                avg_launch_us=round(p["total_ms"] * 1e3 / p["launches"], 3),
                avg_bytes_per_launch=round(p["bytes"] / p["launches"]))


def run_gpu(args):
    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    out = {}
    c = Case(B, inputs, torch, C2, B.FP64)
    c.run(args.warmup)
    log(f"fp64 warmup done: ndof={c.mesh.n} dt={c.dt:.5f}")
    r = c.run(args.steps)
    log(f"fp64 timed: {r['ms_per_step']:.3f} ms/step, {r['krylov_iters_per_step']:.1f} its/step")
    out["fp64"] = r
    out["fp64"]["ndof"], out["fp64"]["dt"] = c.mesh.n, c.dt
    out["fp64"]["l2_rel_err_vs_exact"], q64 = c.exact_error(inputs, np)
    out["profile"] = c.profile(args.steps)
    c.mesh.close()

    # the fourth-order EXPRB42 on the same workload (two phi evaluations per step)
    c42 = Case(B, inputs, torch, C2, B.FP64, scheme=B.EXPRB42)
    c42.run(args.warmup)
    r42 = c42.run(args.steps)
    r42["l2_rel_err_vs_exact"], _ = c42.exact_error(inputs, np)
    log(f"exprb42 timed: {r42['ms_per_step']:.3f} ms/step")
    out["exprb42"] = r42
    c42.mesh.close()

    # incomplete orthogonalization (window of 2, KIOPS' IOP) on the same workload
    if not args.no_iop:
        ci = Case(B, inputs, torch, C2, B.FP64, iop=2)
        ci.run(args.warmup)
        ri = ci.run(args.steps)
        ri["l2_rel_err_vs_exact"], qi = ci.exact_error(inputs, np)
        ri["l2_rel_diff_vs_full"] = float(np.linalg.norm(qi - q64) / np.linalg.norm(q64))
        ri["profile"] = ci.profile(args.steps)["profile"]
        log(f"iop2 timed: {ri['ms_per_step']:.3f} ms/step, "
            f"{ri['krylov_iters_per_step']:.1f} its/step")
        out["iop2"] = ri
        ci.mesh.close()

    if not args.no_fp32:
        # precision mode at equal tolerance: FP32 bulk against FP64, both at the
        # tolerance of the workload (1e-10) and at 1e-7 (what an FP32 basis can
        # resolve); each final state is kept for the comparison with the oracle
        prec = {}
        for name, pr, tol in (("fp64_tol1e-10", B.FP64, 1e-10), ("fp32_tol1e-10", B.FP32_BULK, 1e-10),
                              ("fp64_tol1e-7", B.FP64, 1e-7), ("fp32_tol1e-7", B.FP32_BULK, 1e-7),
                              ("fp64_tol1e-6", B.FP64, 1e-6), ("fp32_tol1e-6", B.FP32_BULK, 1e-6),
                              ("fp64_tol1e-10_adapt", B.FP64, 1e-10),
                              ("fp32_tol1e-10_adapt", B.FP32_BULK, 1e-10),
                              ("fp64_tol1e-7_adapt", B.FP64, 1e-7),
                              ("fp32_tol1e-7_adapt", B.FP32_BULK, 1e-7)):
            kavg = None
            if name == "fp64_tol1e-10":
                rp, qp_ = r, q64
            else:
                cp = Case(B, inputs, torch, dict(C2, tol=tol), pr,
                          adapt=1 if name.endswith("_adapt") else 0)
                cp.run(args.warmup)
                rp = cp.run(args.steps)
                qp_ = cp.q.cpu().numpy()
                if name == "fp32_tol1e-7":
                    pf = cp.profile(args.steps)["profile"]
                    kavg = {k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                            for k, v in pf.items() if v["launches"]}
                cp.mesh.close()
            prec[name] = dict(ms_per_step=round(rp["ms_per_step"], 4), value=round(rp["value"], 1),
                              krylov_iters_per_step=rp["krylov_iters_per_step"], state=qp_)
            if kavg:
                prec[name]["kernel_avg_us"] = kavg
            log(f"precision 64x64 p=4 {name}: {rp['ms_per_step']:.3f} ms/step, "
                f"{rp['krylov_iters_per_step']:.1f} its/step")
        out["precision_c2"] = dict(steps_from_start=args.warmup + args.steps, runs=prec)

    if not args.no_large:
        big = {}
        for prec, name, tol in ((B.FP64, "fp64_tol1e-10", 1e-10),
                                (B.FP32_BULK, "fp32_tol1e-10", 1e-10),
                                (B.FP64, "fp64_tol1e-7", 1e-7),
                                (B.FP32_BULK, "fp32_tol1e-7", 1e-7),
                                (B.FP64, "fp64_tol1e-6", 1e-6),
                                (B.FP32_BULK, "fp32_tol1e-6", 1e-6)):
            cb = Case(B, inputs, torch, dict(C3, tol=tol), prec)
            cb.run(1)
            rb = cb.run(args.large_steps)
            err, qb = cb.exact_error(inputs, np)
            rb["l2_rel_err_vs_exact"] = err
            rb["state"] = qb
            if name == "fp64_tol1e-10":
                rb["profile"] = cb.profile(args.large_steps)["profile"]
            log(f"256^2 p=3 {name}: {rb['ms_per_step']:.3f} ms/step")
            big[name] = rb
            cb.mesh.close()
        out["large"] = big
    return out


SERVED = dict(n_requests=2000, rate=200.0, seed=0, steps=20, tol=1e-10, m_min=10, m_max=64,
              name="served mix: 2000 solves, Poisson arrivals 200/s (seed 0), 50/50 Burgers "
                   "(K log-uniform 32..4096, p 1..4, dt 1e-2) / Euler vortex (n x n log-uniform "
                   "16..128, p 2..4, Courant 5), 20 EPI3 steps each, FP64, tol 1e-10")


def run_served(args, iop=0, compare=True, rate=None, n_requests=None):
    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs, serving

    w = SERVED
    rate = w["rate"] if rate is None else rate
    n_requests = args.serve_requests if n_requests is None else n_requests
    t = time.time()
    mix = inputs.served_mix(n_requests=n_requests, rate=rate, seed=w["seed"],
                            steps=w["steps"])
    items = serving.prepare(mix, tol=w["tol"], m_min=w["m_min"], m_max=w["m_max"], iop=iop)
    log(f"served: {len(items)} requests prepared in {time.time() - t:.1f}s")
    torch.zeros(1, device="cuda")
    srv = B.Server(hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                   max_active=args.serve_max_active)
    marks = [time.time()]

    def progress(done, n):
        if time.time() - marks[0] > 5.0:
            marks[0] = time.time()
            log(f"served: {done}/{n} done at {srv.clock():.1f}s")

    res = serving.run(srv, items, progress=progress)
    srv.sync()
    st = srv.stats()
    srv.close()
    log(f"served (iop {iop}): {res['completed']} solves, {res['solves_per_s']:.1f}/s, "
        f"p50 {res['latency_p50_s']:.2f}s p99 {res['latency_p99_s']:.2f}s")
    out = dict(
        workload=w["name"], requests=res["requests"], completed=res["completed"],
        failed=[dict(request=k, status=e, **{x: mix[k][x] for x in ("equation", "nx", "p")})
                for k, e in res["failed"]],
        latency_p50_s=round(res["latency_p50_s"], 4), latency_p99_s=round(res["latency_p99_s"], 4),
        latency_max_s=round(res["latency_max_s"], 4),
        admission_wait_p50_s=round(res["admission_wait_p50_s"], 4),
        admission_wait_p99_s=round(res["admission_wait_p99_s"], 4),
        solves_per_s=round(res["solves_per_s"], 2), makespan_s=round(res["makespan_s"], 3),
        dof_stage_updates_per_s=round(res["dof_stage_updates_per_s"], 1),
        hbm_budget_gib=args.serve_budget_gib, max_active=args.serve_max_active,
        arena_peak_gib=round(st["arena_peak"] / (1 << 30), 3),
        ticks=st["ticks"], arnoldi_steps_per_tick=round(st["arnoldi_items"] / max(1, st["ticks"]), 2),
        checks_per_batched_launch=round(st["check_items"] / max(1, st["batched_checks"]), 2),
        grouped_launches=st["grouped_launches"])

    # the first requests one after another through expdg_step
    K = min(args.serve_seq, len(items))
    if K < 1 or not compare:
        return out
    t = time.time()
    work = 0.0
    for it in items[:K]:
        r = it["req"]
        d = r.mesh
        m = B.Mesh(d.equation, d.nx, d.p, ny=d.ny, x0=d.x0, x1=d.x1, y0=d.y0, y1=d.y1,
                   m_max=d.m_max)
        q = torch.tensor(it["q0"], dtype=torch.float64, device="cuda")
        qp = torch.zeros_like(q)
        dt = r.dt if r.dt > 0 else r.cfl * m.dx_min / m.max_speed(q)
        o = B.make_opts(r.tol, r.m_min, r.m_max, r.check_every)
        st = B.make_stats(1)
        try:
            for k in range(r.nsteps):
                m.step(r.scheme, dt, q, qp, k > 0, o, st)
        except B.ExpdgError:
            pass
        work += it["ndof"] * (st.rhs_calls + st.jvps)
        m.close()
    torch.cuda.synchronize()
    el = time.time() - t
    seq = dict(requests=K, seconds=round(el, 3), solves_per_s=round(K / el, 2),
               dof_stage_updates_per_s=round(work / el, 1))
    # the same first requests through the server, arriving all at once
    srv = B.Server(hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                   max_active=args.serve_max_active)
    batch = [dict(it, arrival=0.0) for it in items[:K]]
    rb = serving.run(srv, batch)
    srv.close()
    seq["served_all_at_once"] = dict(seconds=round(rb["makespan_s"], 3),
                                     solves_per_s=round(rb["solves_per_s"], 2),
                                     dof_stage_updates_per_s=round(rb["dof_stage_updates_per_s"], 1))
    out["first_requests_compared"] = seq
    log(f"served: first {K} sequential {seq['solves_per_s']}/s vs server "
        f"{seq['served_all_at_once']['solves_per_s']}/s")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_run(oracle, inputs, w, nsteps, timed_from=1):
    """The oracle on the vortex workload w from its initial state: nsteps steps
    (an EPI2 start, then EPI3), the steps from timed_from on timed.  Returns
    (final state, seconds, operator applications timed, mesh, state after the
    first step)."""
    om = oracle.Mesh(oracle.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=0.0, x1=10.0, y0=0.0,
                     y1=10.0)
    x, y = om.nodes()
    q = inputs.vortex(x, y, beta=w["beta"]).reshape(-1)
    c, dx = om.max_speed(q)
    dt = w["cr"] * dx / c
    kw = dict(tol=w["tol"], m_min=w["m_min"], m_max=w["m_max"])
    qp, apps, secs, first = None, 0, 0.0, None
    for k in range(nsteps):
        t0 = time.perf_counter()
        q, qp, st = om.step(oracle.EPI3, dt, q, qp, stats=True, **kw)
        if k >= timed_from:
            secs += time.perf_counter() - t0
            apps += st["rhs_calls"] + st["jvps"]
        if k == 0:
            first = (q.copy(), qp.copy())
    return q, secs, apps, om, first, dt


def run_cpu_baseline(args, g, states):
    """The oracle on the host cores: the 64x64 p=4 vortex for as many steps as
    the GPU runs took from the initial state (EPI2 start untimed), the
    256x256 p=3 vortex for its steps, and two 64x64 steps on one core.  The
    final states are kept in states for the precision comparison."""
    import oracle
    from paper_2011_01316_amd import inputs

    n2 = args.warmup + args.steps
    q2, secs, apps, om, first, dt = oracle_run(oracle, inputs, C2, n2)
    states["c2"] = q2
    res = dict(value=round(om.n * apps / secs, 1), unit=UNIT, cores=oracle.num_threads(),
               kind="oracle", cpu_model=cpu_model(), host_cpus=os.cpu_count(),
               sample=f"{n2 - 1} EPI3 steps of the 64x64 p=4 vortex (409,600 DOF) after an "
                      f"untimed EPI2 start, {secs:.1f} s wall")
    log(f"oracle 64x64 p=4: {res['value']:.3g} DOF-stage updates/s on {res['cores']} threads")
    # one core: two EPI3 steps from the state after the first step
    nt = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        q, qp = first
        kw = dict(tol=C2["tol"], m_min=C2["m_min"], m_max=C2["m_max"])
        t0 = time.perf_counter()
        a1 = 0
        for _ in range(2):
            q, qp, st = om.step(oracle.EPI3, dt, q, qp, stats=True, **kw)
            a1 += st["rhs_calls"] + st["jvps"]
        s1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nt)
    res["one_core"] = dict(value=round(om.n * a1 / s1, 1), unit=UNIT, cores=1,
                           sample=f"2 EPI3 steps of the 64x64 p=4 vortex, {s1:.1f} s wall")
    log(f"oracle 64x64 p=4 on one core: {res['one_core']['value']:.3g}")
    if "large" in g:
        n3 = 1 + args.large_steps
        q3, s3, a3, om3, _, _ = oracle_run(oracle, inputs, C3, n3)
        states["c3"] = q3
        res["vortex_256x256_p3"] = dict(
            value=round(om3.n * a3 / s3, 1), unit=UNIT, cores=oracle.num_threads(),
            sample=f"{n3 - 1} EPI3 steps of the 256x256 p=3 vortex (4,194,304 DOF) after an "
                   f"untimed EPI2 start, {s3:.1f} s wall")
        log(f"oracle 256x256 p=3: {res['vortex_256x256_p3']['value']:.3g}")
    return res


def precision_report(args, g, states):
    """FP32 bulk against FP64 at equal tolerance: ms/step of each (ratio > 1:
    FP32 bulk is faster) and the relative l2 difference of each final state
    from the FP64 oracle's after the same steps from the same initial state."""
    import numpy as np

    def block(runs, ref, steps, workload):
        out = dict(workload=workload, steps_from_start=steps, runs={})
        for name, r in runs.items():
            d = {k: v for k, v in r.items() if k in ("ms_per_step", "krylov_iters_per_step",
                                                     "l2_rel_err_vs_exact", "kernel_avg_us")}
            if "value" in r:
                d["value"] = round(r["value"], 1)
            if ref is not None:
                d["l2_rel_err_vs_oracle"] = float(np.linalg.norm(r["state"] - ref) /
                                                  np.linalg.norm(ref))
            out["runs"][name] = d
        out["step_time_ratio_fp64_over_fp32"] = {
            tol: round(runs["fp64_" + tol]["ms_per_step"] / runs["fp32_" + tol]["ms_per_step"], 3)
            for tol in ("tol1e-10", "tol1e-7", "tol1e-6", "tol1e-10_adapt", "tol1e-7_adapt")
            if "fp64_" + tol in runs and "fp32_" + tol in runs}
        if ref is None:
            out["oracle"] = "not run (--no-cpu-baseline)"
        return out

    rep = {}
    if "precision_c2" in g:
        pc = g["precision_c2"]
        rep["vortex_64x64_p4"] = block(pc["runs"], states.get("c2"), pc["steps_from_start"],
                                       C2["name"])
    if "large" in g:
        rep["vortex_256x256_p3"] = block(g["large"], states.get("c3"), 1 + args.large_steps,
                                         C3["name"])
    rep["note"] = ("FP32 bulk stores the Krylov vectors, b vectors, frozen fields and operator "
                   "outputs in FP32 and computes everything in FP64 from the FP64 master state; "
                   "each pair runs the same steps at the same tolerance, so the step-time ratio "
                   "is the precision mode's own gain and l2_rel_err_vs_oracle its cost")
    return rep


def fp32_probe():
    """An EPI2 and an EPI3 step of the 256x256 p=3 vortex in FP32 bulk at tol
    1e-7 (the run the VALU / MFMA counters of the FP32 linear operator are
    read on)."""
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    c = Case(B, inputs, torch, dict(C3, tol=1e-7), B.FP32_BULK)
    r = c.run(2)
    c.mesh.close()
    return dict(workload=C3["name"] + ", FP32 bulk, tol 1e-7", steps=2,
                ms_per_step=round(r["ms_per_step"], 3),
                krylov_iters_per_step=r["krylov_iters_per_step"])


def euler3d_op_probe(reps=4):
    """The residual and the linear operator (without a dot pass) of the 3D
    run's mesh and state, applied a few times each (the run the instruction
    and wait counters of the 3D operators are read on); per-launch averages
    from the library's kernel timing (the linear operator's call also prepares
    its frozen fields, which that timing leaves out)."""
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = E3
    m = B.Mesh(B.EULER3D, w["nx"], w["p"], ny=w["ny"], nz=w["nz"], x0=0.0, x1=10.0, y0=-5.0,
               y1=5.0, z0=0.0, z1=1.0, m_max=8)
    x, y, z = m.nodes()
    q = torch.tensor(inputs.vortex3d(x, y, z, beta=0.05).reshape(-1), dtype=torch.float64,
                     device="cuda:0")
    del x, y, z
    r = torch.empty_like(q)
    lv = torch.empty_like(q)
    out = dict(workload=w["name"] + ": residual and linear operator alone", reps=reps)
    m.rhs(q, r)
    m.jvp(q, r, lv)
    torch.cuda.synchronize()
    class_id = {name: c for c, name in B.KERNEL_CLASSES.items()}
    for name, call in (("residual", lambda: m.rhs(q, r)),
                       ("linear_operator", lambda: m.jvp(q, r, lv))):
        c = class_id[name]
        B.expdg_profile_enable(m.handle, c, True)
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        pr = B.expdg_profile_read(m.handle, c)
        B.expdg_profile_enable(m.handle, c, False)
        out[name + "_us"] = round(pr["total_ms"] * 1e3 / pr["launches"], 1)
        out[name + "_gbs_algorithmic"] = round(pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9, 1)
    m.close()
    return out


def size_sweep(p, sizes=(32, 48, 64, 96, 128, 192, 256, 384, 512)):
    """The vortex of the 64x64 workload (EPI3, Courant 5, tol 1e-10, FP64) on
    n x n meshes of degree p: two steps, then two more with live kernel timing
    of the linear operator (with the step's dot pass), the update sweep, the
    finish and the residual; one JSON line per mesh with each class's average
    launch time, algorithmic bytes and their fraction of 8 TB/s."""
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    for n in sizes:
        m = B.Mesh(B.EULER2D, n, p, ny=n, x0=0.0, x1=10.0, y0=0.0, y1=10.0, m_max=64)
        x, y = m.nodes()
        q = torch.tensor(inputs.vortex(x, y, beta=5.0).reshape(-1), dtype=torch.float64,
                         device="cuda:0")
        del x, y
        qp = torch.empty_like(q)
        dt = 5.0 * m.dx_min / m.max_speed(q)
        opts = B.make_opts(1e-10, 10, 64)
        m.integrate(B.EPI3, dt, 2, q, qp, False, opts, B.make_stats())
        for c in B.KERNEL_CLASSES:
            B.expdg_profile_enable(m.handle, c, True)
        st = B.make_stats()
        m.integrate(B.EPI3, dt, 2, q, qp, True, opts, st)
        torch.cuda.synchronize()
        pr = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(m.handle, c) for c in B.KERNEL_CLASSES}
        m.close()
        row = dict(n=n, p=p, ndof=n * n * (p + 1) ** 2 * 4,
                   krylov_iters=B.stats_dict(st)["krylov_iters"])
        for k in ("linear_operator", "gs_update", "gs_finish", "gs_fold", "residual"):
            v = pr[k]
            if v["launches"]:
                row[k] = dict(us=round(v["total_ms"] * 1e3 / v["launches"], 2),
                              mb=round(v["bytes"] / v["launches"] / 1e6, 2),
                              frac=round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 3))
        print(json.dumps(row), flush=True)
        del q, qp
        torch.cuda.empty_cache()


def copy_probe(nbytes=1 << 30, reps=20):
    """Plain device-to-device copy of a known size: measured copy bandwidth and
    the reference dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return dict(bytes_read=nbytes, bytes_written=nbytes, ms=ms, gbs=2 * nbytes / (ms * 1e-3) / 1e9)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-viscous", action="store_true")
    ap.add_argument("--no-iop", action="store_true")
    ap.add_argument("--no-euler3d", action="store_true")
    ap.add_argument("--euler3d-only", action="store_true",
                    help="only the 3D Euler strong-scaling run (one JSON line)")
    ap.add_argument("--viscous-only", action="store_true",
                    help="only the viscous Burgers measurements (one JSON line)")
    ap.add_argument("--serve-requests", type=int, default=SERVED["n_requests"])
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-active", type=int, default=256)
    ap.add_argument("--serve-seq", type=int, default=40,
                    help="first requests also run one after another for comparison")
    ap.add_argument("--no-ev", action="store_true")
    ap.add_argument("--no-kh", action="store_true",
                    help="entropy viscosity: skip the Kelvin-Helmholtz runs")
    ap.add_argument("--ev-only", action="store_true",
                    help="only run the entropy-viscosity workloads and print their figures")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the served workload and print its figures")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 1 GiB device copy and print it")
    ap.add_argument("--fp32-probe", action="store_true",
                    help="only two FP32-bulk steps of the 256x256 p=3 vortex (tol 1e-7), for "
                         "instruction counters of its linear operator")
    ap.add_argument("--size-sweep", type=int, default=0, metavar="P",
                    help="only the 64x64 workload's vortex on n x n meshes of degree P, "
                         "n = 32..512: per-kernel times and roofline fractions, one line each")
    ap.add_argument("--euler3d-op-probe", action="store_true",
                    help="only the 3D run's residual and linear operator, a few times each, for "
                         "instruction and wait counters")
    args = ap.parse_args()
    if args.size_sweep:
        size_sweep(args.size_sweep)
        return
    if args.euler3d_op_probe:
        print(json.dumps(euler3d_op_probe()), flush=True)
        return
    if args.fp32_probe:
        print(json.dumps(fp32_probe()), flush=True)
        return
    if args.copy_probe:
        print(json.dumps(copy_probe()), flush=True)
        return
    if args.serve_only:
        print(json.dumps(run_served(args)), flush=True)
        return
    if args.viscous_only:
        print(json.dumps(run_viscous(args)), flush=True)
        return
    if args.euler3d_only:
        print(json.dumps(run_euler3d(args)), flush=True)
        return
    if args.ev_only:
        print(json.dumps(run_ev(args)), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_2011_01316_amd import binding as B

    g = run_gpu(args)
    f64 = g["fp64"]
    prof = g["profile"]["profile"]
    dominant = max(MAIN_STREAM, key=lambda k: prof[k]["total_ms"])
    total_ms = g["profile"]["seconds"] * 1e3
    line = {
        "metric": METRIC,
        "value": round(f64["value"], 1),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": C2["name"], "ndof": f64["ndof"], "dt": f64["dt"],
            "krylov_iters_per_step": f64["krylov_iters_per_step"],
            "applications_per_step": f64["applications"] / args.steps,
            "substeps_per_step": f64["stats"]["substeps"] / args.steps,
        },
        "roofline": roof(prof[dominant], dominant, B.KERNEL_SYMBOLS[dominant],
                         measured_traffic(B.KERNEL_SYMBOLS[dominant])),
        "linear_operator_roofline": roof(prof["linear_operator"], "linear_operator",
                                         B.KERNEL_SYMBOLS["linear_operator"],
                                         measured_traffic(B.KERNEL_SYMBOLS["linear_operator"])),
        "kernel_time_share": {k: round(v["total_ms"] / total_ms, 4) for k, v in prof.items()},
        "kernel_avg_us": {k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                          for k, v in prof.items()},
        "instrumented_ms_per_step": round(g["profile"]["ms_per_step"], 4),
        "l2_rel_err_vs_exact_vortex": f64["l2_rel_err_vs_exact"],
    }
    ei = g.get("iop2")
    pi = ei["profile"] if ei else None
    line["iop2"] = None if ei is None else dict(value=round(ei["value"], 1), unit=UNIT,
                        ms_per_step=round(ei["ms_per_step"], 4),
                        step_speedup_vs_full=round(f64["ms_per_step"] / ei["ms_per_step"], 3),
                        krylov_iters_per_step=ei["krylov_iters_per_step"],
                        l2_rel_err_vs_exact_vortex=ei["l2_rel_err_vs_exact"],
                        l2_rel_diff_vs_full_orthogonalization=ei["l2_rel_diff_vs_full"],
                        kernel_avg_us={k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                                       for k, v in pi.items()},
                        linear_operator_roofline=roof(pi["linear_operator"], "linear_operator",
                                                      B.KERNEL_SYMBOLS["linear_operator"]))
    e42 = g["exprb42"]
    line["exprb42"] = dict(value=round(e42["value"], 1), unit=UNIT,
                           ms_per_step=round(e42["ms_per_step"], 4),
                           krylov_iters_per_step=e42["krylov_iters_per_step"],
                           l2_rel_err_vs_exact_vortex=e42["l2_rel_err_vs_exact"])
    if "large" in g:
        pb = g["large"]["fp64_tol1e-10"]["profile"]
        line["large_256x256_p3"] = dict(
            workload=C3["name"], steps=args.large_steps,
            linear_operator_roofline=roof(
                pb["linear_operator"], "linear_operator", "euler_op<3, double, true, false>",
                measured_traffic("euler_op<3, double, true, false>", "vortex256_p3")),
            residual_roofline=roof(
                pb["residual"], "residual", "euler_op<3, double, false, false>",
                measured_traffic("euler_op<3, double, false, false>", "vortex256_p3")),
            gs_update_roofline=roof(pb["gs_update"], "gs_update", B.KERNEL_SYMBOLS["gs_update"],
                                    measured_traffic(B.KERNEL_SYMBOLS["gs_update"],
                                                     "vortex256_p3")),
            kernel_avg_us={k: round(v["total_ms"] * 1e3 / max(1, v["launches"]), 3)
                           for k, v in pb.items()})
    if not args.no_viscous:
        line["viscous_burgers"] = run_viscous(args)
    if not args.no_euler3d:
        line["euler3d_paper_strong_scaling"] = run_euler3d(args)
    if not args.no_ev:
        line["entropy_viscosity"] = run_ev(args)
        line["shear_layer_512x512_p4_100_steps"] = run_c5(args)
    if not args.no_serve:
        line["served"] = run_served(args)
        if not args.no_iop:
            # the same mix with incomplete orthogonalization (L = 2) in every solve
            si = run_served(args, iop=2, compare=False)
            line["served"]["iop2"] = {k: si[k] for k in (
                "completed", "solves_per_s", "latency_p50_s", "latency_p99_s",
                "dof_stage_updates_per_s", "arnoldi_steps_per_tick")}
        # offered rates the server keeps up with (the same mix, fewer requests):
        # latency is then service time plus a short admission wait
        sus = {}
        for rate, iop in ((100.0, 0), (160.0, 2)):
            r = run_served(args, iop=iop, compare=False, rate=rate,
                           n_requests=min(args.serve_requests, 1000))
            sus[f"rate{rate:g}_iop{iop}"] = {k: r[k] for k in (
                "requests", "completed", "solves_per_s", "latency_p50_s", "latency_p99_s",
                "admission_wait_p50_s", "admission_wait_p99_s", "makespan_s",
                "dof_stage_updates_per_s")}
            sus[f"rate{rate:g}_iop{iop}"]["offered_rate"] = rate
        line["served"]["sustained"] = sus
    oracle_states = {}
    line["cpu_baseline"] = None if args.no_cpu_baseline else run_cpu_baseline(args, g,
                                                                            oracle_states)
    line["precision_mode"] = precision_report(args, g, oracle_states)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
