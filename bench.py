#!/usr/bin/env python3
"""Benchmark of the exponential-DG hot path on one MI355X.

Workload: 2D compressible Euler (gamma = 1.4), isentropic vortex (strength 5,
alpha = 2, centre (5, 5), mean flow (0.2, 0)) on the periodic square [0, 10]^2,
64 x 64 quadrilaterals, tensor LGL degree 4 (409,600 DOF), Rusanov flux, EPI3
steps with adaptive Krylov (tol 1e-10, m_min 10, m_max 64), Courant number 5.
One "step" is one expdg_step call: the residuals, the linear-operator
applications, the Arnoldi passes, the small exponentials and the combines of
one EPI3 step.  Inputs are synthetic and resident in HBM before timing.

value = DOF-stage updates/s = ndof * (residual + linear-operator applications
in the timed steps) / wall time of the timed steps, in FP64.  The same steps
are then repeated with live HIP-event timing of the Gram-Schmidt passes (the
dominant kernel class) and of the linear operator for the roofline fields,
then the FP32-bulk variant of the workload is timed, and the FP64 oracle is
timed on the host cores over a bounded sample.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-stage updates/s, 2D Euler p=4 exp-DG (FP32 vs FP64); served p50/p99 latency"
UNIT = "DOF-stage updates/s"
HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(nx=64, ny=64, p=4, x0=0.0, x1=10.0, y0=0.0, y1=10.0, beta=5.0, cr=5.0,
                tol=1e-10, m_min=10, m_max=64)


def make_case(B, inputs, torch, precision):
    w = WORKLOAD
    mesh = B.Mesh(B.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=w["x0"], x1=w["x1"], y0=w["y0"],
                  y1=w["y1"], m_max=w["m_max"], precision=precision)
    x, y = mesh.nodes()
    q = torch.tensor(inputs.vortex(x, y, beta=w["beta"]).reshape(-1), dtype=torch.float64,
                     device="cuda:0")
    qp = torch.empty_like(q)
    dt = w["cr"] * mesh.dx_min / mesh.max_speed(q)
    return mesh, q, qp, dt, (x, y)


def timed_steps(B, torch, mesh, q, qp, dt, have, steps, opts):
    st = B.make_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mesh.step(B.EPI3, dt, q, qp, have, opts, st)
        have = True
    torch.cuda.synchronize()
    return time.perf_counter() - t0, B.stats_dict(st), have


def run_gpu(args):
    import numpy as np
    import torch

    from paper_2011_01316_amd import binding as B
    from paper_2011_01316_amd import inputs

    w = WORKLOAD
    opts = B.make_opts(w["tol"], w["m_min"], w["m_max"])
    out = {}
    mesh, q, qp, dt, (x, y) = make_case(B, inputs, torch, B.FP64)
    have = False
    for _ in range(args.warmup):
        mesh.step(B.EPI3, dt, q, qp, have, opts)
        have = True
    print(f"# fp64 warmup done: ndof={mesh.n} dt={dt:.5f}", file=sys.stderr, flush=True)
    secs, st, have = timed_steps(B, torch, mesh, q, qp, dt, have, args.steps, opts)
    applications = st["rhs_calls"] + st["jvps"]
    out["fp64"] = dict(seconds=secs, stats=st, applications=applications, ndof=mesh.n,
                       dt=dt, value=mesh.n * applications / secs)
    t_end = (args.warmup + args.steps) * dt
    exact = inputs.vortex(x, y, t=t_end, beta=w["beta"]).reshape(-1)
    qh = q.cpu().numpy()
    out["fp64"]["l2_rel_err_vs_exact"] = float(np.linalg.norm(qh - exact) / np.linalg.norm(exact))
    print(f"# fp64 timed: {secs / args.steps * 1e3:.3f} ms/step, "
          f"{st['krylov_iters'] / args.steps:.1f} Krylov its/step", file=sys.stderr, flush=True)

    # live per-kernel timing (HIP events on the launching stream) over the same
    # number of steps, continuing the trajectory
    for c in (B.K_GRAMSCHMIDT, B.K_LINEAR, B.K_RESIDUAL, B.K_SMALLEXPM, B.K_COMBINE):
        B.expdg_profile_enable(mesh.handle, c, True)
    secs_p, st_p, have = timed_steps(B, torch, mesh, q, qp, dt, have, args.steps, opts)
    prof = {B.KERNEL_CLASSES[c]: B.expdg_profile_read(mesh.handle, c)
            for c in B.KERNEL_CLASSES}
    for c in B.KERNEL_CLASSES:
        B.expdg_profile_enable(mesh.handle, c, False)
    out["profile"] = prof
    out["profile_ms_per_step"] = secs_p / args.steps * 1e3
    mesh.close()

    if not args.no_fp32:
        m32, q32, qp32, dt32, _ = make_case(B, inputs, torch, B.FP32_BULK)
        have = False
        for _ in range(args.warmup):
            m32.step(B.EPI3, dt32, q32, qp32, have, opts)
            have = True
        secs32, st32, have = timed_steps(B, torch, m32, q32, qp32, dt32, have, args.steps, opts)
        a32 = st32["rhs_calls"] + st32["jvps"]
        q32h = q32.cpu().numpy()
        out["fp32"] = dict(seconds=secs32, stats=st32, applications=a32,
                           value=m32.n * a32 / secs32,
                           l2_rel_diff_vs_fp64=float(np.linalg.norm(q32h - qh) /
                                                     np.linalg.norm(qh)))
        print(f"# fp32-bulk timed: {secs32 / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
        m32.close()
    return out


def run_cpu_baseline(args):
    import numpy as np

    import oracle
    from paper_2011_01316_amd import inputs

    w = WORKLOAD
    om = oracle.Mesh(oracle.EULER2D, w["nx"], w["p"], ny=w["ny"], x0=w["x0"], x1=w["x1"],
                     y0=w["y0"], y1=w["y1"])
    x, y = om.nodes()
    q = inputs.vortex(x, y, beta=w["beta"]).reshape(-1)
    c, dx = om.max_speed(q)
    dt = w["cr"] * dx / c
    kw = dict(tol=w["tol"], m_min=w["m_min"], m_max=w["m_max"])
    q, qp = om.step(oracle.EPI3, dt, q, None, **kw)  # EPI2 start, untimed
    apps, t0 = 0, time.perf_counter()
    nsteps = 0
    while nsteps < args.cpu_steps:
        q, qp, st = om.step(oracle.EPI3, dt, q, qp, stats=True, **kw)
        apps += st["rhs_calls"] + st["jvps"]
        nsteps += 1
        if time.perf_counter() - t0 > args.cpu_budget:
            break
    secs = time.perf_counter() - t0
    return dict(value=om.n * apps / secs, unit=UNIT, cores=oracle.num_threads(), kind="oracle",
                sample=f"{nsteps} EPI3 step(s) of the 64x64 p=4 vortex (409,600 DOF) after an "
                       f"untimed EPI2 start; {secs:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=25.0, help="seconds")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    g = run_gpu(args)
    f64 = g["fp64"]
    prof = g["profile"]
    gs = prof["gram_schmidt"]
    lin = prof["linear_operator"]

    def roof(p):
        if not p["launches"] or p["total_ms"] <= 0:
            return None
        achieved = p["bytes"] / (p["total_ms"] * 1e-3) / 1e9
        return dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    kernel=None, launches=p["launches"],
                    avg_launch_us=round(p["total_ms"] * 1e3 / p["launches"], 3),
                    avg_bytes_per_launch=round(p["bytes"] / p["launches"]))

    roofline = roof(gs)
    roofline["kernel"] = "cgs_kernel (Gram-Schmidt dot/update/norm passes)"
    lin_roof = roof(lin)
    lin_roof["kernel"] = "euler_op<4,double,true> (linear operator + augmented block)"
    ms = f64["seconds"] / args.steps * 1e3
    line = {
        "metric": METRIC,
        "value": round(f64["value"], 1),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2D Euler isentropic vortex, 64x64 quads, LGL p=4 (409,600 DOF), "
                        "Rusanov flux, EPI3, adaptive Krylov tol 1e-10 m<=64, Courant 5",
            "ndof": f64["ndof"], "dt": f64["dt"],
            "krylov_iters_per_step": f64["stats"]["krylov_iters"] / args.steps,
            "applications_per_step": f64["applications"] / args.steps,
            "substeps_per_step": f64["stats"]["substeps"] / args.steps,
        },
        "roofline": roofline,
        "linear_operator_roofline": lin_roof,
        "kernel_time_share": {k: round(v["total_ms"] / max(1e-9, g["profile_ms_per_step"] *
                                                           args.steps), 4)
                              for k, v in prof.items()},
        "instrumented_ms_per_step": round(g["profile_ms_per_step"], 4),
        "l2_rel_err_vs_exact_vortex": f64["l2_rel_err_vs_exact"],
    }
    if "fp32" in g:
        f32 = g["fp32"]
        line["fp32_bulk"] = dict(value=round(f32["value"], 1), unit=UNIT,
                                 ms_per_step=round(f32["seconds"] / args.steps * 1e3, 4),
                                 speedup_vs_fp64=round(f32["value"] / f64["value"], 3),
                                 l2_rel_diff_vs_fp64=f32["l2_rel_diff_vs_fp64"],
                                 krylov_iters_per_step=f32["stats"]["krylov_iters"] / args.steps)
    line["cpu_baseline"] = None if args.no_cpu_baseline else run_cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
