"""Open-loop load driver for the solve server (served workload).

The request mix comes from :func:`inputs.served_mix`: Poisson arrivals, a
50/50 mix of Burgers solves (K log-uniform, p in 1..4, u0 = 0.5 + sin(x +
theta), dt = 1e-2) and Euler vortex solves (n x n log-uniform, p in 2..4,
seeded centre and strength, Courant number 5 applied by the server to the
wave speed of q0), each a fixed number of EPI3 steps in FP64.

:func:`prepare` turns the mix into server requests with their initial
states; :func:`run` submits every request at its arrival time on the server
clock, ticks the server, and records for each solve the latency from its
arrival to the moment the server saw it finish.  Everything here is
argument marshalling and bookkeeping: the solves run in the library.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B
from . import inputs

BURGERS_DOMAIN = (0.0, 2.0 * math.pi)
EULER_DOMAIN = (0.0, 10.0, 0.0, 10.0)


def node_coords(nx, ny, p, x0, x1, y0, y1, dim):
    """Node coordinates in the library's layout (e = ey nx + ex, n = j (p+1) + i)."""
    xi, _, _ = B.expdg_lgl(p)
    hx = (x1 - x0) / nx
    if dim == 1:
        return (x0 + np.arange(nx)[:, None] * hx + 0.5 * (xi[None, :] + 1.0) * hx).ravel(), None
    hy = (y1 - y0) / ny
    e = np.arange(nx * ny)
    ex, ey = e % nx, e // nx
    nn = np.arange((p + 1) ** 2)
    i, j = nn % (p + 1), nn // (p + 1)
    x = x0 + ex[:, None] * hx + 0.5 * (xi[i][None, :] + 1.0) * hx
    y = y0 + ey[:, None] * hy + 0.5 * (xi[j][None, :] + 1.0) * hy
    return x.ravel(), y.ravel()


def prepare(mix, tol=1e-10, m_min=10, m_max=64, check_every=1, iop=0):
    """Server requests and initial states for a request mix (iop: the
    orthogonalization window of every request, 0 = full).

    Returns a list of dicts: arrival (s), req (binding.Request), q0 (host
    float64), ndof, equation name, size and degree.
    """
    items = []
    for r in mix:
        p = r["p"]
        if r["equation"] == "burgers1d":
            x, _ = node_coords(r["nx"], 1, p, *BURGERS_DOMAIN, 0.0, 1.0, 1)
            q0 = inputs.burgers_ic(x, r["theta"])
            req = B.make_request(B.BURGERS1D, r["nx"], p, scheme=B.EPI3, nsteps=r["steps"],
                                 dt=r["dt"], tol=tol, m_min=m_min, m_max=m_max,
                                 check_every=check_every, x0=BURGERS_DOMAIN[0],
                                 x1=BURGERS_DOMAIN[1], iop=iop)
        else:
            x, y = node_coords(r["nx"], r["ny"], p, *EULER_DOMAIN, 2)
            q0 = inputs.vortex(x, y, beta=r["beta"], xc=r["xc"], yc=r["yc"]).ravel()
            req = B.make_request(B.EULER2D, r["nx"], p, ny=r["ny"], scheme=B.EPI3,
                                 nsteps=r["steps"], dt=0.0, cfl=r["cr"], tol=tol, m_min=m_min,
                                 m_max=m_max, check_every=check_every, x0=EULER_DOMAIN[0],
                                 x1=EULER_DOMAIN[1], y0=EULER_DOMAIN[2], y1=EULER_DOMAIN[3],
                                 iop=iop)
        items.append(dict(arrival=r["arrival"], req=req, q0=np.ascontiguousarray(q0),
                          ndof=int(q0.size), equation=r["equation"], nx=r["nx"], p=p))
    return items


def percentile(v, q):
    v = np.sort(np.asarray(v, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))


def run(server, items, keep_states=False, progress=None, time_limit=None):
    """Serves items open-loop; returns latency and throughput figures.

    Each item is submitted once the server clock passes its arrival time
    (relative to the start of the run).  Finished states are fetched (kept if
    keep_states) or released at once, so their memory returns to the budget.
    progress(n_done, n_total) is called whenever solves finish.  Latencies and
    solves/s count the solves that completed (DONE); failed solves are listed
    with their status and their work still counts in the DOF-stage rate.
    """
    n = len(items)
    if n == 0:
        raise ValueError("no requests to serve")
    order = sorted(range(n), key=lambda k: items[k]["arrival"])
    t0 = server.clock()
    nxt = 0
    rid_of = {}
    item_of = {}
    lat = np.full(n, np.nan)
    wait = np.full(n, np.nan)
    good = np.zeros(n, dtype=bool)
    work = 0.0
    states = {}
    failed = []
    done = 0
    while done < n:
        now = server.clock() - t0
        if time_limit is not None and now > time_limit:
            break
        while nxt < n and items[order[nxt]]["arrival"] <= now:
            k = order[nxt]
            rid = server.submit(items[k]["req"], items[k]["q0"])
            rid_of[k] = rid
            item_of[rid] = k
            nxt += 1
        if server.stats()["active"] == 0 and server.stats()["queued"] == 0 and nxt < n:
            # idle until the next arrival
            time.sleep(max(0.0, items[order[nxt]]["arrival"] - (server.clock() - t0)))
            continue
        server.tick(block=True)
        fin = server.finished()
        for rid in fin:
            k = item_of[rid]
            info = server.poll(rid)
            arr = t0 + items[k]["arrival"]
            lat[k] = info["t_done"] - arr
            wait[k] = info["t_admit"] - arr
            st = info["stats"]
            work += items[k]["ndof"] * (st["rhs_calls"] + st["jvps"])
            if info["state"] == B.REQ_DONE:
                good[k] = True
                if keep_states:
                    states[k] = server.fetch(rid)
                else:
                    server.cancel(rid)
            else:
                failed.append((k, info["error"]))
                server.cancel(rid)
            done += 1
        if fin and progress:
            progress(done, n)
    t_end = server.clock() - t0
    first = min(it["arrival"] for it in items)
    ok = good
    return dict(
        requests=n, completed=int(ok.sum()), failed=failed, finished=int((~np.isnan(lat)).sum()),
        makespan_s=t_end - first,
        solves_per_s=float(ok.sum()) / max(t_end - first, 1e-12),
        dof_stage_updates_per_s=work / max(t_end - first, 1e-12),
        latency_p50_s=percentile(lat[ok], 50), latency_p99_s=percentile(lat[ok], 99),
        latency_max_s=float(np.max(lat[ok])) if ok.any() else float("nan"),
        admission_wait_p50_s=percentile(wait[ok], 50),
        admission_wait_p99_s=percentile(wait[ok], 99),
        latencies=lat, states=states)
