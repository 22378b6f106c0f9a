"""Failure handling and checkpoint / resume on the GPU, through the C ABI.

  * host-driven NaN injection into the served mix: the request whose initial
    state holds a NaN ends FAILED with EXPDG_ENONFINITE, and every other
    request of the same mix (sharing its grouped launches) finishes bitwise
    equal to expdg_step on its own mesh;
  * a stand-alone step on a state with a NaN returns EXPDG_ENONFINITE and
    leaves the mesh usable: the next step on a valid state is bitwise the step
    of a fresh mesh;
  * checkpoint / resume: an EPI3 integration stopped after k steps, its state
    (q^n, q^{n-1}) written to disk and read back into a new mesh, continues
    bitwise equal to the uninterrupted run (2D Euler with walls and entropy
    viscosity, and 1D Burgers).
"""
import math

import numpy as np
import pytest
import torch

from paper_2011_01316_amd import binding as B
from paper_2011_01316_amd import inputs
from tests.test_gpu_serve import burgers_case, euler_case, serve_all, standalone

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_served_nan_request_fails_alone():
    print("served NaN injection", flush=True)
    cases = [burgers_case(40, 1, 0.1), euler_case(10, 2, 4.0, 6.0, 3.0),
             burgers_case(64, 3, 1.0), euler_case(12, 3, 5.0, 5.0, 5.0)]
    # a given step (no Courant rule on the NaN state): the NaN enters the
    # residual and the Krylov norms inside the grouped launches
    bad_req, bad_q0 = euler_case(10, 2, 2.0, 2.0, 2.0, dt=0.05, cfl=0.0)
    bad_q0 = bad_q0.copy()
    bad_q0[len(bad_q0) // 3] = float("nan")
    with B.Server(hbm_budget=1 << 30, max_active=8) as srv:
        good_ids = [srv.submit(r, q0) for r, q0 in cases[:2]]
        bad_id = srv.submit(bad_req, bad_q0)
        good_ids += [srv.submit(r, q0) for r, q0 in cases[2:]]
        done, failed, guard = {}, {}, 0
        while len(done) + len(failed) < len(cases) + 1:
            srv.tick(block=True)
            for rid in srv.finished():
                info = srv.poll(rid)
                if info["state"] == B.REQ_DONE:
                    done[rid] = srv.fetch(rid)
                else:
                    failed[rid] = info
            guard += 1
            assert guard < 200000
        assert list(failed) == [bad_id], failed
        assert failed[bad_id]["state"] == B.REQ_FAILED
        assert failed[bad_id]["error"] == B.ENONFINITE
        srv.cancel(bad_id)
        srv.sync()
        assert srv.stats()["arena_used"] == 0
    for rid, (r, q0) in zip(good_ids, cases):
        want, _ = standalone(r, q0)
        np.testing.assert_array_equal(done[rid], want)


def test_step_on_nan_state_then_recover():
    print("stand-alone NaN step", flush=True)
    kw = dict(x0=0.0, x1=10.0, y0=0.0, y1=10.0)
    opts = B.make_opts(1e-10, 10, 64)
    with B.Mesh(B.EULER2D, 8, 3, ny=8, **kw) as gm, B.Mesh(B.EULER2D, 8, 3, ny=8, **kw) as fresh:
        x, y = gm.nodes()
        q0 = inputs.vortex(x, y, beta=3.0).reshape(-1)
        bad = q0.copy()
        bad[17] = float("nan")
        qb = torch.tensor(bad, device=DEV)
        with pytest.raises(B.ExpdgError) as ei:
            gm.step(B.EPI2, 0.1, qb, None, False, opts)
        assert ei.value.code == B.ENONFINITE
        q1 = torch.tensor(q0, device=DEV)
        q2 = torch.tensor(q0, device=DEV)
        gm.step(B.EPI2, 0.1, q1, None, False, opts)
        fresh.step(B.EPI2, 0.1, q2, None, False, opts)
        torch.cuda.synchronize()
        assert torch.equal(q1, q2)


def make_mesh(kind):
    if kind == "euler_walls_ev":
        return B.Mesh(B.EULER2D, 12, 4, ny=6, x0=-5.0, x1=5.0, y0=0.0, y1=5.0, bc=B.BC_WALL_Y,
                      ev_ce=1.0, ev_cmax=0.1)
    return B.Mesh(B.BURGERS1D, 64, 3, x0=0.0, x1=2 * math.pi)


@pytest.mark.parametrize("kind", ["euler_walls_ev", "burgers"])
def test_checkpoint_resume_bitwise(kind, tmp_path):
    print(f"checkpoint / resume: {kind}", flush=True)
    opts = B.make_opts(1e-10, 10, 64)
    with make_mesh(kind) as m:
        x, y = m.nodes()
        q0 = (inputs.kelvin_helmholtz(x, y).reshape(-1) if kind != "burgers"
              else inputs.burgers_ic(x))
        dt = 4.0 * m.dx_min / m.max_speed(torch.tensor(q0, device=DEV))
        # uninterrupted: 6 EPI3 steps
        q = torch.tensor(q0, device=DEV)
        qp = torch.empty_like(q)
        m.integrate(B.EPI3, dt, 6, q, qp, False, opts)
        want = q.cpu().numpy()
        # 3 steps, checkpoint to disk
        q = torch.tensor(q0, device=DEV)
        qp = torch.empty_like(q)
        m.integrate(B.EPI3, dt, 3, q, qp, False, opts)
        np.save(tmp_path / "q.npy", q.cpu().numpy())
        np.save(tmp_path / "qp.npy", qp.cpu().numpy())
    # resume in a new mesh from the files, three more steps one call each
    with make_mesh(kind) as m2:
        q = torch.tensor(np.load(tmp_path / "q.npy"), device=DEV)
        qp = torch.tensor(np.load(tmp_path / "qp.npy"), device=DEV)
        for _ in range(3):
            m2.step(B.EPI3, dt, q, qp, True, opts)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(q.cpu().numpy(), want)
