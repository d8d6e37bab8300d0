"""Restart lengths above the 32 Krylov rows that the register-cached first
Gram-Schmidt pass holds: with gmres_m = 48 and 64 that pass runs its
row-looping form, the second pass reads up to 63 basis rows, and the
reductions span up to 128 partial rows (row pairs against the new direction
and against w).  The Newton root does not depend on the restart length, so the states
after two implicit steps of the 8192-triangle P2 incline (the bench's
workload) agree with the gmres_m = 30 run to well within the Newton
tolerance, and the runs with the longer restarts take more than 32 GMRES
iterations per Newton system (cycles past 32 rows)."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def test_long_restarts_reach_the_same_newton_root(ctx):
    import torch
    from paper_2301_11238_amd import bsw
    pb = wl.config2(wl.REG1, 1e-3)
    mesh = bsw.Mesh(ctx, 2, pb.xy, pb.el2vert)
    disc = bsw.Disc(mesh, pb.P, bsw.BSW_FP64)
    cp = bsw.make_params(pb.params)
    W0 = disc.project_ic(pb.ic)
    dt = disc.cfl_dt(cp, W0, pb.cfl)
    out = {}
    for m in (30, 48, 64):
        W = W0.clone()
        st = disc.solve(cp, bsw.Options(t_end=2.5 * dt, dt=dt, max_steps=2, gmres_m=m), W)
        torch.cuda.synchronize()
        assert st["steps"] == 2 and st["capped"] == 0, (m, st)
        out[m] = (W.cpu().numpy(), st)
    ref = out[30][0]
    for m in (48, 64):
        W, st = out[m]
        rel = np.linalg.norm(W - ref) / np.linalg.norm(ref)
        assert rel <= 1e-9, (m, rel)
        assert st["gmres_total"] > 32 * st["newton_total"], (m, st["gmres_total"], st["newton_total"])
