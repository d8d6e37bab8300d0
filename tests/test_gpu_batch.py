"""Batched solves through the solve server (continuous batching).

Served results are checked against the oracle (FP64: 1e-10, FP32: 1e-5
relative L2 on h and h u), against the single-solve path, and for identity:
each solve gives bitwise the same state alone and in a mix of solves of other
sizes, orders and parameters, admitted together or one after another under a
memory budget."""
import math

import numpy as np
import pytest

import workloads as wl
from _gpu_util import have_gpu, mesh_for
from test_gpu_parity import rel_l2_h_hu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

MOUND = wl.IC(kind=wl.IC_MOUND, a=1.0, b=0.5, x0=10.0, y0=10.0, d=4.0)
DISK = wl.IC(kind=wl.IC_DISK, a=2.0, b=0.5, x0=10.0, y0=10.0, r=2.5)
SLOPE = math.atan(0.1)

# (name, n, P, reg, sigma0, eta, eps, alpha, ic, t_end)
MIX = [
    ("x_p2_reg1", 8, 2, 1, 40.0, 1.0, 1e-2, SLOPE, MOUND, 0.1),
    ("a_p2_reg3", 5, 2, 3, 20.0, 0.5, 1e-2, 0.0, DISK, 0.1),
    ("b_p2_reg2", 11, 2, 2, 60.0, 2.0, 1e-2, SLOPE, MOUND, 0.05),
    ("c_p2_reg1", 6, 2, 1, 100.0, 1.0, 1e-3, 0.0, DISK, 0.08),
    ("d_p3_reg1", 6, 3, 1, 30.0, 0.5, 1e-2, 0.0, DISK, 0.06),
    ("e_p1_reg2", 9, 1, 2, 50.0, 1.0, 1e-2, SLOPE, MOUND, 0.1),
    ("f_p3_reg3", 4, 3, 3, 10.0, 0.3, 1e-2, SLOPE, MOUND, 0.08),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def params(case):
    name, n, P, reg, s0, eta, eps, alpha, ic, t_end = case
    return wl.Params(g=9.81, rho=1000.0, alpha=alpha, eta=eta, sigma0=s0, gamma=1 / eps, beta=1 / eps, reg=reg)


def submit(srv, case, precision):
    from paper_2301_11238_amd import bsw
    name, n, P, reg, s0, eta, eps, alpha, ic, t_end = case
    xy, e2v = mesh_for(2, n)
    return srv.submit(xy, e2v, P, precision, bsw.make_params(params(case)), ic=ic,
                      opts=bsw.Options(t_end=t_end, cfl=0.2))


def run_alone(ctx, case, precision):
    from paper_2301_11238_amd import bsw
    srv = bsw.Server(ctx, 1 << 30, 4)
    try:
        t = submit(srv, case, precision)
        assert srv.wait(t, 300.0) == bsw.BSW_REQ_DONE
        return srv.fetch(t)
    finally:
        srv.close()


@pytest.mark.parametrize("case", [MIX[0], MIX[4], MIX[5]], ids=lambda c: c[0])
def test_served_solve_matches_oracle(ctx, case):
    import oracle
    from paper_2301_11238_amd import bsw
    name, n, P, reg, s0, eta, eps, alpha, ic, t_end = case
    xy, e2v = mesh_for(2, n)
    orc = oracle.Oracle(2, P, xy, e2v)
    Wo, so = orc.solve(params(case), orc.project_ic(ic), oracle.SolveOptions(t_end=t_end, cfl=0.2))
    W, st = run_alone(ctx, case, bsw.BSW_FP64)
    assert so["capped"] == 0 and st["capped"] == 0, (so, st)
    assert st["steps"] == so["steps"]
    eh, eq = rel_l2_h_hu(orc, W.astype(np.float64), Wo)
    assert eh <= 1e-10 and eq <= 1e-10, (eh, eq)
    assert st["max_mass_drift"] <= 1e-11
    assert st["queue_seconds"] >= 0.0 and st["seconds"] > 0.0


@pytest.mark.parametrize("case", [MIX[0], MIX[4]], ids=lambda c: c[0])
def test_served_fp32_matches_oracle(ctx, case):
    import oracle
    from paper_2301_11238_amd import bsw
    name, n, P, reg, s0, eta, eps, alpha, ic, t_end = case
    xy, e2v = mesh_for(2, n)
    orc = oracle.Oracle(2, P, xy, e2v)
    Wo, so = orc.solve(params(case), orc.project_ic(ic), oracle.SolveOptions(t_end=t_end, cfl=0.2))
    W, st = run_alone(ctx, case, bsw.BSW_FP32)
    assert st["capped"] == 0 and st["steps"] == so["steps"], st
    eh, eq = rel_l2_h_hu(orc, W.astype(np.float64), Wo)
    assert eh <= 1e-5 and eq <= 1e-5, (eh, eq)


def test_served_matches_single_solve_path(ctx):
    from paper_2301_11238_amd import bsw
    import torch
    case = MIX[1]
    name, n, P, reg, s0, eta, eps, alpha, ic, t_end = case
    xy, e2v = mesh_for(2, n)
    mesh = bsw.Mesh(ctx, 2, xy, e2v)
    disc = bsw.Disc(mesh, P, bsw.BSW_FP64)
    Wd = disc.project_ic(ic)
    s1 = disc.solve(bsw.make_params(params(case)), bsw.Options(t_end=t_end, cfl=0.2), Wd)
    torch.cuda.synchronize()
    W1 = Wd.cpu().numpy()
    W2, s2 = run_alone(ctx, case, bsw.BSW_FP64)
    assert s1["steps"] == s2["steps"] and s1["dt"] == s2["dt"]
    err = np.abs(W2 - W1).max() / np.abs(W1).max()
    assert err <= 1e-10, err


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_result_is_the_same_alone_and_in_the_mix(ctx, precision):
    from paper_2301_11238_amd import bsw
    alone = {c[0]: run_alone(ctx, c, precision) for c in MIX}
    srv = bsw.Server(ctx, 1 << 31, 64)
    try:
        tickets = {c[0]: submit(srv, c, precision) for c in MIX}
        mixed = {}
        for name, t in tickets.items():
            assert srv.wait(t, 300.0) == bsw.BSW_REQ_DONE
            mixed[name] = srv.fetch(t)
        info = srv.info()
    finally:
        srv.close()
    assert info["peak_resident"] >= 2
    for name in tickets:
        Wa, sa = alone[name]
        Wm, sm = mixed[name]
        assert np.array_equal(Wa, Wm), name
        for k in ("steps", "newton_total", "gmres_total", "capped", "mass_end", "max_mass_drift"):
            assert sa[k] == sm[k], (name, k, sa[k], sm[k])


def test_admission_by_footprint_and_slots(ctx):
    from paper_2301_11238_amd import bsw
    # FIFO order: 128, 50, 242, 72 triangles; the budget holds the largest
    # alone or the first two together, never three of them
    cases = [MIX[0], MIX[1], MIX[2], MIX[3]]
    fps = [bsw.request_footprint(c[1] * c[1] * 2, c[2], bsw.BSW_FP64) for c in cases]
    assert fps[0] + fps[1] < max(fps) < fps[0] + fps[1] + fps[3]
    for budget, slots, peak in ((max(fps) + 1, 8, 2), (1 << 31, 1, 1)):
        srv = bsw.Server(ctx, budget, slots)
        try:
            tickets = [submit(srv, c, bsw.BSW_FP64) for c in cases]
            res = []
            for t in tickets:
                assert srv.wait(t, 300.0) == bsw.BSW_REQ_DONE
                res.append(srv.fetch(t))
            info = srv.info()
        finally:
            srv.close()
        assert info["peak_resident"] == peak, (budget, slots, info)
        assert info["completed"] == len(cases) and info["bytes_in_use"] == 0
        for c, (W, st) in zip(cases, res):
            Wa, _ = run_alone(ctx, c, bsw.BSW_FP64)
            assert np.array_equal(W, Wa), c[0]


def test_cancel_and_invalid_requests(ctx):
    from paper_2301_11238_amd import bsw
    srv = bsw.Server(ctx, 1 << 30, 1)
    try:
        long_case = ("long", 8, 2, 1, 40.0, 1.0, 1e-2, SLOPE, MOUND, 5.0)
        t0 = submit(srv, long_case, bsw.BSW_FP64)
        t1 = submit(srv, MIX[0], bsw.BSW_FP64)  # queued behind t0 (one slot)
        srv.cancel(t1)
        srv.cancel(t0)
        assert srv.wait(t1, 60.0) == bsw.BSW_REQ_CANCELLED
        assert srv.wait(t0, 60.0) == bsw.BSW_REQ_CANCELLED
        with pytest.raises(bsw.BswError):
            srv.fetch(t0)
        xy, e2v = mesh_for(2, 4)
        bad = bsw.make_params(params(MIX[0]))
        bad.reg = 7
        with pytest.raises(bsw.BswError):
            srv.submit(xy, e2v, 2, bsw.BSW_FP64, bad, ic=MOUND, opts=bsw.Options(t_end=0.1))
        with pytest.raises(bsw.BswError):
            srv.submit(xy, e2v, 4, bsw.BSW_FP64, bsw.make_params(params(MIX[0])), ic=MOUND)
        # a request larger than the whole budget is refused at submit
        small = bsw.Server(ctx, 1 << 16, 1)
        try:
            with pytest.raises(bsw.BswError):
                small.submit(xy, e2v, 2, bsw.BSW_FP64, bsw.make_params(params(MIX[0])), ic=MOUND)
        finally:
            small.close()
        # the server still serves after the errors
        t2 = submit(srv, MIX[5], bsw.BSW_FP64)
        assert srv.wait(t2, 300.0) == bsw.BSW_REQ_DONE
        W, st = srv.fetch(t2)
        assert st["steps"] > 0 and np.isfinite(W).all()
    finally:
        srv.close()


def test_tile_shapes_give_the_same_bits_and_autotuner_picks_one(ctx):
    """The element pass in its three variants (triangles: occupancy targets of
    1, 2 and 3 waves per SIMD for the same tile code) gives the same state bit
    for bit; with the autotuner on, every variant is timed on live launches
    and one is kept."""
    from paper_2301_11238_amd import bsw
    for case in (MIX[4], MIX[0], MIX[5]):  # P3, P2, P1
        out = []
        try:
            for pol in (0, 1, 2, -1):
                bsw.tile_policy(pol)
                out.append(run_alone(ctx, case, bsw.BSW_FP64))
        finally:
            bsw.tile_policy(-1)
        for W, st in out[1:]:
            assert np.array_equal(W, out[0][0]), case[0]
            assert st["newton_total"] == out[0][1]["newton_total"]
    rows = [r for r in bsw.tile_table() if r["dim"] == 2 and r["P"] == 3 and r["bytes"] == 8]
    assert rows and any(r["mode"] == 1 for r in rows)
    for r in rows:
        if r["variant"] >= 0:
            assert r["variant"] in (0, 1, 2)
            best = min(v for v in r["best_us"].values() if v > 0)
            assert r["best_us"][r["variant"]] == best
    assert any(r["variant"] >= 0 for r in rows if r["mode"] == 1)
    with pytest.raises(bsw.BswError):
        bsw.tile_policy(3)
