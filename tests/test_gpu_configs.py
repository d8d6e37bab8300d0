"""GPU parity on the configured workloads, as configured or on a reduced mesh
of the same physics, against the FP64 oracle (FP64 bar: 1e-10 relative L2 on
h and h u at the volume points).

* The 1-D dam break (200 P1 elements, rho 1000, eta 1, sigma0 50, eps 1e-3,
  walls, CFL 0.2, 1 s: dt = 3.192754e-3, 314 steps) under regularisations 1
  and 2, in full.  Newton is capped at the paper's 10 iterations and most
  steps reach the cap (the first step needs about 20); the Krylov solves run
  to 1e-13 so the capped iterates are those of exact Newton, and the GPU and
  the oracle's exact sparse-LU Newton take the same iterates and cap the same
  steps.
* The same dam break with continuation on gamma (Sec. 6.3: gamma_0 = 100 to
  1e3 in three solves per step), the first 100 steps.
* The circular dam break physics (disk h = 2 | 0.5 of radius 2.5 m, P3,
  sigma0 30, eta 0.5, eps 1e-4, walls) on an 8 x 8 jittered mesh (128
  triangles): one time step solved to Newton convergence (about 22
  iterations with exact solves, beyond the paper's cap of 10; regs 1 and 2,
  Newton stalls under reg 3) and one Newton iteration (all three
  regularisations); the oracle side is its block-Jacobi GMRES Newton, itself
  pinned against its exact sparse-LU Newton.
* The dam break under regularisation 3, whose Newton stalls on every step:
  equal capped counts and mass conservation only.
"""
import math

import numpy as np
import pytest

import workloads as wl
from _gpu_util import Pair, have_gpu
from test_gpu_parity import rel_l2_h_hu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def exact_krylov(bsw, **kw):
    """GPU solve options whose Krylov solves run to 1e-13 (the Eisenstat-Walker
    forcing term pinned there), so Newton iterates match exact solves."""
    return bsw.Options(gmres_rtol=1e-13, forcing_max=1e-13, gmres_m=60, gmres_max_iters=5000,
                       newton_tol=1e-10, **kw)


@pytest.mark.parametrize("reg", [1, 2])
def test_c1_dam_break_in_full(ctx, reg):
    import oracle
    from paper_2301_11238_amd import bsw
    pb = wl.config1(reg)
    pr = Pair(ctx, 1, 1, pb.xy, pb.el2vert)
    W0 = pr.orc.project_ic(pb.ic)
    Wo, so = pr.orc.solve(pb.params, W0, oracle.SolveOptions(t_end=pb.t_end, cfl=pb.cfl))
    Wd = pr.dev(W0)
    sg = pr.disc.solve(bsw.make_params(pb.params), exact_krylov(bsw, t_end=pb.t_end, cfl=pb.cfl), Wd)
    dt_closed = 0.2 * 0.05 / math.sqrt(9.81)
    assert so["steps"] == sg["steps"] == 314
    assert abs(sg["dt"] - dt_closed) <= 1e-13 * dt_closed and abs(so["dt"] - dt_closed) <= 1e-13 * dt_closed
    assert sg["capped"] == so["capped"] and so["capped"] > 100
    eh, eq = rel_l2_h_hu(pr.orc, pr.host(Wd), Wo)
    assert eh <= 1e-10 and eq <= 1e-10, (eh, eq)
    assert sg["max_mass_drift"] < 1e-12


def test_c1_dam_break_with_continuation(ctx):
    import oracle
    from paper_2301_11238_amd import bsw
    pb = wl.config1(1)
    pr = Pair(ctx, 1, 1, pb.xy, pb.el2vert)
    W0 = pr.orc.project_ic(pb.ic)
    n = 100
    Wo, so = pr.orc.solve(pb.params, W0, oracle.SolveOptions(t_end=pb.t_end, cfl=pb.cfl, max_steps=n,
                                                             cont_steps=3, cont_gamma0=100.0))
    Wd = pr.dev(W0)
    sg = pr.disc.solve(bsw.make_params(pb.params),
                       exact_krylov(bsw, t_end=pb.t_end, cfl=pb.cfl, max_steps=n, cont_steps=3, cont_gamma0=100.0),
                       Wd)
    assert so["steps"] == sg["steps"] == n
    assert sg["capped"] == so["capped"]
    assert sg["newton_total"] == so["newton_total"]
    eh, eq = rel_l2_h_hu(pr.orc, pr.host(Wd), Wo)
    assert eh <= 1e-10 and eq <= 1e-10, (eh, eq)


@pytest.mark.parametrize("reg", [1, 2, 3])
def test_c3_physics_on_a_reduced_mesh(ctx, reg):
    import oracle
    from paper_2301_11238_amd import bsw
    pb = wl.config3(reg, N=8)
    pr = Pair(ctx, 2, 3, pb.xy, pb.el2vert)
    W0 = pr.orc.project_ic(pb.ic)
    dt = pr.orc.cfl_dt(pb.params, W0, pb.cfl)
    b = pr.orc.step_begin(pb.params, W0, dt)
    cp = bsw.make_params(pb.params)
    # the converged step meets the FP64 bar; a single Newton iteration is an
    # unconverged iterate that carries its Krylov solve's error (the relative
    # tolerance 1e-13 times the conditioning of the step's Jacobian, which at
    # gamma = 1e4 and reg 3 (rest viscosity sigma0 gamma = 3e5 against eta =
    # 0.5) reaches about 1e-8), so it is held to 1e-7.  Under reg 3 Newton
    # stalls on this step (40 iterations with exact sparse-LU solves do not
    # reach the tolerance; whether the Krylov variant does depends on
    # rounding), so only the single iteration is compared there.
    cases = ((40, 1e-10), (1, 1e-7)) if reg != 3 else ((1, 1e-7),)
    for max_newton, bar in cases:
        Wo, so = pr.orc.newton_step(pb.params, W0, b, dt, oracle.SolveOptions(
            max_newton=max_newton, gmres_max_restarts=200, gmres_rtol=1e-13), linear="gmres")
        Wd = pr.dev(W0)
        sg = pr.disc.solve(cp, exact_krylov(bsw, t_end=10 * dt, dt=dt, max_steps=1, max_newton=max_newton), Wd)
        assert sg["steps"] == 1
        if max_newton == 40:
            assert so["converged"] and sg["capped"] == 0, (so, sg)
            assert abs(sg["newton_total"] - so["newton"]) <= 1, (sg["newton_total"], so["newton"])
        eh, eq = rel_l2_h_hu(pr.orc, pr.host(Wd), Wo)
        assert eh <= bar and eq <= bar, (max_newton, eh, eq)
        assert sg["max_mass_drift"] < 1e-12


def test_c1_dam_break_reg3_caps_like_the_oracle(ctx):
    """Regularisation 3 at gamma = 1e3 (slope 2 sigma0 gamma = 1e5 at rest
    against eta = 1): Newton stalls on every step, exact solves included
    (its line search stops decreasing ||R||), so the states after a capped
    step depend on the iteration path and are not compared; both sides cap
    every one of the first 20 steps.  The oracle's exact solves conserve mass
    to rounding; on the GPU the block-Jacobi GMRES(60) systems of this stiff
    viscous limit stagnate near the 5000-iteration cap (4000-5000 iterations
    per Newton system), so its mass drift is that of the capped Krylov
    solves, held to 1e-5."""
    import oracle
    from paper_2301_11238_amd import bsw
    pb = wl.config1(3)
    pr = Pair(ctx, 1, 1, pb.xy, pb.el2vert)
    W0 = pr.orc.project_ic(pb.ic)
    n = 20
    _, so = pr.orc.solve(pb.params, W0, oracle.SolveOptions(t_end=pb.t_end, cfl=pb.cfl, max_steps=n))
    Wd = pr.dev(W0)
    sg = pr.disc.solve(bsw.make_params(pb.params), exact_krylov(bsw, t_end=pb.t_end, cfl=pb.cfl, max_steps=n), Wd)
    assert so["capped"] == sg["capped"] == n
    assert so["max_mass_drift"] < 1e-12 and sg["max_mass_drift"] < 1e-5



def _c2_golden():
    import json
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_first_steps.json")
    with open(p) as f:
        return json.load(f)["runs"]


def _samples_close(pr, W, ref, bar):
    vals = pr.orc.eval_points(W)
    t, md = pr.orc.ref_tables(), pr.orc.mesh_data()
    w = t["qw"][None, :] * md["detJ"][:, None]
    h = vals[..., 0]
    hu = vals[..., :1] * vals[..., 1:3]
    idx = np.asarray(ref["elements"])
    hs, hus = np.asarray(ref["h"]), np.asarray(ref["hu"])
    eh = np.linalg.norm(h[idx] - hs) / np.linalg.norm(hs)
    eq = np.linalg.norm(hu[idx] - hus) / np.linalg.norm(hus)
    assert eh <= bar and eq <= bar, (eh, eq)
    nh, nq = np.sqrt((w * h ** 2).sum()), np.sqrt((w[..., None] * hu ** 2).sum())
    assert abs(nh - ref["norm_h"]) <= bar * ref["norm_h"] and abs(nq - ref["norm_hu"]) <= bar * ref["norm_hu"]


@pytest.mark.parametrize("run", range(9))
def test_c2_incline_first_steps(ctx, run):
    """The nine incline runs (8192 triangles, P2, regs 1-3 x eps 1e-2, 1e-3,
    1e-4) against stored oracle results (tests/golden/c2_first_steps.json,
    written by make_c2_golden.py from the oracle alone).  Runs whose first two
    steps converge within the Newton cap (eps 1e-2 and 1e-3 under regs 1-2,
    eps 1e-2 under reg 3): the same step, Newton counts within one, the mass
    to rounding, and h and h u at the volume points of 64 sampled elements
    and the mesh-wide L2 norms within 1e-10.  The other runs reach the cap of
    10 in the oracle, whose Krylov solves are then truncated at its restart
    cap too (the GPU's GMRES(60) needs up to 5000 iterations per system
    there), so their capped steps are no reference for exact Newton; for
    those the first Newton iterate of the first step, its linear solve run
    to 1e-13 on both sides, is compared within 1e-7 (the Krylov tolerance
    times the conditioning of these systems at gamma = 1e3-1e4), with the
    mass to rounding."""
    from paper_2301_11238_amd import bsw
    g = _c2_golden()[run]
    pb = wl.config2(g["reg"], g["eps"])
    assert abs(pb.params.sigma0 - g["sigma0"]) < 1e-12
    pr = Pair(ctx, 2, pb.P, pb.xy, pb.el2vert)
    W0 = pr.orc.project_ic(pb.ic)
    cp = bsw.make_params(pb.params)
    Wd = pr.dev(W0)
    dt = pr.disc.cfl_dt(cp, Wd, pb.cfl)
    assert abs(dt - g["dt"]) <= 1e-13 * g["dt"]
    if "first_newton" in g:
        ref = g["first_newton"]
        o = exact_krylov(bsw, t_end=10 * dt, dt=dt, max_steps=1, max_newton=1)
        o.gmres_max_iters = 20000
        st = pr.disc.solve(cp, o, Wd)
        assert st["newton_total"] == 1
        assert abs(st["mass_end"] - ref["mass"]) <= 1e-12 * g["mass0"]
        _samples_close(pr, pr.host(Wd), ref, 1e-7)
        return
    for k, gs in enumerate(g["steps"]):
        st = pr.disc.solve(cp, exact_krylov(bsw, t_end=10 * dt, dt=dt, max_steps=1), Wd)
        assert st["capped"] == gs["capped"] == 0, (k, st["capped"], gs)
        assert abs(st["newton_total"] - gs["newton"]) <= 1, (k, st["newton_total"], gs)
        assert abs(st["mass_end"] - gs["mass"]) <= 1e-12 * g["mass0"]
    _samples_close(pr, pr.host(Wd), g, 1e-10)
