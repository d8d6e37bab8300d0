"""Writes c2_first_steps.json: the first two backward-Euler steps of the nine
runs of the 2-D incline configuration (64x64 jittered -> 8192 triangles, P2,
regularisations 1-3 x eps 1e-2, 1e-3, 1e-4), computed by the FP64 oracle
alone (its block-Jacobi GMRES Newton, pinned against its exact sparse-LU
Newton in tests/test_oracle_pins.py).  Per run and step: the Newton count and
whether the step reached the 10-iteration cap, the mass; after two steps: h
and h u at the volume points of 64 seeded elements and the weighted L2 norms
of h and h u over the mesh.

Where a step reaches the Newton cap, its Krylov solves are truncated too (at
40 restarts of GMRES(30)), so the steps are not a reference for exact Newton;
for those runs the script also stores the first Newton iterate of the first
step with its linear solve run to 1e-13 (up to 400 restarts), or, where that
GMRES reaches its cap, solved exactly by the sparse LU path (about 13 minutes
per system here): the same samples and norms under "first_newton", with the
linear solver used.  Run from the repository root:
    python tests/golden/make_c2_golden.py            (everything)
    python tests/golden/make_c2_golden.py --update   (only missing first_newton entries)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

STEPS = 2
N_SAMPLE = 64
FN_RESTARTS = 400  # GMRES(30) restarts for the first-Newton references


def sample_elements(n_el):
    return np.sort(wl.rng_for(2, 99).choice(n_el, N_SAMPLE, replace=False))


def samples(orc, W):
    vals = orc.eval_points(W)
    t, md = orc.ref_tables(), orc.mesh_data()
    w = t["qw"][None, :] * md["detJ"][:, None]
    h = vals[..., 0]
    hu = vals[..., :1] * vals[..., 1:3]
    idx = sample_elements(orc.n_el)
    return {"norm_h": float(np.sqrt((w * h ** 2).sum())), "norm_hu": float(np.sqrt((w[..., None] * hu ** 2).sum())),
            "elements": idx.tolist(), "h": h[idx].tolist(), "hu": hu[idx].tolist()}


def first_newton(reg, eps):
    pb = wl.config2(reg, eps)
    orc = oracle.Oracle(2, pb.P, pb.xy, pb.el2vert)
    W0 = orc.project_ic(pb.ic)
    dt = orc.cfl_dt(pb.params, W0, pb.cfl)
    b = orc.step_begin(pb.params, W0, dt)
    o = oracle.SolveOptions(max_newton=1, gmres_max_restarts=FN_RESTARTS, gmres_rtol=1e-13, newton_tol=1e-10)
    W, st = orc.newton_step(pb.params, W0, b, dt, o, linear="gmres")
    out = {"linear": "gmres", "gmres": int(st["gmres"])}
    if st["gmres"] >= FN_RESTARTS * 30:
        W, st = orc.newton_step(pb.params, W0, b, dt, o, linear="direct")
        out["linear"] = "direct"
    out["mass"] = float(orc.diagnostics(pb.params, W)["mass"])
    out.update(samples(orc, W))
    return out


def run(reg, eps):
    pb = wl.config2(reg, eps)
    orc = oracle.Oracle(2, pb.P, pb.xy, pb.el2vert)
    W = orc.project_ic(pb.ic)
    dt = orc.cfl_dt(pb.params, W, pb.cfl)
    o = oracle.SolveOptions(t_end=10 * dt, dt_override=dt, max_steps=1, gmres_max_restarts=40,
                            gmres_rtol=1e-13, newton_tol=1e-10)
    steps = []
    for _ in range(STEPS):
        W, st = orc.solve(pb.params, W, o, linear="gmres")
        steps.append({"newton": int(st["newton_total"]), "capped": int(st["capped"]),
                      "gmres": int(st["gmres_total"]), "mass": float(st["mass_end"])})
    out = {"reg": reg, "eps": eps, "sigma0": pb.params.sigma0, "dt": dt, "steps": steps,
           "mass0": float(orc.diagnostics(pb.params, orc.project_ic(pb.ic))["mass"])}
    out.update(samples(orc, W))
    return out


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_first_steps.json")
    if "--update" in sys.argv:
        with open(path) as f:
            out = json.load(f)
    else:
        out = {"config": "2-D incline, 64x64 jittered (seed 2) -> 8192 triangles, P2, 10 % slope, mound, walls",
               "steps": STEPS, "runs": []}
        for reg in (1, 2, 3):
            for eps in wl.C2_EPS:
                t0 = time.time()
                out["runs"].append(run(reg, eps))
                r = out["runs"][-1]
                print(f"reg {reg} eps {eps}: {[s['newton'] for s in r['steps']]} newton, "
                      f"{[s['capped'] for s in r['steps']]} capped, {time.time() - t0:.0f} s", flush=True)
    for r in out["runs"]:
        fn = r.get("first_newton")
        stale = fn is not None and fn.get("linear") != "direct" and fn["gmres"] >= FN_RESTARTS * 30
        if any(s["capped"] for s in r["steps"]) and (fn is None or stale):
            t0 = time.time()
            r["first_newton"] = first_newton(r["reg"], r["eps"])
            print(f"reg {r['reg']} eps {r['eps']}: first Newton iterate, {r['first_newton']['gmres']} GMRES "
                  f"iterations, solved by {r['first_newton']['linear']}, {time.time() - t0:.0f} s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
