"""Benchmark of the regularised-Bingham shallow-water DG hot path on one MI355X.

Headline workload: the circular dam-break mesh, 256x256 jittered squares split
into 131,072 triangles on a 20 m x 20 m box, DG P3 (10 modes, 12-point rule,
4 points per edge), 7 fields, 9,175,040 DOFs, FP64, walls, yield stress 30 Pa,
plastic viscosity 0.5 Pa s, regularisation 1 with eps = 1e-4.  Inputs are
synthetic and seeded and sit in HBM before any timed region starts.

value = DG DOF-updates/s: the degrees of freedom of one operator apply (the
residual of Eq. WeakForm7: volume fluxes, HLL and central face fluxes,
regularised Bingham stress and source) divided by the median duration of one
apply, with the state, b_old and residual buffers cycled through >= 2 GiB of
independent sets so every apply reads from HBM (HIP events on the library's
stream).  The Jacobian-apply rate is reported beside it.

One step (--steps, --warmup) = one pass over the whole hot path on the same
mesh and state: b_old, the residual, the linearisation (traces, diagonal
blocks, their Schur-complement factors), one restarted-GMRES cycle of 30
block-Jacobi-preconditioned matrix-free Jacobian applies, the Newton update
with its line search and the FP64 reductions: one Newton iteration of one
backward-Euler time step.  ms_per_step is its time.

Other blocks: the same applies in FP32 with their error against FP64; the
2-D incline configuration (8192 triangles, P2) solved to Newton convergence,
and its first two steps against the FP64 oracle's stored result (FP64 and
FP32-mixed, scored in the CPU-baseline leg);
the batched FP32 solve server against plain one-at-a-time FP64 solves (solves/s
and p50/p99 time-to-solution under the same arrivals); the stated request
stream (Poisson arrivals at 200/s, 2 % 999,698-triangle incline runs,
admission by device-memory footprint); an ensemble of dam-break instances of
mixed size, order and parameters through the batched server; the FP64 CPU
oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
# HBM bytes of one operator apply from the rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes (KiB per dispatch), scaled by the same counters on a plain device
# copy of known size; None until the counters are taken on the current kernel.
TRAFFIC_BYTES = {"operator": 216961024.0}  # FETCH 70098 KiB x 2 + WRITE 71680 KiB, current kernel


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed hot-path passes (Newton iterations)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 applies")
    ap.add_argument("--no-c2", action="store_true", help="skip the incline solve")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving comparison, the request stream and the ensemble")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-steps", type=int, default=3,
                    help="time steps per served request (each draw's horizon is cut to this many steps)")
    ap.add_argument("--stream-seconds", type=float, default=10.0,
                    help="length of the Poisson arrival window of the request stream (the stated stream is 60 s)")
    ap.add_argument("--stream-rate", type=float, default=200.0)
    ap.add_argument("--ensemble", type=int, default=48, help="dam-break instances of the ensemble leg (512 stated)")
    ap.add_argument("--ensemble-steps", type=int, default=3)
    ap.add_argument("--tile-policy", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="element-pass variant: -1 autotune (default), 0/1/2 force one (triangles: occupancy "
                         "target of 1/2/3 waves per SIMD)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="no solves: a 256 MiB device copy (counter calibration) and 20 launches of each hot "
                         "kernel on the workload's mesh, for rocprofv3 passes")
    ap.add_argument("--workload", choices=["c3", "c2"], default="c3",
                    help="mesh of --kernels-only: c3 (131072 triangles, P3) or c2 (8192 triangles, P2)")
    return ap.parse_args()


_T0 = time.perf_counter()


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _np(P, dim=2):
    return P + 1 if dim == 1 else (P + 1) * (P + 2) // 2


def bytes_per_element(dim, P, w):
    """Algorithmic HBM bytes of one operator apply per element: read W (n_f N_p),
    b_old (N_v N_p), write R (n_f N_p), the affine metric, normals and face
    lengths (dim^2 + 1 + (dim+1)(dim+1) reals) and the neighbour codes."""
    nf, nv, npm, nfc = 1 + dim + dim * dim, 1 + dim, _np(P, dim), dim + 1
    geo = dim * dim + 1 + nfc * dim + nfc
    return w * (2 * nf * npm + nv * npm + geo) + 4 * nfc


def jac_bytes_per_element(dim, P, w):
    """Matrix-free Jacobian apply: read W and x, write y, plus the geometry."""
    nf, npm, nfc = 1 + dim + dim * dim, _np(P, dim), dim + 1
    geo = dim * dim + 1 + nfc * dim + nfc
    return w * (3 * nf * npm + geo) + 4 * nfc


def ev_pair():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_kernel(fn, stream, reps=20):
    """Mean HIP-event time of reps calls on `stream`, after one untimed call."""
    fn()
    a, b = ev_pair()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def median_call_seconds(fn, count, stream):
    """Median HIP-event duration of fn(i), i = 0 .. count - 1, each call
    bracketed by its own events on the library's stream."""
    fn(0)
    ev = [ev_pair() for _ in range(count)]
    for i in range(count):
        ev[i][0].record(stream)
        fn(i)
        ev[i][1].record(stream)
    ev[-1][1].synchronize()
    ts = sorted(a.elapsed_time(b) / 1e3 for a, b in ev)
    return ts[len(ts) // 2]


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second), median."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = ev_pair()
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / sorted(ts)[len(ts) // 2]


def hbm_resident(problem, mesh, disc, cp, dt, stream, op_bytes, jac_bytes, min_total=2 << 30):
    """Operator and Jacobian applies whose working sets cycle through enough
    independent buffers (>= 2 GiB in all) that every call finds its data
    evicted from the 256 MB Infinity Cache and reads it from HBM; the median
    of per-call event times.  Operator: (W, b_old, R) sets on one
    discretisation.  Jacobian: three discretisations linearised at their own
    states (each with its own face traces), each applied to several (x, y)
    sets in turn."""
    import torch
    import workloads as wl
    from paper_2301_11238_amd import bsw
    n_el, P, dtype = disc.n_el, problem.P, disc.dtype
    base = [torch.from_numpy(wl.random_state(2, P, n_el, 900 + k)).cuda().to(dtype) for k in range(4)]
    vec = base[0].numel() * base[0].element_size()
    b0 = disc.step_begin(cp, dt, base[0])
    op_set = 2 * vec + b0.numel() * b0.element_size()
    k_op = max(8, math.ceil(min_total / op_set))
    Ws = [base[k % 4].clone() for k in range(k_op)]
    Bs = [disc.step_begin(cp, dt, Ws[k]) for k in range(k_op)]
    Rs = [disc.empty() for _ in range(k_op)]
    t_op = median_call_seconds(lambda i: disc.operator_apply(cp, dt, Ws[i % k_op], Bs[i % k_op], Rs[i % k_op]),
                               max(64, 2 * k_op), stream)
    del Bs, Rs
    n_lin, n_xy = 3, max(4, math.ceil(min_total / (3 * 2 * vec)))
    discs = []
    for k in range(n_lin):
        d = bsw.Disc(mesh, P, disc.precision)
        d.jacobian_linearize(cp, dt, Ws[k])
        discs.append(d)
    xs = [torch.randn_like(Ws[0]) for _ in range(n_xy)]
    ys = [disc.empty() for _ in range(n_xy)]
    t_j = median_call_seconds(lambda i: discs[i % n_lin].jacobian_apply(xs[i % n_xy], ys[i % n_xy]),
                              max(64, 2 * n_lin * n_xy), stream)
    for d in discs:
        d.close()
    del discs, xs, ys, Ws
    torch.cuda.synchronize()
    n_dof = disc.state_len()

    def row(t, nbytes, sets, set_bytes):
        return {"buffer_sets": sets, "working_set_GiB": sets * set_bytes / 2 ** 30, "median_us": 1e6 * t,
                "GB/s": nbytes / t / 1e9, "frac_of_8TBs": nbytes / t / 8e12,
                "dof_updates_per_s": n_dof / t, "element_applies_per_s": n_el / t}
    return {"operator": row(t_op, op_bytes, k_op, op_set),
            "jacobian_apply": row(t_j, jac_bytes, n_lin * n_xy, 3 * vec),
            "note": "algorithmic bytes per call over the median per-call time; the buffers cycle through "
                    ">= 2 GiB so every call reads from HBM"}


def hot_path_passes(disc, cp, W, dt, args):
    """`warmup` untimed and `steps` timed passes over the whole hot path: each
    one backward-Euler time step cut to one Newton iteration whose GMRES runs
    one cycle of 30 Arnoldi steps (b_old, residual, linearisation with the
    block-Jacobi factors, 30 preconditioned Jacobian applies with Gram-Schmidt, the
    update with its line search, FP64 norms and diagnostics)."""
    import torch
    from paper_2301_11238_amd import bsw
    o = bsw.Options(t_end=10 * dt, dt=dt, max_steps=1, max_newton=1, gmres_m=30, gmres_max_iters=30,
                    forcing_max=1e-13, gmres_rtol=1e-13)
    for _ in range(args.warmup):
        disc.solve(cp, o, W)
    torch.cuda.synchronize()
    tot = dict(newton=0, gmres=0, operator_applies=0.0, jacobian_applies=0.0)
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = disc.solve(cp, o, W)
        log(f"hot-path pass {i + 1} of {args.steps}")
        tot["newton"] += st["newton_total"]
        tot["gmres"] += st["gmres_total"]
        tot["operator_applies"] += st["operator_applies"]
        tot["jacobian_applies"] += st["jacobian_applies"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, tot


def cpu_baseline(problem, seconds):
    """The FP64 C oracle's operator applies on the same mesh and state, on the
    host cores (a bounded sample), the same sample on one core, and one full
    oracle solve of the 1-D dam break."""
    import oracle
    import subprocess
    import workloads as wl
    orc = oracle.Oracle(problem.dim, problem.P, problem.xy, problem.el2vert)
    W = orc.project_ic(problem.ic)
    dt = 1e-3
    b = orc.step_begin(problem.params, W, dt)
    applies, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds or applies == 0:
        orc.residual(problem.params, W, b, dt)
        applies += 1
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=W.size * applies / el, unit="DOF-updates/s", cores=threads, kind="oracle",
               sample=f"{applies} operator applies of the FP64 C oracle on the same {orc.n_el}-triangle P{problem.P} "
                      f"mesh and initial state, {el:.1f} s")
    out["cpu_model"] = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                             if ln.startswith("model name")), None) if os.path.exists("/proc/cpuinfo") else None
    out["nproc"] = os.cpu_count()
    code = ("import sys; sys.path.insert(0, %r); import bench, workloads as wl; "
            "print(bench.cpu_baseline_applies(wl.config3(wl.REG1), %f))") % (ROOT, max(2.0, seconds / 3))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                             timeout=240)
        out["one_core_value"] = float(res.stdout.strip().splitlines()[-1])
    except Exception:  # reported as missing rather than failing the bench
        out["one_core_value"] = None
    c1 = wl.config1(wl.REG1)
    o1 = oracle.Oracle(c1.dim, c1.P, c1.xy, c1.el2vert)
    t1 = time.perf_counter()
    o1.solve(c1.params, o1.project_ic(c1.ic), oracle.SolveOptions(t_end=c1.t_end, cfl=c1.cfl))
    out["c1_solves_per_s"] = 1.0 / (time.perf_counter() - t1)
    return out


def cpu_baseline_applies(problem, seconds):
    """DOF-updates/s of the oracle's operator applies (the all-core measure of
    cpu_baseline, for a child run on one core)."""
    import oracle
    orc = oracle.Oracle(problem.dim, problem.P, problem.xy, problem.el2vert)
    W = orc.project_ic(problem.ic)
    b = orc.step_begin(problem.params, W, 1e-3)
    applies, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds or applies == 0:
        orc.residual(problem.params, W, b, 1e-3)
        applies += 1
    return W.size * applies / (time.perf_counter() - t0)


def fp32_applies(problem, mesh, cp, dt, stream, W64):
    """FP32 operator and Jacobian applies on the same mesh: HBM-resident rates
    and the error of one FP32 apply against the FP64 apply of the same state."""
    import numpy as np
    import torch
    from paper_2301_11238_amd import bsw
    d32 = bsw.Disc(mesh, problem.P, bsw.BSW_FP32)
    d64 = bsw.Disc(mesh, problem.P, bsw.BSW_FP64)
    W32 = W64.float()
    b64, b32 = d64.step_begin(cp, dt, W64), d32.step_begin(cp, dt, W32)
    R64, R32 = d64.operator_apply(cp, dt, W64, b64), d32.operator_apply(cp, dt, W32, b32)
    x = torch.randn_like(W64)
    d64.jacobian_linearize(cp, dt, W64)
    d32.jacobian_linearize(cp, dt, W32)
    y64, y32 = d64.jacobian_apply(x), d32.jacobian_apply(x.float())
    torch.cuda.synchronize()

    def rel(a, b):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {"rel_l2_operator_vs_fp64": rel(R32, R64), "rel_l2_jacobian_vs_fp64": rel(y32, y64)}
    d64.close()
    out["hbm_resident"] = hbm_resident(problem, mesh, d32, cp, dt, stream,
                                       bytes_per_element(2, problem.P, 4) * d32.n_el,
                                       jac_bytes_per_element(2, problem.P, 4) * d32.n_el)
    d32.close()
    return out


def c2_solve(ctx):
    """The incline configuration (8192 triangles, P2, reg 1, eps 1e-3) solved
    to Newton convergence: FP64 and FP32-mixed, one warm-up step, then five
    timed steps; the FP32 final state's error against FP64."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2301_11238_amd import bsw
    pb = wl.config2(wl.REG1, 1e-3)
    mesh = bsw.Mesh(ctx, 2, pb.xy, pb.el2vert)
    cp = bsw.make_params(pb.params)
    out, states = {}, {}
    for name, prec in (("fp64", bsw.BSW_FP64), ("fp32_mixed", bsw.BSW_FP32)):
        d = bsw.Disc(mesh, pb.P, prec)
        W = d.project_ic(pb.ic)
        dt = d.cfl_dt(cp, W, pb.cfl)
        d.solve(cp, bsw.Options(t_end=1.5 * dt, dt=dt, max_steps=1, precond_lag=1), W)
        torch.cuda.synchronize()
        n = 5
        t0 = time.perf_counter()
        st = d.solve(cp, bsw.Options(t_end=(n + 0.5) * dt, dt=dt, max_steps=n, precond_lag=1), W)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        states[name] = W.double().cpu().numpy()
        out[name] = {"ms_per_step": 1e3 * el / n, "newton_per_step": st["newton_total"] / n,
                     "gmres_per_step": st["gmres_total"] / n, "capped_steps": st["capped"],
                     "meets_accuracy_bar": st["capped"] == 0,
                     "max_mass_drift": st["max_mass_drift"], "dof_steps_per_s": d.state_len() * n / el}
        d.close()
    a, b = states["fp32_mixed"], states["fp64"]
    out["fp32_mixed"]["rel_l2_h_vs_fp64"] = float(np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0]))
    out["fp32_mixed"]["rel_l2_hu_vs_fp64"] = float(np.linalg.norm(a[1:3] - b[1:3]) /
                                                   max(np.linalg.norm(b[1:3]), 1e-300))
    out["workload"] = "2-D incline, 64x64 jittered -> 8192 triangles, P2, reg 1, eps 1e-3, 5 steps after 1"
    # the first two steps from the initial state with the Krylov solves run to
    # 1e-13, for the comparison with the stored oracle result (cpu_baseline leg)
    parity = {}
    for name, prec in (("fp64", bsw.BSW_FP64), ("fp32_mixed", bsw.BSW_FP32)):
        d = bsw.Disc(mesh, pb.P, prec)
        W = d.project_ic(pb.ic)
        dt = d.cfl_dt(cp, W, pb.cfl)
        for _ in range(2):
            d.solve(cp, bsw.Options(t_end=10 * dt, dt=dt, max_steps=1, gmres_rtol=1e-13, forcing_max=1e-13,
                                    gmres_m=60, gmres_max_iters=5000), W)
        parity[name] = W.double().cpu().numpy()
        d.close()
    mesh.close()
    return out, parity


def oracle_parity(states):
    """The incline's first two steps (reg 1, eps 1e-3; FP64 and FP32-mixed)
    against the oracle's result stored in tests/golden/c2_first_steps.json:
    relative L2 of h and h u at the volume points of the stored sample of 64
    elements, the points evaluated by the oracle."""
    import json
    import numpy as np
    import oracle
    import workloads as wl
    with open(os.path.join(ROOT, "tests", "golden", "c2_first_steps.json")) as f:
        g = next(r for r in json.load(f)["runs"] if r["reg"] == wl.REG1 and r["eps"] == 1e-3)
    pb = wl.config2(wl.REG1, 1e-3)
    orc = oracle.Oracle(2, pb.P, pb.xy, pb.el2vert)
    idx = np.asarray(g["elements"])
    hs, hus = np.asarray(g["h"]), np.asarray(g["hu"])
    out = {"workload": "2-D incline, 8192 triangles, P2, reg 1, eps 1e-3: the first two steps",
           "reference": "FP64 oracle (stored), Krylov solves to 1e-13 on both sides"}
    for name, bar in (("fp64", 1e-10), ("fp32_mixed", 1e-5)):
        vals = orc.eval_points(states[name])
        h = vals[..., 0]
        hu = vals[..., :1] * vals[..., 1:3]
        eh = float(np.linalg.norm(h[idx] - hs) / np.linalg.norm(hs))
        eq = float(np.linalg.norm(hu[idx] - hus) / np.linalg.norm(hus))
        out[name] = {"rel_l2_h": eh, "rel_l2_hu": eq, "bar": bar, "within_bar": eh <= bar and eq <= bar}
    return out


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def _opts(p, steps, gmres_max_iters=1200):
    from paper_2301_11238_amd import bsw
    return bsw.Options(t_end=p.t_end, cfl=p.cfl, max_steps=steps, gmres_max_iters=gmres_max_iters)


# GMRES iterations per Newton system of the stream and ensemble requests: most
# of their draws (eps down to 1e-5) cap Newton whatever the Krylov accuracy,
# and a batch advances in time-step lockstep, so unbounded Krylov work on a few
# hard requests would hold up every request resident with them
STREAM_GMRES_MAX = 150


def serving(ctx, n_req, steps):
    """Batched FP32 solve server against plain one-at-a-time FP64 solves on
    the same request list: slope flows and dam breaks of 512-8192 triangles,
    P 1-3, regularisations 1-3, eps in [1e-3, 1e-2], random yield stress and
    viscosity, each cut to `steps` time steps.  Throughput: all requests
    present at t = 0.  Latency: the same Poisson arrivals (70 % of the
    batched throughput) sent to the batched FP32 server and to a server that
    holds one FP64 solve at a time.  Accuracy: relative L2 of the (h, u1, u2)
    coefficients of the FP32 results against the FP64 ones, over the requests
    whose FP64 Newton converged in every step."""
    import numpy as np
    import workloads as wl
    from paper_2301_11238_amd import bsw
    probs = [wl.serving_request(k) for k in range(n_req)]

    def served(prec, slots, arrivals=None):
        srv = bsw.Server(ctx, 128 << 30, slots)
        out, lat = [None] * len(probs), []
        t0 = time.perf_counter()
        tickets = []
        for k, p in enumerate(probs):
            if arrivals is not None:
                dtw = t0 + arrivals[k] - time.perf_counter()
                if dtw > 0:
                    time.sleep(dtw)
            tickets.append(srv.submit(p.xy, p.el2vert, p.P, prec, bsw.make_params(p.params), ic=p.ic,
                                      opts=_opts(p, steps)))
        for k, t in enumerate(tickets):
            while srv.wait(t, 30.0) in (bsw.BSW_REQ_QUEUED, bsw.BSW_REQ_RUNNING):
                log(f"serving: waiting on request {k}")
            out[k] = srv.fetch(t)
            lat.append(out[k][1]["queue_seconds"] + out[k][1]["seconds"])
        T = time.perf_counter() - t0
        info = srv.info()
        srv.close()
        return T, out, lat, info

    T_plain, R_plain, _, _ = served(bsw.BSW_FP64, 1)
    log(f"serving: plain FP64 {T_plain:.1f} s")
    T32, R32, lat32_closed, info32 = served(bsw.BSW_FP32, 128)
    log(f"serving: batched FP32 {T32:.1f} s")
    T64, R64, _, _ = served(bsw.BSW_FP64, 128)
    log(f"serving: batched FP64 {T64:.1f} s")
    conv = [k for k in range(n_req) if R_plain[k][1]["capped"] == 0]
    err = max(float(np.linalg.norm(R32[k][0][:3].astype(np.float64) - R_plain[k][0][:3]) /
                    np.linalg.norm(R_plain[k][0][:3])) for k in conv) if conv else None
    ident = all(np.array_equal(R64[k][0], R_plain[k][0]) for k in range(n_req))
    rate = 0.7 * n_req / T32
    rng = np.random.default_rng(5)
    arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
    arr -= arr[0]
    _, _, lat32, _ = served(bsw.BSW_FP32, 128, arrivals=arr)
    log("serving: open-loop batched FP32 done")
    _, _, lat_plain, _ = served(bsw.BSW_FP64, 1, arrivals=arr)
    log("serving: open-loop plain FP64 done")
    return {
        "requests": n_req, "steps_per_request": steps, "dofs_total": sum(p.n_dof for p in probs),
        "workload": "slope flows and dam breaks, 512-8192 triangles, P 1-3, regs 1-3, eps 1e-3..1e-2",
        "converged_requests": len(conv), "capped_requests": n_req - len(conv),
        "plain_fp64": {"solves_per_s": n_req / T_plain, "seconds": T_plain,
                       "p50_s": pct(lat_plain, 50), "p99_s": pct(lat_plain, 99)},
        "batched_fp32": {"solves_per_s": n_req / T32, "seconds": T32, "p50_s": pct(lat32, 50),
                         "p99_s": pct(lat32, 99), "closed_loop_p50_s": pct(lat32_closed, 50),
                         "peak_resident": info32["peak_resident"], "launches": info32["launches"],
                         "max_rel_l2_vs_plain_fp64_converged": err},
        "batched_fp64": {"solves_per_s": n_req / T64, "seconds": T64, "bitwise_equal_to_plain": ident},
        "open_loop_rate_per_s": rate,
        "latency_note": "both p50/p99 measured: the same open-loop arrivals sent to each server",
        "speedup_fp32_batched_vs_plain_fp64": T_plain / T32,
    }


def request_stream(ctx, seconds, rate, steps, prec, slots, max_waiting=64, drain_s=15.0):
    """The stated request stream: Poisson arrivals at `rate` per second for
    `seconds`, 98 % dam-break draws of the ensemble's distribution (500-50,000
    triangles, P 1-3, eps 1e-5..1e-2) and 2 % 999,698-triangle P2 incline runs,
    each cut to `steps` time steps (the large runs to one) and to
    STREAM_GMRES_MAX Krylov iterations per Newton system.  Every request
    goes to the server, whose admission takes it when its device footprint
    fits the 128 GiB budget and one of `slots` slots is free; an arrival finding
    `max_waiting` requests already queued is rejected.  Requests unfinished
    `drain_s` after the window closes are cancelled.  Latencies per class."""
    import workloads as wl
    from paper_2301_11238_amd import bsw
    arrivals = wl.config5_arrivals(rate=rate, duration=seconds)
    large = wl.config5_large()
    srv = bsw.Server(ctx, 128 << 30, slots)
    sub, rejected = [], {"c4": 0, "large": 0}
    t0 = time.perf_counter()
    try:
        for ta, kind, k in arrivals:
            dtw = t0 + ta - time.perf_counter()
            if dtw > 0:
                time.sleep(dtw)
            if srv.info()["queued"] >= max_waiting:
                rejected[kind] += 1
                continue
            p = large if kind == "large" else wl.config4_instance(k, seed=5)
            t = srv.submit(p.xy, p.el2vert, p.P, prec, bsw.make_params(p.params), ic=p.ic,
                           opts=_opts(p, 1 if kind == "large" else steps, STREAM_GMRES_MAX))
            sub.append((t, kind))
        lat, done, capped, unfinished = {"c4": [], "large": []}, {"c4": 0, "large": 0}, 0, 0
        t_close = time.perf_counter()
        for t, kind in sub:
            left = drain_s - (time.perf_counter() - t_close)
            if srv.wait(t, min(max(left, 0.0), 60.0)) == bsw.BSW_REQ_DONE:
                _, st = srv.fetch(t)
                lat[kind].append(st["queue_seconds"] + st["seconds"])
                done[kind] += 1
                capped += int(st["capped"] > 0)
            else:
                srv.cancel(t)
                unfinished += 1
        T = time.perf_counter() - t0
        info = srv.info()
    finally:
        srv.close()
    log(f"request stream ({'FP32' if prec else 'FP64'}, {slots} slots): {sum(done.values())} done, "
        f"{unfinished} cancelled, {T:.1f} s")
    out = {"gmres_max_iters": STREAM_GMRES_MAX, "offered": len(arrivals),
           "offered_large": sum(1 for a in arrivals if a[1] == "large"),
           "submitted": len(sub), "rejected_queue_full": rejected, "completed": done,
           "completed_with_capped_steps": capped,
           "note_capped": "a request with a capped step did not meet the accuracy bar (Newton stopped at its "
                          "cap of 10 iterations); it is counted as served, not as converged",
           "cancelled_after_drain": unfinished,
           "achieved_solves_per_s": sum(done.values()) / T, "seconds": T, "peak_resident": info["peak_resident"]}
    for kind in ("c4", "large"):
        out[f"p50_s_{kind}"] = pct(lat[kind], 50)
        out[f"p99_s_{kind}"] = pct(lat[kind], 99)
    return out


def ensemble(ctx, n_inst, steps):
    """Dam-break instances of mixed size (500-50,000 triangles), order (1-3),
    step height, yield stress, viscosity, eps (1e-5..1e-2) and regularisation,
    all submitted at once to the batched FP32 server (at most 128 resident per
    order), each cut to `steps` time steps and to STREAM_GMRES_MAX Krylov
    iterations per Newton system."""
    import collections
    import workloads as wl
    from paper_2301_11238_amd import bsw
    probs = [wl.config4_instance(k) for k in range(n_inst)]
    srv = bsw.Server(ctx, 200 << 30, 3 * 128)
    per_order = collections.defaultdict(lambda: {"instances": 0, "capped": 0, "newton": 0, "gmres": 0})
    t0 = time.perf_counter()
    try:
        tickets = [srv.submit(p.xy, p.el2vert, p.P, bsw.BSW_FP32, bsw.make_params(p.params), ic=p.ic,
                              opts=_opts(p, steps, STREAM_GMRES_MAX)) for p in probs]
        for i, (p, t) in enumerate(zip(probs, tickets)):
            while srv.wait(t, 30.0) in (bsw.BSW_REQ_QUEUED, bsw.BSW_REQ_RUNNING):
                log(f"ensemble: waiting on instance {i}, {srv.info()['completed']:.0f} done")
            _, st = srv.fetch(t)
            r = per_order[f"P{p.P}"]
            r["instances"] += 1
            r["capped"] += int(st["capped"] > 0)
            r["newton"] += st["newton_total"]
            r["gmres"] += st["gmres_total"]
        T = time.perf_counter() - t0
        info = srv.info()
    finally:
        srv.close()
    return {"instances": n_inst, "steps_each": steps, "gmres_max_iters": STREAM_GMRES_MAX,
            "triangles_total": int(sum(p.n_el for p in probs)),
            "dofs_total": int(sum(p.n_dof for p in probs)), "seconds": T, "solves_per_s": n_inst / T,
            "peak_resident": info["peak_resident"], "kernel_launches": info["launches"],
            "per_order": dict(per_order),
            "note_capped": "'capped' counts instances with a step that stopped at the Newton cap: those did "
                           "not meet the accuracy bar"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path is built "
              f"and measured on one GPU; its sharding is a design note, not code)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as wl
    from paper_2301_11238_amd import bsw

    ctx = bsw.Context(0)
    bsw.tile_policy(args.tile_policy)
    stream = ctx.stream
    problem = wl.config3(wl.REG1) if args.workload == "c3" else wl.config2(wl.REG1, 1e-3)
    mesh = bsw.Mesh(ctx, 2, problem.xy, problem.el2vert)
    disc = bsw.Disc(mesh, problem.P, bsw.BSW_FP64)
    cp = bsw.make_params(problem.params)
    W = disc.project_ic(problem.ic)
    dt = disc.cfl_dt(cp, W, problem.cfl)
    n_dof, n_el = disc.state_len(), disc.n_el
    op_bytes = bytes_per_element(2, problem.P, 8) * n_el
    jac_bytes = jac_bytes_per_element(2, problem.P, 8) * n_el
    bs = disc.nf * disc.np
    nv, nu, ne = 3 * disc.np, 2 * disc.np, 4 * disc.np
    nb_schur = nv * nv + nu * ne  # block-Jacobi factors per triangle: S^-1 and A_UE (FP32)
    nb_read = nv * nv + 2 * nu * ne + ne  # the block entries the factors use (A_VV, A_UE, A_EU, diag A_EE)

    def single_set_kernels(Wk):
        b = disc.step_begin(cp, dt, Wk)
        R = disc.empty()
        t_op = time_kernel(lambda: disc.operator_apply(cp, dt, Wk, b, R), stream)
        t_lin = time_kernel(lambda: disc.jacobian_linearize(cp, dt, Wk), stream, reps=3)
        x = torch.randn_like(Wk)
        y = disc.empty()
        t_jac = time_kernel(lambda: disc.jacobian_apply(x, y), stream)
        t_pc = time_kernel(lambda: disc.precond_apply(x, y), stream)
        return {
            "operator": dict(seconds=t_op, bytes=op_bytes),
            "jacobian_apply": dict(seconds=t_jac, bytes=jac_bytes),
            # the FP32 factors (S^-1, A_UE), x and y
            "block_jacobi_apply": dict(seconds=t_pc, bytes=(4 * nb_schur + 2 * 8 * bs) * n_el),
            # the parts of the FP64 diagonal blocks the factors use (written
            # by the assembly, read by the factor build) and the FP32 factors
            "linearisation": dict(seconds=t_lin, bytes=(2 * 8 * nb_read + 4 * nb_schur) * n_el),
        }

    if args.kernels_only:
        Wr = torch.from_numpy(wl.random_state(2, problem.P, n_el, 11)).cuda()
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        kern = single_set_kernels(Wr)
        print(json.dumps({"workload": args.workload, "n_el": n_el, "P": problem.P,
                          "kernels": {k: {"us": 1e6 * v["seconds"], "GB/s": v["bytes"] / v["seconds"] / 1e9}
                                      for k, v in kern.items()}}))
        return

    log(f"mesh {n_el} triangles, P{problem.P}, {n_dof} DOFs, dt {dt:.3e}")
    # ---------------------------------------------------------------- timed: hot-path passes
    el, tot = hot_path_passes(disc, cp, W, dt, args)
    log(f"hot-path passes: {1e3 * el / args.steps:.1f} ms each")
    # ---------------------------------------------------------------- value: HBM-resident applies
    hbm = hbm_resident(problem, mesh, disc, cp, dt, stream, op_bytes, jac_bytes)
    t_op = hbm["operator"]["median_us"] * 1e-6
    log(f"HBM-resident operator {1e6 * t_op:.1f} us, Jacobian apply {hbm['jacobian_apply']['median_us']:.1f} us")
    value = n_dof / t_op
    kern = single_set_kernels(W)
    achieved = op_bytes / t_op / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": TRAFFIC_BYTES.get("operator"),
            "kernel": "k_elem<2,3,double,0,1> (the operator apply: one element pass on tiles of 64 triangles, "
                      "one lane per element)",
            "bytes_per_launch": op_bytes, "launch_seconds": t_op,
            "bytes_per_element": bytes_per_element(2, problem.P, 8),
            "note": "algorithmic bytes per apply over the median HIP-event duration of HBM-resident applies "
                    "on the library's stream"}
    out = {
        "metric": "DG DOF-updates/s (+% HBM roofline); solves/s and p50/p99 latency, batched vs plain",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded jittered mesh, analytic initial states)",
        "config": {"workload": "2-D circular dam break mesh: 256x256 jittered -> 131072 triangles, DG P3, "
                               "FP64, walls, reg 1, eps 1e-4 (gamma = beta = 1e4)",
                   "n_el": n_el, "n_dof": n_dof, "dt": dt,
                   "value_definition": "n_dof / median HBM-resident operator-apply time",
                   "step": "one pass over the whole hot path: b_old, residual, linearisation (traces, diagonal "
                           "blocks, FP32 Schur-complement factors), one GMRES(30) cycle of preconditioned matrix-free "
                           "Jacobian applies, the Newton update with its line search, FP64 reductions",
                   "per_step": {k: v / args.steps for k, v in tot.items()},
                   "operator_dof_updates_per_s": value,
                   "jacobian_apply_dof_updates_per_s": hbm["jacobian_apply"]["dof_updates_per_s"],
                   "operator_roofline_gap": f"{roof['frac']:.3f} of 8 TB/s against the 0.60 target"},
        "roofline": roof,
        "hbm_resident": hbm,
        "kernels": {k: {"us": 1e6 * v["seconds"], "GB/s": v["bytes"] / v["seconds"] / 1e9,
                        "frac_of_8TBs": v["bytes"] / v["seconds"] / 8e12} for k, v in kern.items()},
        "copy_GB/s": copy_bandwidth() / 1e9,
    }
    out["kernels"]["note"] = "single buffer set (Infinity-Cache resident where it fits), mean of 20 calls"
    if not args.no_fp32:
        Wr = torch.from_numpy(wl.random_state(2, problem.P, n_el, 21)).cuda()
        out["fp32"] = fp32_applies(problem, mesh, cp, dt, stream, Wr)
        del Wr
        log("FP32 applies done")
    out["tile_autotuner"] = [{"pass": "jacobian" if r["mode"] else "residual", "P": r["P"],
                              "precision": "f64" if r["bytes"] == 8 else "f32", "size_class": r["size_class"],
                              "variant": r["variant"],
                              "best_us": {str(n): round(v, 2) for n, v in r["best_us"].items()}}
                             for r in bsw.tile_table() if r["dim"] == 2]
    disc.close()
    mesh.close()
    torch.cuda.synchronize()
    parity_states = None
    if not args.no_c2:
        out["c2_solve"], parity_states = c2_solve(ctx)
        log("incline solve done")
    if not args.no_serving:
        out["serving"] = serving(ctx, args.serve_requests, args.serve_steps)
        log("serving comparison done")
        out["request_stream"] = {
            "window_s": args.stream_seconds, "rate_per_s": args.stream_rate, "steps_per_request": args.serve_steps,
            "batched_fp32": request_stream(ctx, args.stream_seconds, args.stream_rate, args.serve_steps,
                                           bsw.BSW_FP32, 128),
            "plain_fp64": request_stream(ctx, args.stream_seconds, args.stream_rate, args.serve_steps,
                                         bsw.BSW_FP64, 1)}
        log("request streams done")
        out["ensemble"] = ensemble(ctx, args.ensemble, args.ensemble_steps)
        log("ensemble done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, args.cpu_seconds)
        if parity_states is not None:
            out["oracle_parity"] = oracle_parity(parity_states)
        log("CPU baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
