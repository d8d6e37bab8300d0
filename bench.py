"""Benchmark: implicit steps of the regularised-Bingham DG solver on one MI355X.

Workload (the 2-D incline configuration): 64x64 jittered squares split into
8192 triangles on a 20 m x 20 m domain, DG P2 (6 modes, 7-point rule), 10 %
slope, Gaussian mound h = 1 + 0.5 exp(-r^2/4), regularisation 1 with
eps = 1e-3 (gamma = beta = 1e3), yield stress drawn U[20, 200] Pa, FP64.
Inputs are synthetic and seeded; the state sits in HBM before timing starts.

One step = one backward-Euler time step: b_old, Newton iterations (operator
apply, Jacobian linearisation and block LU, block-Jacobi GMRES with matrix-free
Jacobian applies, backtracking, stage update) -- every row of the hot path.

value = DOF-updates/s: degrees of freedom times the number of whole-mesh
operator and Jacobian applies done in the timed steps, divided by the time.
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
# HBM bytes per launch from the rocprofv3 FETCH_SIZE + WRITE_SIZE passes,
# scaled by the same counters on a plain copy of known size; None until the
# counters are taken on the current kernel.
TRAFFIC_BYTES = {"jacobian_apply": 14612480.0}  # element pass; counter summary under profiles/


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: the 8192-triangle P2 incline (default); c3: the 131072-triangle P3 mesh of the "
                         "circular dam break (kernel timings only)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed leg of the solve")
    ap.add_argument("--no-hbm-resident", action="store_true",
                    help="skip the operator and Jacobian applies cycled through >= 2 GiB of buffer sets")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving comparison (batched FP32 server vs plain FP64 solves)")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-steps", type=int, default=3,
                    help="time steps per served request (each draw's horizon is cut to this many steps)")
    ap.add_argument("--tile-policy", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="element-pass variant: -1 autotune (default), 0/1/2 force one (triangles: occupancy "
                         "target of 1/2/3 waves per SIMD) "
                         "(profiling runs repeat the shape the autotuner picked in the bench run)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="no solve: a 256 MiB device copy (counter calibration) and 20 launches of each hot "
                         "kernel, for rocprofv3 --pmc passes")
    return ap.parse_args()


def bytes_per_element(dim, P, w):
    """Algorithmic HBM bytes of one operator apply per element: read W (n_f N_p),
    b_old (N_v N_p), write R (n_f N_p), the affine metric, normals and face
    lengths (dim^2 + 1 + (dim+1)(dim+1) reals) and the neighbour codes."""
    nf, nv = 1 + dim + dim * dim, 1 + dim
    npm = P + 1 if dim == 1 else (P + 1) * (P + 2) // 2
    nfc = dim + 1
    geo = dim * dim + 1 + nfc * dim + nfc
    return w * (2 * nf * npm + nv * npm + geo) + 4 * nfc


def jac_bytes_per_element(dim, P, w):
    """Matrix-free Jacobian apply: read W and x, write y, plus the geometry."""
    nf = 1 + dim + dim * dim
    npm = P + 1 if dim == 1 else (P + 1) * (P + 2) // 2
    nfc = dim + 1
    geo = dim * dim + 1 + nfc * dim + nfc
    return w * (3 * nf * npm + geo) + 4 * nfc


def time_kernel(fn, stream, reps=20):
    import torch
    fn()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / 1e3 / reps


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second), median."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / sorted(ts)[len(ts) // 2]


def median_call_seconds(fn, count, stream):
    """Median HIP-event duration of fn(i), i = 0 .. count - 1, each call
    bracketed by its own events on the library's stream."""
    import torch
    fn(0)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    for i in range(count):
        ev[i][0].record(stream)
        fn(i)
        ev[i][1].record(stream)
    ev[-1][1].synchronize()
    ts = sorted(a.elapsed_time(b) / 1e3 for a, b in ev)
    return ts[len(ts) // 2]


def hbm_resident(problem, mesh, disc, cp, dt, stream, op_bytes, jac_bytes, min_total=2 << 30):
    """Operator and Jacobian applies whose working sets cycle through enough
    independent buffer sets (>= 2 GiB in all) that every call finds its data
    evicted from the 256 MB Infinity Cache and reads it from HBM; the median
    of per-call event times.  Operator sets: (W, b_old, R) on one
    discretisation.  Jacobian sets: one discretisation per set, linearised
    at its own W, with its own x and y (the traces of W and x are per set)."""
    import math as _m
    import torch
    import workloads as wl
    from paper_2301_11238_amd import bsw
    n_el, P = disc.n_el, problem.P
    base = [torch.from_numpy(wl.random_state(2, P, n_el, 900 + k)).cuda() for k in range(4)]
    b0 = disc.step_begin(cp, dt, base[0])
    vec = base[0].numel() * 8
    # operator
    k_op = max(8, _m.ceil(min_total / (2 * vec + b0.numel() * 8)))
    Ws = [base[k % 4].clone() for k in range(k_op)]
    Bs = [disc.step_begin(cp, dt, Ws[k]) for k in range(k_op)]
    Rs = [disc.empty() for _ in range(k_op)]
    t_op = median_call_seconds(lambda i: disc.operator_apply(cp, dt, Ws[i % k_op], Bs[i % k_op], Rs[i % k_op]),
                               max(64, 2 * k_op), stream)
    op_set = 2 * vec + b0.numel() * 8
    del Bs, Rs
    # Jacobian
    nfp = disc.nf * 3 * (P + 1) * n_el * 8          # face traces of one vector (3 faces, P + 1 points)
    jac_set = 3 * vec + 2 * nfp
    k_j = max(8, _m.ceil(min_total / jac_set))
    discs, xs, ys = [], [], []
    for k in range(k_j):
        d = bsw.Disc(mesh, P, bsw.BSW_FP64)
        W = Ws[k % k_op] if k < k_op else base[k % 4].clone()
        Ws.append(W)
        d.jacobian_linearize(cp, dt, W)
        discs.append(d)
        xs.append(torch.randn_like(W))
        ys.append(d.empty())
    t_j = median_call_seconds(lambda i: discs[i % k_j].jacobian_apply(xs[i % k_j], ys[i % k_j]),
                              max(64, 2 * k_j), stream)
    for d in discs:
        d.close()
    del discs, xs, ys, Ws
    torch.cuda.synchronize()
    copy = copy_bandwidth()

    def row(t, nbytes, k, set_bytes):
        return {"buffer_sets": k, "working_set_GiB": k * set_bytes / 2 ** 30, "median_us": 1e6 * t,
                "GB/s": nbytes / t / 1e9, "frac_of_8TBs": nbytes / t / 8e12, "frac_of_copy": nbytes / t / copy,
                "element_applies_per_s": n_el / t}
    return {"operator": row(t_op, op_bytes, k_op, op_set), "jacobian_apply": row(t_j, jac_bytes, k_j, jac_set),
            "copy_GB/s": copy / 1e9,
            "note": "algorithmic bytes per call over the median per-call time, data cycled through >= 2 GiB "
                    "of buffer sets so it comes from HBM; the `kernels` section is the same calls on one "
                    "buffer set (Infinity-Cache resident)"}


def cpu_baseline(problem, seconds):
    """Oracle operator and Jacobian applies on the same mesh and state."""
    import numpy as np
    import oracle
    import workloads as wl
    orc = oracle.Oracle(problem.dim, problem.P, problem.xy, problem.el2vert)
    W = orc.project_ic(problem.ic)
    dt = 0.01
    b = orc.step_begin(problem.params, W, dt)
    x = wl.random_vector(problem.dim, problem.P, orc.n_el, 1)
    n_dof = W.size
    applies, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        orc.residual(problem.params, W, b, dt)
        orc.jac_apply(problem.params, W, x, dt)
        applies += 2
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=n_dof * applies / el, unit="DOF-updates/s", cores=threads, kind="oracle",
               sample=f"{applies} whole-mesh applies (operator + Jacobian, alternating) of the FP64 C oracle "
                      f"on the same 8192-triangle P2 mesh, {el:.1f} s")
    out["cpu_model"] = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                             if ln.startswith("model name")), None) if os.path.exists("/proc/cpuinfo") else None
    out["nproc"] = os.cpu_count()
    # the same sample on one core, in a child process started with one OpenMP thread
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import bench, workloads as wl; "
            "p = wl.config2(wl.REG1, 1e-3); r = bench.cpu_baseline_applies(p, %f); print(r)") % (ROOT, seconds / 3)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        out["one_core_value"] = float(res.stdout.strip().splitlines()[-1])
    except Exception:  # reported as missing rather than failing the bench
        out["one_core_value"] = None
    # one full solve of the 1-D dam break (200 P1 elements, reg 1, 314 steps to t = 1)
    c1 = wl.config1(wl.REG1)
    o1 = oracle.Oracle(c1.dim, c1.P, c1.xy, c1.el2vert)
    t1 = time.perf_counter()
    o1.solve(c1.params, o1.project_ic(c1.ic), oracle.SolveOptions(t_end=c1.t_end, cfl=c1.cfl))
    out["c1_solves_per_s"] = 1.0 / (time.perf_counter() - t1)
    return out


def cpu_baseline_applies(problem, seconds):
    """DOF-updates/s of the oracle's alternating operator and Jacobian applies
    (the all-core measure of cpu_baseline, for a child run on one core)."""
    import oracle
    import workloads as wl
    orc = oracle.Oracle(problem.dim, problem.P, problem.xy, problem.el2vert)
    W = orc.project_ic(problem.ic)
    dt = 0.01
    b = orc.step_begin(problem.params, W, dt)
    x = wl.random_vector(problem.dim, problem.P, orc.n_el, 1)
    applies, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        orc.residual(problem.params, W, b, dt)
        orc.jac_apply(problem.params, W, x, dt)
        applies += 2
    return W.size * applies / (time.perf_counter() - t0)


def fp32_leg(problem, mesh, cp, dt, args, W64, el64):
    """The same warm-up and timed steps on the FP32-mixed path (FP32 state and
    arithmetic, FP64 reductions and small-shear series), from the same
    initial state; error of its final (h, h u) against the FP64 run's."""
    import numpy as np
    import torch
    from paper_2301_11238_amd import bsw
    d32 = bsw.Disc(mesh, problem.P, bsw.BSW_FP32)
    W = d32.project_ic(problem.ic)
    if args.warmup > 0:
        d32.solve(cp, bsw.Options(t_end=(args.warmup + 0.5) * dt, dt=dt, max_steps=args.warmup, precond_lag=1), W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = d32.solve(cp, bsw.Options(t_end=(args.steps + 0.5) * dt, dt=dt, max_steps=args.steps, precond_lag=1), W)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    a = W.double().cpu().numpy()
    b = W64.double().cpu().numpy()
    h_a, h_b = a[0], b[0]
    err_h = float(np.linalg.norm(h_a - h_b) / np.linalg.norm(h_b))
    err_u = float(np.linalg.norm(a[1:3] - b[1:3]) / max(np.linalg.norm(b[1:3]), 1e-300))
    d32.close()
    return {"ms_per_step": 1e3 * el / args.steps, "speedup_vs_fp64": el64 / el,
            "newton_per_step": st["newton_total"] / max(1, st["steps"]),
            "gmres_per_step": st["gmres_total"] / max(1, st["steps"]),
            "capped_steps": st["capped"],
            "rel_l2_coeff_h_vs_fp64": err_h, "rel_l2_coeff_u_vs_fp64": err_u}


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def overload(ctx, steps, rate=200.0, window_s=1.0, max_admitted=32, dof_cap=4.0e6, deadline_s=90.0):
    """The stated request stream above capacity, with a bounded admission
    window: Poisson arrivals at `rate` per second for `window_s` seconds
    (2 % of them large 999,698-triangle P2 incline runs).  A large run is
    rejected for exceeding the per-request cap of `dof_cap` DOFs; any other
    arrival is admitted to the batched FP32 server while fewer than
    `max_admitted` admitted requests are unfinished, and rejected otherwise.
    Admitted requests are drawn from the serving mix (512-8192 triangles, P
    1-3, regs 1-3), cut to `steps` time steps; those still unfinished
    `deadline_s` after the first arrival are cancelled and counted."""
    import numpy as np
    import workloads as wl
    from paper_2301_11238_amd import bsw
    arrivals = wl.config5_arrivals(rate=rate, duration=window_s)
    srv = bsw.Server(ctx, 128 << 30, 128)
    admitted, rej_full, rej_large = [], 0, 0
    t0 = time.perf_counter()
    try:
        for ta, kind, k in arrivals:
            dtw = t0 + ta - time.perf_counter()
            if dtw > 0:
                time.sleep(dtw)
            if kind == "large":          # 999,698 x 42 DOFs
                rej_large += 1
                continue
            live = sum(1 for t, _ in admitted if srv.poll(t) in (bsw.BSW_REQ_QUEUED, bsw.BSW_REQ_RUNNING))
            if live >= max_admitted:
                rej_full += 1
                continue
            p = wl.serving_request(2000 + k)
            if p.n_dof > dof_cap:
                rej_large += 1
                continue
            t = srv.submit(p.xy, p.el2vert, p.P, bsw.BSW_FP32, bsw.make_params(p.params), ic=p.ic,
                           opts=bsw.Options(t_end=p.t_end, cfl=p.cfl, max_steps=steps))
            admitted.append((t, ta))
        lat, done, unfinished = [], 0, 0
        for t, ta in admitted:
            left = deadline_s - (time.perf_counter() - t0)
            if srv.wait(t, max(left, 0.0)) == bsw.BSW_REQ_DONE:
                _, st = srv.fetch(t)
                lat.append(st["queue_seconds"] + st["seconds"])
                done += 1
            else:
                srv.cancel(t)
                unfinished += 1
        T = time.perf_counter() - t0
    finally:
        srv.close()
    return {"offered_rate_per_s": rate, "window_s": window_s, "offered": len(arrivals),
            "admitted": len(admitted), "rejected_window_full": rej_full, "rejected_over_cap": rej_large,
            "max_admitted": max_admitted, "completed": done, "cancelled_at_deadline": unfinished,
            "achieved_solves_per_s": done / T, "seconds": T,
            "p50_s": float(np.percentile(lat, 50)) if lat else None,
            "p99_s": float(np.percentile(lat, 99)) if lat else None}


def serving(ctx, n_req, steps):
    """Batched FP32 solve server against plain one-solve-at-a-time FP64 solves
    on the same request list: slope flows and dam breaks of 512-8192
    triangles, P 1-3, regularisations 1-3, eps in [1e-3, 1e-2], random yield
    stress and viscosity, each cut to `steps` time steps.  Throughput: all
    requests present at t = 0.  Latency: Poisson arrivals at 70% of the
    batched server's measured throughput; the plain method's latencies come
    from its measured service times in a FIFO queue.  Accuracy: relative L2
    of the (h, u1, u2) coefficients of the FP32 results against the FP64 ones,
    over the requests whose FP64 Newton converged in every step."""
    import numpy as np
    import workloads as wl
    from paper_2301_11238_amd import bsw
    probs = [wl.serving_request(k) for k in range(n_req)]

    def opts(p):
        return bsw.Options(t_end=p.t_end, cfl=p.cfl, max_steps=steps)

    # plain: FP64, one solve at a time (upload, project, solve, copy back)
    t0 = time.perf_counter()
    svc, plain = [], []
    for p in probs:
        a = time.perf_counter()
        m = bsw.Mesh(ctx, 2, p.xy, p.el2vert)
        d = bsw.Disc(m, p.P, bsw.BSW_FP64)
        W = d.project_ic(p.ic)
        st = d.solve(bsw.make_params(p.params), opts(p), W)
        plain.append((W.cpu().numpy(), st))
        svc.append(time.perf_counter() - a)
        d.close()
        m.close()
    T_plain = time.perf_counter() - t0

    def served(prec, arrivals=None):
        srv = bsw.Server(ctx, 128 << 30, 128)
        out, lat = [None] * len(probs), []
        t0 = time.perf_counter()
        tickets = []
        for k, p in enumerate(probs):
            if arrivals is not None:
                dtw = t0 + arrivals[k] - time.perf_counter()
                if dtw > 0:
                    time.sleep(dtw)
            tickets.append(srv.submit(p.xy, p.el2vert, p.P, prec, bsw.make_params(p.params), ic=p.ic,
                                      opts=opts(p)))
        for k, t in enumerate(tickets):
            srv.wait(t, 3600.0)
            out[k] = srv.fetch(t)
            lat.append(out[k][1]["queue_seconds"] + out[k][1]["seconds"])
        T = time.perf_counter() - t0
        info = srv.info()
        srv.close()
        return T, out, lat, info

    T32, R32, lat32_closed, info32 = served(bsw.BSW_FP32)
    T64, R64, _, _ = served(bsw.BSW_FP64)
    conv = [k for k in range(n_req) if plain[k][1]["capped"] == 0]
    err = max(float(np.linalg.norm(R32[k][0][:3].astype(np.float64) - plain[k][0][:3]) /
                    np.linalg.norm(plain[k][0][:3])) for k in conv) if conv else None
    ident = all(np.array_equal(R64[k][0], plain[k][0]) for k in range(n_req))
    rate = 0.7 * n_req / T32
    rng = np.random.default_rng(5)
    arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
    arr -= arr[0]
    _, _, lat32, _ = served(bsw.BSW_FP32, arrivals=arr)
    done, lat_plain = 0.0, []
    for a, s_ in zip(arr, svc):
        done = max(done, a) + s_
        lat_plain.append(done - a)
    dofs = sum(p.n_dof for p in probs)
    return {
        "requests": n_req, "steps_per_request": steps, "dofs_total": dofs,
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
        "speedup_fp32_batched_vs_plain_fp64": T_plain / T32,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path is built "
              f"and measured on one GPU; its sharding is a design note, not code)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as wl
    from paper_2301_11238_amd import bsw

    problem = wl.config2(wl.REG1, 1e-3) if args.workload == "c2" else wl.config3(wl.REG1)
    if args.workload == "c3":
        args.kernels_only = True
    ctx = bsw.Context(0)
    bsw.tile_policy(args.tile_policy)
    stream = ctx.stream
    mesh = bsw.Mesh(ctx, 2, problem.xy, problem.el2vert)
    disc = bsw.Disc(mesh, problem.P, bsw.BSW_FP64)
    cp = bsw.make_params(problem.params)
    W = disc.project_ic(problem.ic)
    dt = disc.cfl_dt(cp, W, problem.cfl)
    n_dof = disc.state_len()

    if args.kernels_only:
        W = torch.from_numpy(wl.random_state(2, problem.P, disc.n_el, 11)).cuda()
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        st = {"steps": 0, "newton_total": 0, "gmres_total": 0, "capped": 0}
        el, applies, value = 0.0, 0.0, 0.0
        fp32 = None
    else:
        # warm-up steps, then exactly `steps` timed steps from where warm-up ended
        if args.warmup > 0:
            disc.solve(cp, bsw.Options(t_end=(args.warmup + 0.5) * dt, dt=dt, max_steps=args.warmup, precond_lag=1), W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = disc.solve(cp, bsw.Options(t_end=(args.steps + 0.5) * dt, dt=dt, max_steps=args.steps, timing=1,
                                        precond_lag=1), W)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if st["steps"] != args.steps:
            raise RuntimeError(f"solve stopped after {st['steps']} of {args.steps} steps: {st}")
        applies = st["operator_applies"] + st["jacobian_applies"]
        value = n_dof * applies / el
        if not args.no_fp32:
            fp32 = fp32_leg(problem, mesh, cp, dt, args, W, el)

    # live roofline of the operator and Jacobian kernels (HIP events on the library's stream)
    b = disc.step_begin(cp, dt, W)
    R = disc.empty()
    t_op = time_kernel(lambda: disc.operator_apply(cp, dt, W, b, R), stream)
    t_lin = time_kernel(lambda: disc.jacobian_linearize(cp, dt, W), stream, reps=5)
    x = torch.randn_like(W)
    y = disc.empty()
    t_jac = time_kernel(lambda: disc.jacobian_apply(x, y), stream)
    t_pc = time_kernel(lambda: disc.precond_apply(x, y), stream)
    n_el = disc.n_el
    op_bytes = bytes_per_element(2, problem.P, 8) * n_el
    jac_bytes = jac_bytes_per_element(2, problem.P, 8) * n_el
    bs = disc.nf * disc.np
    pc_bytes = (4 * bs * bs + 2 * 8 * bs) * n_el   # FP32 inverse blocks, FP64 x read and y written
    kern = {
        "operator": dict(seconds=t_op, bytes=op_bytes),
        "jacobian_apply": dict(seconds=t_jac, bytes=jac_bytes),
        "block_jacobi_solve": dict(seconds=t_pc, bytes=pc_bytes),
        # linearisation: traces of W, the element Jacobian blocks (FP64,
        # written then read by the inversion) and their FP32 inverses
        "preconditioner_setup": dict(seconds=t_lin, bytes=(8 + 8 + 4) * bs * bs * n_el),
    }
    # the matrix-free Jacobian apply runs once per GMRES iteration: the dominant
    # kernel; its duration is the HIP-event average over the timed steps
    dominant = "jacobian_apply"
    k = kern[dominant]
    if not args.kernels_only and st["jac_apply_launches"] > 0:
        k = dict(bytes=k["bytes"], seconds=st["jac_apply_seconds"] / st["jac_apply_launches"])
    achieved = k["bytes"] / k["seconds"] / 1e9
    # the element-tile shape the autotuner kept for this pass (Jacobian, FP64, P2, this size class)
    tuned = [r for r in bsw.tile_table() if (r["dim"], r["P"], r["bytes"], r["mode"]) == (2, problem.P, 8, 1)
             and r["size_class"] == int(math.floor(math.log2(n_el)))]
    variant = tuned[0]["variant"] if tuned and tuned[0]["variant"] >= 0 else 1
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": TRAFFIC_BYTES.get(dominant),
            "kernel": f"kb_elem<2,{problem.P},double,1,{variant}> (matrix-free Jacobian apply inside the solve: "
                      "one element pass in the autotuned tile shape, the neighbours' side of x evaluated in it)",
            "bytes_per_launch": k["bytes"], "launch_seconds": k["seconds"],
            "launches_timed": st.get("jac_apply_launches", 0)}
    hbm = None
    if not args.kernels_only and not args.no_hbm_resident:
        hbm = hbm_resident(problem, mesh, disc, cp, dt, stream, op_bytes, jac_bytes)
    if args.kernels_only:
        print(json.dumps({"workload": args.workload, "n_el": n_el, "P": problem.P,
                          "kernels": {n: {"ms": 1e3 * v["seconds"], "GB/s": v["bytes"] / v["seconds"] / 1e9}
                                      for n, v in kern.items()}}))
        return

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
        "data": "synthetic (seeded jittered mesh, analytic initial mound)",
        "config": {"workload": "2-D Bingham flow on a 10% incline, 64x64 jittered -> 8192 triangles, "
                               "DG P2, reg 1, eps 1e-3, FP64, backward Euler at CFL 0.2",
                   "solver": "Newton (<= 10 its, ||dW|| <= 1e-10 (1 + ||W||) or ||R|| <= 1e-13 ||b_old||), "
                             "GMRES(30) with block-Jacobi kept across Newton iterations while it serves, "
                             "forcing term <= 3e-2",
                   "n_el": n_el, "n_dof": n_dof, "dt": dt,
                   "newton_per_step": st["newton_total"] / max(1, st["steps"]),
                   "gmres_per_step": st["gmres_total"] / max(1, st["steps"]),
                   "capped_steps": st["capped"],
                   "applies_per_step": applies / max(1, st["steps"]),
                   # per pipelined Arnoldi step (seven launches): host time to issue it and
                   # host time blocked on its results; issue < step time means the launch
                   # path is not the limit (the device is)
                   "arnoldi_step_us": 1e6 * el / max(1.0, st["arnoldi_steps"]) if st["arnoldi_steps"] else None,
                   "host_issue_us_per_arnoldi_step": 1e6 * st["host_issue_seconds"] / max(1.0, st["arnoldi_steps"]),
                   "host_wait_us_per_arnoldi_step": 1e6 * st["host_wait_seconds"] / max(1.0, st["arnoldi_steps"]),
                   "dof_steps_per_s": n_dof * st["steps"] / el},
        "roofline": roof,
        "fp32_mixed": fp32 if not args.no_fp32 else None,
        "kernels": {name: {"ms": 1e3 * v["seconds"], "GB/s": v["bytes"] / v["seconds"] / 1e9}
                    for name, v in kern.items()},
        "hbm_resident": hbm,
        "tile_autotuner": [{"pass": "jacobian" if r["mode"] else "residual",
                            "precision": "f64" if r["bytes"] == 8 else "f32", "size_class": r["size_class"],
                            "variant": r["variant"],
                            "best_us": {str(n): round(v, 2) for n, v in r["best_us"].items()}}
                           for r in bsw.tile_table() if r["dim"] == 2 and r["P"] == problem.P],
    }
    if not args.no_serving:
        out["serving"] = serving(ctx, args.serve_requests, args.serve_steps)
        out["serving"]["overload"] = overload(ctx, args.serve_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
