"""Benchmark of the fused LSRK4 stage kernel: DOF-updates/s on one MI355X.

A "step" is one full five-stage LSRK4 step of the whole hot path (volume
differentiation, face gather + upwind flux, LIFT, RK update, fused in one
kernel per stage).  Default workload: the 2D TM PEC cavity on a 512x512 grid
-> 524288 jittered triangles, order N=7 (Np=36), mode (2,3), CFL time step,
in FP32 (`value`), with the split-BF16 and split-FP16 forms timed beside it
and every variant's relative L2 error against the closed-form mode at t = 1.
Inputs are resident in HBM before the timed region.  A short serving leg
(continuous batching of a seeded request mix) adds p50/p99 latency.

    python bench.py [--steps K] [--warmup W] [--config c3|c2|c1|c5] [--prec P]
                    [--variants LIST] [--serve-short N] [--no-cpu]

Prints one JSON line (metric, value, roofline, cpu_baseline, accuracy, per
precision variant the throughput and the L2 error at t = 1, serving).
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

METRIC = "DOF-updates/s (FP32 vs split-BF16 at stated L2 err); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: (grid s, mesh seed, permute, order N, mode, description); "c5" is 3D
    "c1": (8, 1, False, 3, (1, 1), "2D TM PEC cavity, 8x8 grid -> 128 triangles, N=3, mode (1,1)"),
    "c2": (256, 2, True, 5, (2, 3), "2D TM PEC cavity, 256x256 grid -> 131072 randomly permuted triangles "
                                    "(interior vertices jittered +-0.1h), N=5 (Np=21), mode (2,3), "
                                    "5-stage LSRK4 at the CFL step"),
    "c3": (512, 3, False, 7, (2, 3), "2D TM PEC cavity, 512x512 grid -> 524288 triangles, N=7 (Np=36), "
                                     "mode (2,3), 5-stage LSRK4 at the CFL step"),
    "c5": (48, 5, False, 4, (1, 1, 1), "3D Maxwell PEC cube, 48^3 cubes x 6 -> 663552 tetrahedra (interior "
                                        "vertices jittered +-0.05h), N=4 (Np=35), mode (1,1,1), 5-stage LSRK4 "
                                        "at the CFL step"),
}


def cpu_baseline(mesh, N, mode, min_seconds: float = 12.0, max_stages: int = 200):
    """The FP64 oracle as it stands, on this host's cores, over a bounded
    sample of the same workload: whole RK stages on the full mesh, repeated
    until about `min_seconds` of work (at most `max_stages` stages)."""
    import numpy as np

    import oracle
    from oracle.maxwell import LSRK4_A, LSRK4_B

    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    cores = min(threads, len(os.sched_getaffinity(0)))
    d = oracle.Discretization2D(mesh.vx, mesh.vy, mesh.elem_verts, N)
    op = oracle.Maxwell2D(d)
    dt = oracle.cfl_dt(d, N)
    q = oracle.cavity_mode_2d(d.x, d.y, 0.0, *mode)
    res = np.zeros_like(q)
    # one untimed stage, then the timed sample
    res = LSRK4_A[0] * res + dt * op.rhs(q)
    q = q + LSRK4_B[0] * res
    t0 = time.perf_counter()
    stages = 0
    while stages < max_stages and (time.perf_counter() - t0) < min_seconds:
        s = (stages + 1) % 5
        res = LSRK4_A[s] * res + dt * op.rhs(q)
        q = q + LSRK4_B[s] * res
        stages += 1
    el = time.perf_counter() - t0
    dofs = 3 * d.K * d.Np
    return {"value": dofs * stages / 5.0 / el, "unit": "DOF-updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{stages} LSRK4 stages (= {stages / 5:g} steps) of the FP64 NumPy oracle on the full "
                      f"{d.K}-element mesh, {el:.1f} s wall, BLAS threads {threads}"}


def recorded_traffic(kernel: str, K: int):
    """HBM bytes per launch of `kernel` at K elements from the committed
    rocprofv3 counter summary, or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))["kernels"][f"{kernel}@K={K}"]
        src = open(os.path.join(ROOT, rec["source_file"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_prefix"]:
        return None
    return rec["traffic_bytes"]


def serve_run(n_requests: int, seed: int = 4, mode: str = "burst", rate: float = 0.0, sequential: bool = False,
              max_chunk_steps: int = 0):
    """Run the serving mix (2D TM cavities: s ~ U{16..256}, N in {3,5,7},
    modes in 1..4, eps = 2.25 in a random disk, t_final ~ U[0.5, 2]) through
    the request server, or one request at a time through the plain FP32
    solver (sequential=True).  Returns latency percentiles and aggregate
    DOF-updates/s over the makespan."""
    import threading

    import numpy as np

    from paper_1304_5546_amd import dgw, inputs

    reqs = inputs.make_requests(n_requests, seed=seed)
    meshes = [inputs.request_mesh(r) for r in reqs]
    np_of = {3: 10, 5: 21, 7: 36}
    if sequential:
        t0 = time.perf_counter()
        dof = 0.0
        lat = []
        device_s = 0.0
        for r, m in zip(reqs, meshes):
            a = time.perf_counter()
            with dgw.Solver(m, r.order) as s:
                s.set_cavity_mode(*r.mode)
                n = s.advance(r.t_final)
                device_s += s.info()["solve_ms"] * 1e-3
                s.energy()
            dof += 3.0 * m.K * np_of[r.order] * n
            lat.append(time.perf_counter() - a)
            if len(lat) % 16 == 0:
                print(f"[serve] sequential: {len(lat)}/{n_requests} done", file=sys.stderr, flush=True)
        span = time.perf_counter() - t0
        return {"mode": "sequential plain FP32 solver", "requests": n_requests, "makespan_s": span,
                "dof_updates_per_s": dof / span, "device_s": device_s,
                "device_dof_updates_per_s": dof / device_s,
                "p50_solve_s": float(np.percentile(lat, 50)), "p99_solve_s": float(np.percentile(lat, 99))}
    arrivals = np.zeros(n_requests) if mode == "burst" else inputs.poisson_arrivals(n_requests, rate, seed + 1000)
    results = {}
    with dgw.Server(max_chunk_steps=max_chunk_steps) as srv:
        tickets = [None] * n_requests
        t0 = time.perf_counter()

        def submitter():
            for i, (r, m) in enumerate(zip(reqs, meshes)):
                wait = arrivals[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                tickets[i] = srv.submit(m, r.order, mode=r.mode, t_final=r.t_final)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for i, t in enumerate(tickets):
            results[i] = srv.wait(t)[0]
            if (i + 1) % 16 == 0:
                print(f"[serve] {mode}: {i + 1}/{n_requests} collected", file=sys.stderr, flush=True)
        span = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array([results[i]["t_finish"] - results[i]["t_arrival"] for i in range(n_requests)])
    queue = np.array([results[i]["t_start"] - results[i]["t_arrival"] for i in range(n_requests)])
    ok = sum(1 for i in results if results[i]["status"] == "DGW_OK")
    return {"mode": f"server, {mode} arrivals" + (f" at {rate:.3g} req/s" if mode != "burst" else ""),
            "requests": n_requests, "completed_ok": ok, "makespan_s": span,
            "dof_updates_per_s": st["dof_updates"] / span,
            "device_dof_updates_per_s": st["dof_updates"] / st["busy_s"],
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_queue_s": float(np.percentile(queue, 50)), "busy_s": st["busy_s"]}


def serving_leg(n: int):
    """Short serving leg for the default line: the first n requests of the
    seeded mix arriving at once (capacity), then the same requests with
    Poisson arrivals at 0.8 x that capacity (p50/p99 latency), then one at a
    time through the plain FP32 solver (device time of the same work)."""
    burst = serve_run(n)
    cap = burst["requests"] / burst["makespan_s"]
    pois = serve_run(n, mode="poisson", rate=0.8 * cap)
    seq = serve_run(n, sequential=True)
    return {"poisson": pois, "burst": burst, "sequential_fp32": seq,
            "capacity_vs_sequential": burst["dof_updates_per_s"] / seq["dof_updates_per_s"],
            "device_time_vs_sequential": burst["device_dof_updates_per_s"] / seq["device_dof_updates_per_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel", type=int, default=0,
                    help="2D stage kernel: 0 auto, 1 scalar-operand VALU, 2 fused-operand MFMA, 3 derivative-first MFMA, "
                         "4 element-major MFMA")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "split_bf16", "split_fp16", "fp64"],
                    help="arithmetic of the timed path (value and roofline)")
    ap.add_argument("--autotune", action="store_true",
                    help="time every kernel variant and launch shape first (dgw_autotune) and time the fastest")
    ap.add_argument("--serve", action="store_true", help="run the full serving configuration instead")
    ap.add_argument("--serve-n", type=int, default=256, help="requests in the full serving run")
    ap.add_argument("--serve-short", type=int, default=24,
                    help="requests in the short serving leg of the default line (0: none)")
    ap.add_argument("--variants", default=None,
                    help="comma-separated precision variants timed beside --prec, each with its L2 error at "
                         "t = 1 (default: fp32,split_bf16,split_fp16 in 2D, fp32,split_bf16 in 3D; 'none')")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB (a kernel of known "
                         "traffic, for calibrating HBM byte counters in a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; running the path across several GPUs "
                                   "(a halo exchange of face traces) is a design, not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.serve:
        # the full serving configuration: burst (capacity: `value`), then
        # Poisson arrivals at 0.8 x that capacity (p50/p99 latency), then the
        # same requests one at a time through the plain FP32 solver
        sv = serving_leg(args.serve_n)
        out = {"metric": METRIC, "value": sv["burst"]["dof_updates_per_s"], "unit": "DOF-updates/s",
               "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": f"serving: {args.serve_n} 2D TM cavity requests, s ~ U{{16..256}}, "
                                      "N in {3,5,7}, eps in {1, 2.25} by random disk, t_final ~ U[0.5, 2]",
                          "seed": 4},
               "p50_latency_s": sv["poisson"]["p50_latency_s"], "p99_latency_s": sv["poisson"]["p99_latency_s"],
               "serving": sv}
        print(json.dumps(out))
        return

    import torch

    from paper_1304_5546_amd import dgw, inputs

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    s_grid, seed, permute, N, mode, desc = CONFIGS[args.config]
    dim = 3 if len(mode) == 3 else 2
    if dim == 2:
        mesh = inputs.tri_grid(s_grid, seed=seed, permute=permute)
    else:
        mesh = inputs.tet_grid(s_grid, seed=seed, permute=permute)
    stream = torch.cuda.Stream()
    mode3 = (mode[0], mode[1], mode[2] if dim == 3 else 0)

    def timed(prec, to_t1=False):
        """Warm up, then time exactly args.steps steps on the solver's stream
        with HIP events recorded on that stream; the fields start from the
        device-initialised mode.  With to_t1 the solver first advances the
        mode to t = 1 at the CFL step (the accuracy run, error against the
        closed form returned) and the warm-up and timed steps follow it on
        the same solver without an idle gap."""
        solver = dgw.Solver(mesh, N, stream=stream, kernel=args.kernel, prec=prec)
        dt = solver.cfl_dt()
        solver.set_cavity_mode(*mode)
        t0, acc, q1 = 0.0, None, None
        if to_t1:
            # the fields at t = 1 are kept (one device copy) and their error
            # evaluated after the timed steps: the FP64 closed-form reduction
            # takes ~10 ms, a pause for the stage kernel
            if prec != "fp64":
                q1 = torch.empty(solver.shape, dtype=torch.float32, device="cuda")
            n1 = solver.advance(1.0)
            t0 = 1.0
            if q1 is None:
                acc = (solver.cavity_error(*mode3, 1.0), n1)
            else:
                solver.get_fields_dev(q1, stream)
                acc = n1
        solver.tune = solver.autotune() if args.autotune else None
        solver.launch_steps(args.warmup, dt, stream)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        solver.launch_steps(args.steps, dt, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        t_reached = t0 + (args.warmup + args.steps) * dt
        err = solver.cavity_error(*mode3, t_reached)
        log(f"{prec}: {args.steps} steps in {ms:.2f} ms ({ms / (5 * args.steps) * 1e3:.1f} us per stage)")
        if q1 is not None:
            solver.set_fields_dev(q1, stream)
            torch.cuda.synchronize()
            acc = (solver.cavity_error(*mode3, 1.0), acc)
            del q1
        if acc is not None:
            log(f"{prec}: t = 1 in {acc[1]} steps, rel L2 vs closed form {acc[0]:.3e}")
        solver.acc_t1 = acc
        return solver, dt, ms, t_reached, err

    log(f"{args.config}: K = {mesh.K}, N = {N}")
    if args.variants is None:
        vlist = ["fp32", "split_bf16", "split_fp16"] if dim == 2 else ["fp32", "split_bf16"]
    else:
        vlist = [] if args.variants == "none" else [v for v in args.variants.split(",") if v]
    # Each precision's accuracy run to t = 1 (thousands of steps) comes right
    # before its warm-up and timed steps, on the same solver, so that every
    # precision is timed in the sustained state of the GPU: after an idle gap
    # the stage kernels' duration swings by up to a third over the first ~100
    # launches while the clocks settle, which a 20-step window right after a
    # solver's set-up would catch.
    solver, dt, ms, t_reached, err = timed(args.prec, to_t1=args.prec in vlist)
    t1 = {args.prec: solver.acc_t1}
    bytes_per_launch, flops_per_launch = solver.stage_cost()
    dofs = solver.n_fields * solver.K * solver.Np
    value = dofs * args.steps / (ms * 1e-3)
    launch_s = ms * 1e-3 / (5 * args.steps)
    achieved = bytes_per_launch / launch_s / 1e9
    pcode = {"fp32": 0, "split_bf16": 1, "split_fp16": 2, "fp64": 3}[args.prec]
    sinfo = solver.info()
    variant = sinfo["kernel"]
    if dim == 3:
        kname = (f"stage3d_kernel<{N}, {'true' if pcode else 'false'}, "
                 f"{'false' if sinfo['wave_private'] else 'true'}>")
    elif pcode == 3:
        kname = f"stage2d_kernel<double, {N}, false>" if variant == 1 else f"stage2d_df_kernel<double, {N}, false, 1>"
    elif pcode:
        kname = f"stage2d_split_kernel<{N}, false, {pcode}>"
    else:
        kname = {1: f"stage2d_kernel<float, {N}, false>",
                 3: f"stage2d_df_kernel<float, {N}, false, {2 if sinfo['lane_elems'] == 2 else 1}>",
                 4: f"stage2d_em_kernel<{N}, false>"}.get(variant,
                                                                          f"stage2d_mfma_kernel<{N}, false, false>")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ["f32", "bf16x2+f32acc", "f16x2+f32acc", "f64"][pcode],
        "data": "synthetic",
        "config": {"workload": desc, "K": solver.K, "N": N, "Np": solver.Np, "dofs": dofs, "dt": dt,
                   "t_reached": t_reached, "precision": args.prec},
        "accuracy": {"rel_l2_vs_closed_form": err, "t": t_reached},
        "gflops_paper_model": flops_per_launch / launch_s / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(kname, solver.K),
                     "kernel": kname, "avg_launch_us": launch_s * 1e6,
                     "bytes_per_launch": bytes_per_launch},
    }
    if solver.tune:
        out["autotune"] = solver.tune
    solver.close()
    if vlist:
        # the same timed run for every precision variant, each with its
        # relative L2 error against the closed-form mode at t = 1
        var = {}
        for prec in vlist:
            if prec == args.prec:
                v_ms = ms
                e1, n1 = t1[prec]
            else:
                sv, _, v_ms, _, _ = timed(prec, to_t1=True)
                e1, n1 = sv.acc_t1
                sv.close()
            var[prec] = {"value": dofs * args.steps / (v_ms * 1e-3), "ms_per_step": v_ms / args.steps,
                         "us_per_stage": v_ms * 1e3 / (5 * args.steps),
                         "rel_l2_vs_closed_form_t1": e1, "steps_to_t1": n1}
        out["variants"] = var
    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": n * 4, "bytes_written": n * 4}
    if args.serve_short > 0:
        log(f"serving leg: {args.serve_short} requests")
        sv = serving_leg(args.serve_short)
        out["p50_latency_s"] = sv["poisson"]["p50_latency_s"]
        out["p99_latency_s"] = sv["poisson"]["p99_latency_s"]
        out["serving"] = sv
    if not args.no_cpu and dim == 2:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(mesh, N, mode)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
