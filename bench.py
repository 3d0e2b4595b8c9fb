"""Frequency-response benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mimo64]

A step is one pass of the whole path over one synthetic model: submit the
model with its frequency grid already resident in HBM (a device-memory
request), let the library reduce A to Hessenberg form, run every per-frequency
solve, and poll the result.  The throughput run keeps up to --window requests
in flight (each is still a full step with its own reduction); the latency
percentiles come from a second run with one request at a time.  The default workload is the 64-state, 4-input,
4-output model on 2000 log-spaced frequencies evaluated on the plain float64
path; the same workload is also timed on the refined float32 path and
reported beside it.

Printed: one JSON line with points/s (counting only points whose relative
error against the CPU oracle is <= 1e-10), per-step latency percentiles, the
roofline of the per-frequency sweep kernel (timed with HIP events inside
the library on the stream it runs on) and the CPU oracle timed
on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frequency-response points/sec at ≤1e-10 rel err (refined vs plain FP64); p50/p99 latency"
TOL = 1e-10
FP64_VALU_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PROFILES = os.path.join(ROOT, "profiles")


def sweep_flops_per_point(n: int, m: int, p: int) -> float:
    """Algorithmic flops of one frequency on the float64 path: the column
    rotations (14 flops per row per step, 7 n^2), the fused back-substitution
    (8 flops per row, step and right-hand side, 4 m n^2) and G = Ct^T X
    (4 n m p); O(n m) terms are left out."""
    return 7.0 * n * n + 4.0 * m * n * n + 4.0 * n * m * p


def sweep_kernel_family(n: int) -> tuple[str, list[str]]:
    """The sweep kernel the library launches for an n-state float64 request
    (with its default tiling) and the source files that define it."""
    common = ["sweep_common.h", "dpp.h", "lti_kernels.h"]
    if n <= 64:
        return "sweep16_kernel", ["sweep16.hip"] + common
    if n <= 256:
        return "sweep_kernel", ["sweep.hip"] + common
    return "sweep_wg_kernel", ["sweepwg.hip"] + common


def _source_digest(files: list[str]) -> str:
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_2401_04068_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic_record(workload: str, files: list[str], window: int):
    """HBM bytes per point swept, from committed rocprofv3 counter runs over
    every sweep dispatch of a bench run, used only while the kernel sources
    and the number of requests in flight (which decides how launches are
    formed) are the ones the counters were taken with."""
    path = os.path.join(PROFILES, f"sweep_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != _source_digest(files) or rec.get("window") != window:
        return None
    return rec.get("hbm_bytes_per_point")


# ------------------------------------------------------------------ CPU leg

def _oracle_chunk(args):
    A, B, C, D, w = args
    import oracle

    return oracle.freqresp(A, B, C, D, w)


def reference_points(mdl) -> np.ndarray:
    """Grid points the oracle checks: all of them while the dense solves stay
    cheap (K n^3 <= 1e9), else an evenly spread sample of 32."""
    if mdl.K * float(mdl.n) ** 3 <= 1e9:
        return np.arange(mdl.K)
    return np.unique(np.linspace(0, mdl.K - 1, 32).round().astype(int))


def cpu_baseline(mdl, idx, target_s: float = 12.0):
    """The oracle on this host's cores: the reference points split over a
    process pool (one single-threaded-BLAS worker per core, at most 16),
    repeated until about target_s seconds of wall time.  Returns (record,
    G_ref at idx)."""
    cores = min(16, os.cpu_count() or 1)
    K = len(idx)
    chunks = np.array_split(np.asarray(idx), cores)
    jobs = [(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega[c]) for c in chunks if len(c)]
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS")}
    os.environ["OPENBLAS_NUM_THREADS"] = "1"  # inherited by the spawned workers only
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        pool = ctx.Pool(len(jobs))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    with pool:
        pool.map(_oracle_chunk, jobs[:1])  # start-up
        t0 = time.perf_counter()
        reps = 0
        G_ref = None
        while True:
            parts = pool.map(_oracle_chunk, jobs)
            reps += 1
            if G_ref is None:
                G_ref = np.concatenate(parts)
            if time.perf_counter() - t0 >= target_s:
                break
        dt = time.perf_counter() - t0
    rec = {
        "value": reps * K / dt,
        "unit": "points/s",
        "cores": len(jobs),
        "kind": "oracle",
        "sample": f"{reps} passes over {K} points of the same model's grid "
                  f"({'all of it' if K == mdl.K else 'an evenly spread sample'}; "
                  f"dense complex LU per frequency, {len(jobs)} worker processes)",
    }
    return rec, G_ref


# ------------------------------------------------------------------ GPU leg

def _make_model(workload: str):
    from paper_2401_04068_amd import workloads as wl

    if workload == "mimo64":
        return wl.mimo64()
    if workload == "siso8":
        return wl.siso8()
    if workload == "damped256":
        return wl.damped256_model(0)
    if workload == "large1024":
        return wl.large1024_models(seeds=wl.LARGE_SEEDS[:1])[0]
    raise SystemExit(f"unknown workload {workload}")


def run_gpu(mdl, precision: int, steps: int, warmup: int, window: int):
    """Time `steps` device-memory requests of one model (each its own
    reduction and all its solves).  Throughput run: up to `window` requests
    in flight (each has its own output buffers; a new one is submitted as the
    oldest completes).  Latency run: the same number of requests one at a
    time, submit -> results visible."""
    import torch

    from paper_2401_04068_amd import binding

    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(mdl, k))).to(dev) for k in ("A", "B", "C", "D", "omega")}
    W = max(1, window)
    Gs = [torch.empty((mdl.K, mdl.p, mdl.m, 2), dtype=torch.float64, device=dev) for _ in range(W)]
    infos = [torch.empty((mdl.K * 8,), dtype=torch.uint8, device=dev) for _ in range(W)]
    eng = binding.Engine(arena_bytes=1 << 30, kernel_timing=True)
    try:
        def submit(slot):
            return eng.submit_device(t["A"], t["B"], t["C"], t["D"], t["omega"], Gs[slot], infos[slot],
                                     precision=precision)

        def pipelined(n):
            inflight = []
            t_last = time.perf_counter()
            for i in range(n):
                if len(inflight) == W:
                    eng.wait(inflight.pop(0))
                inflight.append(submit(i % W))
                if time.perf_counter() - t_last > 5.0:  # long steps: show progress
                    print(f"bench: step {i} of {n} submitted", file=sys.stderr, flush=True)
                    t_last = time.perf_counter()
            for h in inflight:
                eng.wait(h)

        pipelined(warmup)
        torch.cuda.synchronize()
        s0 = eng.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pipelined(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = eng.stats()
        torch.cuda.synchronize()
        # every output buffer of the throughput run (the last request of
        # each slot), checked against the oracle in main()
        Gall = []
        for g in Gs[:min(W, steps)]:
            gh = g.cpu().numpy()
            Gall.append(gh[..., 0] + 1j * gh[..., 1])
        infoh = infos[0].cpu().numpy().view(binding.POINT_INFO_DTYPE)
    finally:
        eng.close()
    # latency: one request at a time, on an engine without kernel-timing
    # events (a user's configuration)
    lat = []
    with binding.Engine(arena_bytes=1 << 30) as eng2:
        for i in range(warmup + steps):
            a = time.perf_counter()
            eng2.wait(eng2.submit_device(t["A"], t["B"], t["C"], t["D"], t["omega"], Gs[0], infos[0],
                                         precision=precision))
            if i >= warmup:
                lat.append(time.perf_counter() - a)
    launches = s1["timed_sweep_launches"] - s0["timed_sweep_launches"]
    sweep_ms = (s1["sweep_kernel_ms"] - s0["sweep_kernel_ms"]) / max(launches, 1)
    rlaunch = s1["timed_reduce_launches"] - s0["timed_reduce_launches"]
    reduce_ms = (s1["reduce_kernel_ms"] - s0["reduce_kernel_ms"]) / max(rlaunch, 1)
    return {
        "seconds": dt,
        "lat": np.array(lat),
        "sweep_ms_per_launch": sweep_ms,
        "sweep_launches_per_step": launches / steps,
        "reduce_ms_per_launch": reduce_ms,
        "reductions_per_step": (s1["reductions"] - s0["reductions"]) / steps,
        "G": Gall[0],
        "G_all": Gall,
        "info": infoh,
    }


def serving(args):
    """Serving replay: the mixed-size request stream (n ~ U{4..128},
    m, p ~ U{1..8}, K ~ U{256..4096}) submitted from host memory on the refined
    path.  Open loop: each request is submitted at its Poisson arrival time
    (2000 requests/s) and its latency runs from that arrival to the moment its
    results are visible to poll().  Closed loop: all requests submitted at
    once; throughput = points / (first submit -> last result)."""
    import torch  # noqa: F401  (device memory for the arena)

    import oracle
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    nreq = args.requests
    reqs = wl.serving_requests(nreq)
    arrivals = wl.serving_arrivals(nreq)
    total_points = sum(r.K for r in reqs)
    out = {"metric": METRIC, "workload": f"serving: {nreq} requests, Poisson 2000/s, refined path, host memory",
           "requests": nreq, "points": total_points}
    with binding.Engine(arena_bytes=8 << 30, host_staging_bytes=1 << 30) as eng:
        # warm-up (kernel loading, pools)
        for r in reqs[:8]:
            eng.wait(eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=binding.PREC_REFINED))
        # open loop
        handles = []
        t0 = time.perf_counter()
        for r, ta in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            lag = max(0.0, time.perf_counter() - t0 - ta)  # submission behind the arrival
            handles.append((eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=binding.PREC_REFINED), lag))
        lat = []
        for h, _ in handles:
            eng.wait(h)
        for h, lag in handles:
            # arrival -> results visible: submission lag plus the library's
            # submit -> done interval (both stamps on the library clock)
            lat.append(lag + (h.result["t_done_us"] - h.result["t_submit_us"]) * 1e-6)
        t_open = time.perf_counter() - t0

        def pct(x):
            x = np.asarray(x) * 1e3
            return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "max": float(x.max())}

        res = [h.result for h, _ in handles]
        work = np.array([r.K * r.n * r.n * (r.m + 2) for r in reqs], dtype=float)
        small = work <= np.median(work)
        lat_a = np.array(lat)
        out["open_loop"] = {
            "wall_s": t_open,
            "points_per_s": total_points / t_open,
            "latency_ms": pct(lat),
            # where the time goes: waiting for admission, admission to first
            # sweep launch, first launch to results visible
            "queue_ms": pct([(x["t_admit_us"] - x["t_submit_us"]) * 1e-6 for x in res]),
            "start_ms": pct([(x["t_first_launch_us"] - x["t_admit_us"]) * 1e-6 for x in res]),
            "run_ms": pct([(x["t_done_us"] - x["t_first_launch_us"]) * 1e-6 for x in res]),
            "latency_ms_smaller_half": pct(lat_a[small]),
            "latency_ms_larger_half": pct(lat_a[~small]),
        }
        open_handles = [h for h, _ in handles]
        # closed loop
        t0 = time.perf_counter()
        hs = [eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=binding.PREC_REFINED) for r in reqs]
        for h in hs:
            eng.wait(h)
        t_closed = time.perf_counter() - t0
        st = eng.stats()
    # accuracy on a sample: every 64th request, every 61st point, against the oracle
    worst = 0.0
    n_fb = 0
    for idx in range(0, nreq, 64):
        r = reqs[idx]
        sub = slice(None, None, 61)
        ref = oracle.freqresp(r.A, r.B, r.C, r.D, r.omega[sub])
        for G in (open_handles[idx].G, hs[idx].G):
            worst = max(worst, float(oracle.rel_err(G[sub], ref).max()))
    for h in hs:
        n_fb += int(h.result["n_fallback"])
    out["closed_loop"] = {"wall_s": t_closed, "points_per_s": total_points / t_closed}
    out["accuracy_sample_max_rel_err"] = worst
    out["fallback_points"] = n_fb
    out["stats"] = {k: st[k] for k in ("reductions", "sweep_launches", "tiles_launched", "arena_peak_bytes")}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="mimo64", choices=["mimo64", "siso8", "damped256", "large1024", "serving"])
    ap.add_argument("--requests", type=int, default=4096, help="serving replay: number of requests")
    ap.add_argument("--window", type=int, default=16,
                    help="requests in flight in the throughput run (each step is still one full request)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--paths", default="both", choices=["both", "fp64", "refined"],
                    help="which precision paths to time (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this engine's work units are independent "
              "and its multi-GPU sharding is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        serving(args)
        return
    mdl = _make_model(args.workload)
    n, m, p, K = mdl.n, mdl.m, mdl.p, mdl.K

    ref_idx = reference_points(mdl)
    # The CPU leg runs first, before anything touches the GPU, so that its
    # worker processes start from a process with no device state.
    if args.no_cpu:
        import oracle

        G_ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega[ref_idx])
        cpu = None
    else:
        cpu, G_ref = cpu_baseline(mdl, ref_idx)

    import torch

    from paper_2401_04068_amd import binding

    binding.load()
    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fp64 = ref = None
    if args.paths in ("both", "fp64"):
        fp64 = run_gpu(mdl, binding.PREC_FP64, args.steps, args.warmup, args.window)
    if args.paths in ("both", "refined"):
        ref = run_gpu(mdl, binding.PREC_REFINED, args.steps, args.warmup, args.window)
    if fp64 is None or ref is None:
        done = fp64 or ref
        print(json.dumps({"profiling_run": args.paths, "ms_per_step": 1e3 * done["seconds"] / args.steps,
                          "sweep_ms_per_launch": done["sweep_ms_per_launch"]}), flush=True)
        return

    import oracle

    # the worst point over every output buffer of the throughput run
    err64 = np.max([oracle.rel_err(g[ref_idx], G_ref) for g in fp64["G_all"]], axis=0)
    err32 = np.max([oracle.rel_err(g[ref_idx], G_ref) for g in ref["G_all"]], axis=0)
    ok64 = float(np.mean(err64 <= TOL))
    ok32 = float(np.mean(err32 <= TOL))

    pts64 = K * args.steps / fp64["seconds"]
    pts32 = K * args.steps / ref["seconds"]
    if fp64["reductions_per_step"] != 1.0 or ref["reductions_per_step"] != 1.0:
        raise RuntimeError("every step must reduce its own model exactly once")
    value = pts64 * ok64
    # a launch (one batch of the sweep stream) may carry the tiles of several
    # requests in flight
    flops_launch = sweep_flops_per_point(n, m, p) * K / max(fp64["sweep_launches_per_step"], 1e-9)
    achieved = flops_launch / (fp64["sweep_ms_per_launch"] * 1e-3) / 1e12
    kname, kfiles = sweep_kernel_family(n)
    bpp = _traffic_record(args.workload, kfiles, args.window)
    traffic = None if bpp is None else bpp * K / max(fp64["sweep_launches_per_step"], 1e-9)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * fp64["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: n={n}, m={m}, p={p}, K={K} log-spaced frequencies, "
                        f"one model per step (its own reduction), up to {args.window} requests in flight, "
                        "inputs resident in HBM, float64 path",
            "n": n, "m": m, "p": p, "points_per_step": K, "requests_in_flight": args.window,
            "reductions_per_step": fp64["reductions_per_step"],
        },
        "latency_ms": {  # one request alone: submit -> results visible
            "p50": float(np.percentile(fp64["lat"], 50) * 1e3),
            "p99": float(np.percentile(fp64["lat"], 99) * 1e3),
        },
        "accuracy": {"max_rel_err": float(err64.max()), "frac_within_1e-10": ok64},
        "refined": {
            "points_per_s": pts32 * ok32,
            "points_per_s_raw": pts32,
            "max_rel_err": float(err32.max()),
            "frac_within_1e-10": ok32,
            "ms_per_step": 1e3 * ref["seconds"] / args.steps,
            "latency_ms": {"p50": float(np.percentile(ref["lat"], 50) * 1e3),
                           "p99": float(np.percentile(ref["lat"], 99) * 1e3)},
            "mean_fp32_solves": float(np.mean(ref["info"]["iters"])),
            "sweep_ms_per_launch": ref["sweep_ms_per_launch"],
            "vs_fp64": (pts32 * ok32) / value if value else None,
        },
        "kernels": {
            "sweep_ms_per_launch": fp64["sweep_ms_per_launch"],
            "sweep_launches_per_step": fp64["sweep_launches_per_step"],
            "reduce_ms_per_launch": fp64["reduce_ms_per_launch"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": f"{kname}<fp64> (per-frequency Givens sweep)",
            "kernel_source_sha256_16": _source_digest(kfiles),
            "flops_per_launch": flops_launch,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
