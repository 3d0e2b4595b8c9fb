"""Frequency-response benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload serving]

Default workload (the configuration the metric is quoted on): the serving
mix of 4096 requests, each its own model with n ~ U{4..128} states,
m, p ~ U{1..8}, K ~ U{256..4096} log-spaced frequencies in [1e-3, 1e3]
(8.9 M points in all), on the refined path (complex-float32 solves with
float64 Hessenberg reduction and float64 refinement to 1e-10) and, beside it,
on the plain float64 path.

A step is one closed-loop pass of the whole hot path over the whole mix: all
4096 requests submitted through the C ABI with their inputs already resident
in HBM (device-memory requests), each reduced to Hessenberg form and solved
at every frequency, and every result polled.  W untimed steps, then K timed
steps.  `value` = refined points/s times the fraction of sampled points whose
error against the CPU oracle is <= 1e-10.  Also reported:

* the plain float64 path on the same mix (`fp64`), and refined / float64;
* open-loop serving latency: the requests replayed from host memory at their
  Poisson arrival times (2000 requests/s), arrival -> results visible,
  p50/p99 (`latency_ms`);
* the PCIe-inclusive closed-loop rate (host-memory requests: H2D and D2H in
  the timed region), which is never `value`;
* `roofline`: the kernel family that dominates the refined run's kernel
  time, its algorithmic flops over its HIP-event time (events recorded by the
  library on the stream the kernels run on), against the peak of the
  arithmetic it does (float32 and float64 vector FMA);
* `cpu_baseline`: the oracle (dense complex LU per point) on this host's
  cores over a sample of the same mix;
* `secondary`: the 64-state model (2000 points), the 1024-state model (ten
  10,000-point queries, two of them repeats), and the 512 lightly damped
  256-state models (4096 points each), one pass each.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frequency-response points/sec at ≤1e-10 rel err (refined vs plain FP64); p50/p99 latency"
TOL = 1e-10
# Vector peaks of the MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x
# 2.4 GHz = 78.6 TFLOP/s in float64; twice that in float32 (the chip's
# published 157.3 TFLOP/s vector float32 rate)
FP64_VALU_PEAK = 78.6
FP32_VALU_PEAK = 157.3
PROFILES = os.path.join(ROOT, "profiles")
# kernel families (the library's LTI_KF_* numbers); the sweep phase of a
# batch runs SWEEP_FAMILIES, the double-double refinement follows it
KF_NAMES = {0: "sweep16_kernel (four frequencies per wavefront, n <= 64)",
            5: "sweep32_kernel (two frequencies per wavefront, 64 < n <= 128)",
            1: "sweep_kernel (one frequency per wavefront, n <= 256)",
            2: "sweep_wg_kernel (one frequency per workgroup, n <= 1024)",
            3: "refine_dd_kernel (double-double refinement)"}
SWEEP_FAMILIES = [0, 5, 1, 2]
KF_COUNT = 6
SWEEP_SOURCES = ["sweep16.hip", "sweep.hip", "sweepwg.hip", "sweep_common.h", "dpp.h", "lti_kernels.h"]


def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def family_of(n: int, m: int, p: int) -> int:
    """Kernel family the library runs a request on (state-space model, the
    library's default knobs)."""
    if n <= 64:
        return 0
    if n <= 128:
        return 5
    return 1 if n <= 256 else 2


def solve_flops(n: int, m: int, p: int) -> float:
    """Algorithmic flops of one point's solve with m right-hand sides and p
    outputs: the column rotations (14 flops per row and step, 7 n^2), the
    fused back-substitution (8 flops per row, step and right-hand side,
    4 m n^2) and G = (CQ) X (4 n m p)."""
    return 7.0 * n * n + 4.0 * m * n * n + 4.0 * n * m * p


def point_flops(n: int, m: int, p: int, iters: np.ndarray, refined: bool):
    """(float32 flops, float64 flops) of a request's points.  The library
    solves the transposed system when p < m, so m here is min(m, p).
    Refined: `iters` float32 sweeps (7 n^2 + 4 m n^2 each), iters - 1 float64
    residuals (2 m n^2: the real Hessenberg H times complex X) and the float64
    output (4 n m p)."""
    ms, ps = min(m, p), max(m, p)
    if not refined:
        return 0.0, float(len(iters)) * solve_flops(n, ms, ps)
    it = iters.astype(np.float64)
    f32 = float(np.sum(it)) * (7.0 * n * n + 4.0 * ms * n * n)
    f64 = float(np.sum(it - 1.0)) * 2.0 * ms * n * n + len(iters) * 4.0 * n * ms * ps
    return f32, f64


def _source_digest(files: list[str]) -> str:
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_2401_04068_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic_record(name: str, files: list[str]):
    """HBM bytes per point of a kernel family on a workload, from committed
    rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE), used only while the
    kernel sources are the ones the counters were taken with."""
    path = os.path.join(PROFILES, f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != _source_digest(files):
        return None
    return rec.get("hbm_bytes_per_point")


def host_description() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name', '?')} {b.get('version', '?')} ({b.get('openblas configuration', '')})".strip()
    except Exception:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "blas": blas}


# ------------------------------------------------------------------ CPU leg

def _oracle_job(args):
    A, B, C, D, w = args
    import oracle

    return oracle.freqresp(A, B, C, D, w)


def _pool(cores: int):
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS")}
    os.environ["OPENBLAS_NUM_THREADS"] = "1"  # inherited by the spawned workers only
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        return ctx.Pool(cores)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def cpu_oracle(jobs, target_s: float, what: str, timed: bool = True):
    """The oracle over `jobs` (lists of (A, B, C, D, omega)) on a process pool
    of single-threaded-BLAS workers (one per core, at most 16), repeated until
    about target_s seconds of wall time.  Returns (record or None, results)."""
    cores = min(16, os.cpu_count() or 1)
    npts = sum(len(j[4]) for j in jobs)
    with _pool(cores) as pool:
        pool.map(_oracle_job, jobs[:cores])  # start-up
        t0 = time.perf_counter()
        reps = 0
        out = None
        while True:
            res = pool.map(_oracle_job, jobs, chunksize=max(1, len(jobs) // (4 * cores)))
            reps += 1
            if out is None:
                out = res
            if not timed or time.perf_counter() - t0 >= target_s:
                break
        dt = time.perf_counter() - t0
    if not timed:
        return None, out
    rec = {"value": reps * npts / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": f"{reps} passes over {npts} points ({what}); dense complex LU per point "
                     f"(numpy.linalg.solve), {cores} single-threaded worker processes"}
    rec.update(host_description())
    return rec, out


# ------------------------------------------------------------------ GPU helpers

def _stats_delta(s0, s1):
    return {
        "family_ms": [b - a for a, b in zip(s0["family_ms"], s1["family_ms"])],
        "family_launches": [b - a for a, b in zip(s0["family_launches"], s1["family_launches"])],
        "reductions": s1["reductions"] - s0["reductions"],
        "reduce_kernel_ms": s1["reduce_kernel_ms"] - s0["reduce_kernel_ms"],
        "timed_reduce_launches": s1["timed_reduce_launches"] - s0["timed_reduce_launches"],
        "sweep_launches": s1["sweep_launches"] - s0["sweep_launches"],
        "sweep_kernel_ms": s1["sweep_kernel_ms"] - s0["sweep_kernel_ms"],
        "timed_sweep_launches": s1["timed_sweep_launches"] - s0["timed_sweep_launches"],
    }


def _pct(x):
    x = np.asarray(x, dtype=np.float64) * 1e3
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "max": float(x.max())}


class DeviceMix:
    """A list of models with their inputs, outputs and point records resident
    in HBM, submitted as device-memory requests."""

    def __init__(self, models, dev):
        import torch

        self.models = models
        self.t = []
        for mdl in models:
            d = {k: torch.from_numpy(np.ascontiguousarray(getattr(mdl, k))).to(dev)
                 for k in ("A", "B", "C", "D", "omega")}
            d["G"] = torch.empty((mdl.K, mdl.p, mdl.m, 2), dtype=torch.float64, device=dev)
            d["info"] = torch.empty((mdl.K * 8,), dtype=torch.uint8, device=dev)
            self.t.append(d)

    def run(self, eng, precision, keys=None):
        hs = []
        for i, d in enumerate(self.t):
            key = 0 if keys is None else keys[i]
            hs.append(eng.submit_device(d["A"], d["B"], d["C"], d["D"], d["omega"], d["G"], d["info"],
                                        precision=precision, model_key=key))
        for h in hs:
            eng.wait(h)
        return hs

    def G(self, i, idx=None):
        g = self.t[i]["G"].cpu().numpy()
        g = g[..., 0] + 1j * g[..., 1]
        return g if idx is None else g[idx]

    def info(self, i):
        from paper_2401_04068_amd import binding

        return self.t[i]["info"].cpu().numpy().view(binding.POINT_INFO_DTYPE)


def timed_steps(eng, mix, precision, steps, warmup, label):
    import torch

    for i in range(warmup):
        mix.run(eng, precision)
    torch.cuda.synchronize()
    s0 = eng.stats()
    t0 = time.perf_counter()
    last = time.perf_counter()
    for i in range(steps):
        hs = mix.run(eng, precision)
        if time.perf_counter() - last > 10.0:
            log(f"{label}: step {i + 1} of {steps}")
            last = time.perf_counter()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = eng.stats()
    return dt, _stats_delta(s0, s1), hs


def roofline_of(delta, fam_flops, fp32: bool):
    """The sweep phase of a batch (the launches of every sweep kernel class of
    the batch, spread over the sweep streams and timed by the library as the
    union of the batches' intervals): algorithmic flops per batch over the
    average phase time, against the vector peak of the arithmetic done."""
    f32 = sum(fam_flops[f][0] for f in SWEEP_FAMILIES)
    f64 = sum(fam_flops[f][1] for f in SWEEP_FAMILIES)
    launches = max(delta["timed_sweep_launches"], 1)
    t = delta["sweep_kernel_ms"] * 1e-3
    achieved = (f32 + f64) / t / 1e12
    # time the same work would take at the peak rates of its two parts
    t_peak = (f32 / FP32_VALU_PEAK + f64 / FP64_VALU_PEAK) / 1e12
    peak = (f32 + f64) / t_peak / 1e12 if t_peak > 0 else FP64_VALU_PEAK
    return {
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": t_peak / t,
        "traffic": None,
        "kernel": "sweep phase of a batch: " + "; ".join(KF_NAMES[f] for f in SWEEP_FAMILIES),
        "kernel_source_sha256_16": _source_digest(SWEEP_SOURCES),
        "flops_per_launch": (f32 + f64) / launches,
        "fp32_share": f32 / max(f32 + f64, 1.0),
        "avg_launch_ms": delta["sweep_kernel_ms"] / launches,
        "launches": launches,
        "peak_note": ("float64 FMA at 78.6 TFLOP/s, float32 FMA at the chip's 157.3 TFLOP/s vector rate "
                      "(blended by the kernel's flop mix)" if fp32 else "float64 FMA, 78.6 TFLOP/s"),
        # the library is compiled without packed float32 instructions, so its
        # float32 FMAs issue at the float64 rate: the rate this code can reach
        "frac_of_unpacked_peak": achieved / FP64_VALU_PEAK,
    }


# ------------------------------------------------------------------ headline

def serving_headline(args, out):
    import torch

    import oracle
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    N = args.requests
    t_gen = time.perf_counter()
    reqs = wl.serving_requests(N)
    arrivals = wl.serving_arrivals(N)
    total = int(sum(r.K for r in reqs))
    log(f"serving mix: {N} requests, {total} points (generated in {time.perf_counter() - t_gen:.1f} s)")
    # accuracy / CPU sample: every 16th request, every 8th point of it
    samp = list(range(0, N, 16))
    sidx = {i: np.arange(0, reqs[i].K, 8) for i in samp}
    jobs = [(reqs[i].A, reqs[i].B, reqs[i].C, reqs[i].D, reqs[i].omega[sidx[i]]) for i in samp]
    npts_s = sum(len(v) for v in sidx.values())
    cpu, refs = cpu_oracle(jobs, 12.0, f"every 16th request of the mix, every 8th point of each",
                           timed=not args.no_cpu)
    G_ref = dict(zip(samp, refs))
    log(f"cpu leg done ({npts_s} sampled points)")

    dev = torch.device("cuda:0")
    binding.load()
    mix = DeviceMix(reqs, dev)
    torch.cuda.synchronize()
    res = {}
    with binding.Engine(arena_bytes=8 << 30, kernel_timing=True, host_staging_bytes=1 << 30) as eng:
        for name, prec in (("refined", binding.PREC_REFINED), ("fp64", binding.PREC_FP64)):
            dt, delta, hs = timed_steps(eng, mix, prec, args.steps, args.warmup, name)
            worst, ok, n = 0.0, 0, 0
            for i in samp:
                e = oracle.rel_err(mix.G(i, sidx[i]), G_ref[i])
                worst = max(worst, float(e.max()))
                ok += int(np.sum(e <= TOL))
                n += len(e)
            fam_flops = [[0.0, 0.0] for _ in range(KF_COUNT)]
            paths = np.zeros(5, dtype=np.int64)
            for i, r in enumerate(reqs):
                info = mix.info(i)
                f32, f64 = point_flops(r.n, r.m, r.p, info["iters"], prec == binding.PREC_REFINED)
                f = family_of(r.n, r.m, r.p)
                fam_flops[f][0] += f32 * args.steps
                fam_flops[f][1] += f64 * args.steps
                paths += np.bincount(info["path"], minlength=5)[:5]
            res[name] = {
                "seconds": dt, "points_per_s_raw": total * args.steps / dt, "frac_within_1e-10": ok / n,
                "max_rel_err": worst, "delta": delta, "fam_flops": fam_flops, "paths": paths.tolist(),
                "mean_fp32_solves": None,
            }
            if prec == binding.PREC_REFINED:
                it = np.concatenate([mix.info(i)["iters"] for i in range(0, N, 8)])
                res[name]["mean_fp32_solves"] = float(np.mean(it))
            log(f"{name}: {res[name]['points_per_s_raw'] / 1e6:.2f} M points/s, max err {worst:.2e}")
        del mix
        torch.cuda.empty_cache()
        # open loop: host-memory requests at their Poisson arrival times.  The
        # trace is replayed three times and the last replay reported (p50 and
        # p99 of every replay beside it).
        # result buffers reused by every replay, as a server reuses its own:
        # allocated and written once here, so that no replay takes page faults
        # on first touch of 2.9 GB of fresh result arrays
        outs = []
        for r in reqs:
            g = np.empty((r.K, r.p, r.m), dtype=np.complex128)
            inf = np.empty(r.K, dtype=binding.POINT_INFO_DTYPE)
            g.fill(0)
            inf.view(np.uint8).fill(0)
            outs.append((g, inf))

        def replay():
            handles = []
            t0 = time.perf_counter()
            for r, ta, o in zip(reqs, arrivals, outs):
                now = time.perf_counter() - t0
                if ta > now:
                    time.sleep(ta - now)
                lag = max(0.0, time.perf_counter() - t0 - ta)
                handles.append((eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=binding.PREC_REFINED, out=o),
                                lag))
            for h, _ in handles:
                eng.wait(h)
            t_open = time.perf_counter() - t0
            lat = [lag + (h.result["t_done_us"] - h.result["t_submit_us"]) * 1e-6 for h, lag in handles]
            rs = [h.result for h, _ in handles]
            return {
                "wall_s": t_open,
                "latency_ms": _pct(lat),
                "submit_lag_ms": _pct([lag for _, lag in handles]),
                "queue_ms": _pct([(x["t_admit_us"] - x["t_submit_us"]) * 1e-6 for x in rs]),
                "run_ms": _pct([(x["t_done_us"] - x["t_first_launch_us"]) * 1e-6 for x in rs]),
            }

        # the submitting thread's own pauses count as latency (submit_lag);
        # Python's cyclic collector, which a replay's allocations trigger and
        # which walks every live object of the process, is held off meanwhile
        gc.collect()
        gc.disable()
        try:
            replays = [replay() for _ in range(3)]
        finally:
            gc.enable()
        del outs
        open_loop = replays[-1]
        open_loop["first_replay"] = replays[0]
        open_loop["p50_p99_ms_of_each_replay"] = [[x["latency_ms"]["p50"], x["latency_ms"]["p99"]] for x in replays]
        # closed loop from host memory (H2D and D2H inside the timed region),
        # twice: the first pass's result arrays are fresh allocations whose
        # pages the library's result copies touch first (page faults taken
        # on the thread that copies, about 0.5 s for the mix's 2.9 GB of
        # results); the second pass is reported
        t_host_first = None
        for _ in range(2):
            hs = None
            t0 = time.perf_counter()
            hs = [eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=binding.PREC_REFINED) for r in reqs]
            for h in hs:
                eng.wait(h)
            t_host = time.perf_counter() - t0
            if t_host_first is None:
                t_host_first = t_host
        worst_h = 0.0
        for i in samp[::4]:
            worst_h = max(worst_h, float(oracle.rel_err(hs[i].G[sidx[i]], G_ref[i]).max()))
        del hs
        # kernel time of each family over everything this engine ran (both
        # precisions, warm-up, timed steps and replays): the figure a kernel
        # trace of the same command sums to
        s_end = eng.stats()
        engine_totals = {"sweep_phase_ms": s_end["sweep_kernel_ms"], "sweep_batches": s_end["timed_sweep_launches"],
                         "family_ms": s_end["family_ms"], "family_launches": s_end["family_launches"]}
    log("serving replays done")

    ref, f64 = res["refined"], res["fp64"]
    value = ref["points_per_s_raw"] * ref["frac_within_1e-10"]
    v64 = f64["points_per_s_raw"] * f64["frac_within_1e-10"]
    roof = roofline_of(ref["delta"], ref["fam_flops"], fp32=True)
    bpp = _traffic_record("sweep_serving", SWEEP_SOURCES)
    per_launch = total * args.steps / max(ref["delta"]["timed_sweep_launches"], 1)
    roof["traffic"] = None if bpp is None else bpp * per_launch
    roof["traffic_bytes_per_point"] = bpp
    roof["points_per_launch"] = per_launch
    roof64 = roofline_of(f64["delta"], f64["fam_flops"], fp32=False)

    def fam_table(r):
        """Flops of each sweep family (their launches overlap, so only the
        whole sweep phase is timed) and the refinement kernel's time."""
        d = r["delta"]
        rows = {}
        for f in SWEEP_FAMILIES:
            f32, fl64 = r["fam_flops"][f]
            if f32 + fl64 > 0:
                rows[KF_NAMES[f].split(" ")[0]] = {"gflop_per_step": (f32 + fl64) / args.steps / 1e9}
        rows["sweep_phase"] = {"ms": d["sweep_kernel_ms"], "batches": d["timed_sweep_launches"]}
        rows["refine_dd_kernel"] = {"ms": d["family_ms"][3], "launches": d["family_launches"][3]}
        return rows

    out.update({
        "value": value,
        "ms_per_step": 1e3 * ref["seconds"] / args.steps,
        "dtype": "c32+f64",
        "config": {
            "workload": f"serving mix: {N} requests (one model each), n~U{{4..128}}, m,p~U{{1..8}}, "
                        f"K~U{{256..4096}} log-spaced w in [1e-3,1e3], {total} points per step; "
                        "refined path (complex-float32 solves, float64 reduction and refinement to 1e-10); "
                        "inputs resident in HBM; one step = all requests submitted and completed",
            "requests": N, "points_per_step": total,
        },
        "accuracy": {"max_rel_err": ref["max_rel_err"], "frac_within_1e-10": ref["frac_within_1e-10"],
                     "sampled_points": npts_s, "oracle": "float64 dense LU per point"},
        "latency_ms": open_loop["latency_ms"],
        "refined": {"points_per_s": value, "points_per_s_raw": ref["points_per_s_raw"],
                    "mean_fp32_solves": ref["mean_fp32_solves"], "points_by_path": ref["paths"],
                    "kernels": fam_table(ref),
                    "reductions_per_step": ref["delta"]["reductions"] / args.steps},
        "fp64": {"points_per_s": v64, "points_per_s_raw": f64["points_per_s_raw"],
                 "max_rel_err": f64["max_rel_err"], "frac_within_1e-10": f64["frac_within_1e-10"],
                 "ms_per_step": 1e3 * f64["seconds"] / args.steps, "points_by_path": f64["paths"],
                 "kernels": fam_table(f64), "roofline": roof64},
        "refined_vs_fp64": value / v64 if v64 else None,
        "open_loop": open_loop,
        "pcie_inclusive": {"points_per_s": total / t_host, "wall_s": t_host, "sampled_max_rel_err": worst_h,
                           "first_pass": {"points_per_s": total / t_host_first, "wall_s": t_host_first},
                           "note": "host-memory requests, all submitted at once: H2D and D2H inside; second "
                                   "of two passes (the first touches fresh result arrays)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "engine_kernel_totals": engine_totals,
    })


# ------------------------------------------------------------------ secondary

def secondary(args, out):
    import torch

    dev = torch.device("cuda:0")
    sec = {}
    want = (lambda name: True) if not args.only else (lambda name: name == args.only)
    if want("mimo64"):
        _mimo64(args, sec, dev)
    if want("large1024"):
        _large1024(args, sec)
    if want("damped256"):
        _damped256(args, sec)
    if want("imdp"):
        _imdp(args, sec)
    out["secondary"] = sec


def _imdp(args, sec):
    """The paper's own method at the shape of its largest benchmark model
    (42,634 states x 3 actions, 48.1 M transitions; synthetic stand-in):
    200 iterations of finite-horizon maximal pessimistic reachability, the
    query of its computational study."""
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    t0 = time.perf_counter()
    m = wl.imdp_pimdp2_shape()
    log(f"imdp: {m.n_states} states, {m.n_columns} columns, {m.nnz} transitions "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    with binding.IMDPSolver(m.n_states, m.stateptr, m.colptr, m.rowval, m.lower, m.upper) as sol:
        sol.run(horizon=5, targets=m.targets)
        K = 200
        t0 = time.perf_counter()
        V, it, res, pol, kms = sol.run(horizon=K, targets=m.targets)
        wall = time.perf_counter() - t0
    # algorithmic HBM bytes per iteration: per transition rowval (4), lower
    # (8), gap (8); per column colptr (4), 1 - sum lower (8), sum of gaps (8),
    # threshold position (4); per state stateptr (4), the list entry (4), held
    # value (8), V_k written (8), policy (4), V_{k-1} read once (8: the vector
    # stays in L2 for the gathers)
    bpi = m.nnz * 20 + m.n_columns * 24 + m.n_states * 36
    achieved = bpi * it / (kms * 1e-3) / 1e9
    sec["imdp"] = {
        "workload": "synthetic interval MDP of the paper's largest benchmark shape: 42,634 states x 3 actions, "
                    f"{m.nnz} transitions; {K} iterations of finite-horizon max-pessimistic reachability",
        "iterations": it, "kernel_ms": kms, "wall_s": wall, "ms_per_iteration": kms / it,
        "transitions_per_s": m.nnz * it / (kms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "bytes_per_iteration": bpi},
        "v_range": [float(V.min()), float(V.max())], "residual": res,
        "paper_context": "the paper reports 30 s for this model's query on a GTX 1060 (other hardware)",
    }
    log(f"imdp: {kms:.1f} ms for {it} iterations ({achieved:.0f} GB/s algorithmic)")


def _mimo64(args, sec, dev):
    import torch

    import oracle
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    # the 64-state model: 16 requests in flight, device memory
    mdl = wl.mimo64()
    mix = DeviceMix([mdl] * 16, dev)
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    with binding.Engine(arena_bytes=1 << 30) as eng:
        row = {}
        for name, prec in (("fp64", binding.PREC_FP64), ("refined", binding.PREC_REFINED)):
            mix.run(eng, prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(12):
                mix.run(eng, prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(oracle.rel_err(mix.G(0), ref).max())
            row[name] = {"points_per_s": 12 * 16 * mdl.K / dt, "max_rel_err": err}
        lat = []
        d = mix.t[0]
        for i in range(60):
            a = time.perf_counter()
            eng.wait(eng.submit_device(d["A"], d["B"], d["C"], d["D"], d["omega"], d["G"], d["info"]))
            if i >= 10:
                lat.append(time.perf_counter() - a)
        row["latency_one_request_ms"] = _pct(lat)
        sec["mimo64"] = row
    del mix
    log("secondary: mimo64 done")


def _large1024(args, sec):
    import oracle
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    # the 1024-state model: ten queries (two repeats), refined and float64
    models = wl.large1024_models()
    queries = wl.large1024_queries(models)
    with binding.Engine(arena_bytes=8 << 30, kernel_timing=True) as eng:
        row = {}
        for name, prec in (("refined", binding.PREC_REFINED), ("fp64", binding.PREC_FP64)):
            base = 10 if name == "refined" else 100
            t0 = time.perf_counter()
            hs = [eng.submit(models[i].A, models[i].B, models[i].C, models[i].D, w, precision=prec,
                             model_key=base + i) for i, w in queries]
            for h in hs:
                eng.wait(h)
            dt = time.perf_counter() - t0
            idx = np.arange(0, 10_000, 1250)
            errs = []
            for (i, w), h in list(zip(queries, hs))[::3]:
                errs.append(float(oracle.rel_err(h.G[idx], oracle.freqresp(models[i].A, models[i].B, models[i].C,
                                                                          models[i].D, w[idx])).max()))
            row[name] = {"points_per_s": 100_000 / dt, "wall_s": dt, "sampled_max_rel_err": max(errs),
                         "reductions_reused": int(sum(h.result["reduction_reused"] for h in hs))}
        row["note"] = "host-memory requests (inputs 8 MB each), ten queries in flight"
        sec["large1024"] = row
    log("secondary: large1024 done")


def _damped256(args, sec):
    import oracle
    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    # 512 lightly damped 256-state models at once, refined
    models = wl.damped256(args.damped_models)
    with binding.Engine(arena_bytes=16 << 30, kernel_timing=True, host_staging_bytes=2 << 30) as eng:
        row = {}
        for prec in (binding.PREC_REFINED, binding.PREC_FP64):  # untimed: code objects, pinned pages
            for h in [eng.submit(m.A, m.B, m.C, m.D, m.omega, precision=prec) for m in models[:8]]:
                eng.wait(h)
        for name, prec in (("refined", binding.PREC_REFINED), ("fp64", binding.PREC_FP64)):
            t0 = time.perf_counter()
            hs = [eng.submit(m.A, m.B, m.C, m.D, m.omega, precision=prec) for m in models]
            for h in hs:
                eng.wait(h)
            dt = time.perf_counter() - t0
            errs = []
            for j in range(0, len(models), 64):
                mdl, h = models[j], hs[j]
                d = np.abs(1j * mdl.omega[:, None] - mdl.poles[None, :])
                idx = np.unique(np.concatenate([np.argsort(d.max(1) / d.min(1))[-2:], [0, 3500]]))
                errs.append(float(oracle.rel_err(h.G[idx], oracle.freqresp_extended(
                    mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega[idx])).max()))
            row[name] = {"points_per_s": 4096 * len(models) / dt, "wall_s": dt,
                         "sampled_max_rel_err_vs_extended": max(errs),
                         "fallback_points": int(sum(h.result["n_fallback"] for h in hs)),
                         "fp64_dd_points": int(sum(h.result["n_fp64_dd"] for h in hs))}
        row["note"] = f"{len(models)} models submitted at once from host memory"
        sec["damped256"] = row
    log("secondary: damped256 done")


# ------------------------------------------------------------------ counters

def profile_pass(args):
    """The run that HBM counters are taken on: one 256 MiB device copy (the
    calibration: FETCH_SIZE / WRITE_SIZE of a copy of known size), then
    `args.profile_pass` refined passes over the serving mix (device-memory
    requests).  Prints the points each kernel family swept."""
    import torch

    from paper_2401_04068_amd import binding
    from paper_2401_04068_amd import workloads as wl

    dev = torch.device("cuda:0")
    src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    reqs = wl.serving_requests(args.requests)
    mix = DeviceMix(reqs, dev)
    with binding.Engine(arena_bytes=8 << 30) as eng:
        for _ in range(args.profile_pass):
            mix.run(eng, binding.PREC_REFINED)
    torch.cuda.synchronize()
    pts = [0] * KF_COUNT
    for r in reqs:
        pts[family_of(r.n, r.m, r.p)] += r.K * args.profile_pass
    print(json.dumps({"copy_bytes": 256 << 20, "passes": args.profile_pass, "requests": args.requests,
                      "points_by_family": pts}), flush=True)


def _pmc_totals(csv_path, counter):
    """Sum of `counter` per kernel name over every dispatch in a rocprofv3
    counter-collection CSV."""
    import csv

    tot = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            k = row["Kernel_Name"]
            tot[k] = tot.get(k, 0.0) + float(row["Counter_Value"])
    return tot


def _pmc_max_dispatch(csv_path, counter, name_part):
    import csv

    best = 0.0
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter and name_part in row["Kernel_Name"]:
                best = max(best, float(row["Counter_Value"]))
    return best


def traffic_record(args):
    """profiles/kf<f>_serving_traffic.json from two counter runs of
    `--profile-pass` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch): HBM
    bytes per point of the refined kernels of family f, each counter scaled by
    true bytes / counter for the calibration copy."""
    fetch_csv, write_csv, pass_json = args.traffic_record
    with open(pass_json) as f:
        ps = json.loads(f.read().strip().splitlines()[-1])
    fetch = _pmc_totals(fetch_csv, "FETCH_SIZE")
    write = _pmc_totals(write_csv, "WRITE_SIZE")
    copy_kib = ps["copy_bytes"] / 1024.0
    # the calibration copy is the largest single copy dispatch of the run
    fk = _pmc_max_dispatch(fetch_csv, "FETCH_SIZE", "copyBuffer")
    wk = _pmc_max_dispatch(write_csv, "WRITE_SIZE", "copyBuffer")
    if not fk or not wk:
        raise SystemExit("calibration copy not found in the counter CSVs")
    ff, wf = copy_kib / fk, copy_kib / wk
    tags = ["sweep16_kernel<1,", "sweep32_kernel<1,", "sweep_kernel<1,", "sweep_wg_kernel<1,"]
    names = [k for k in fetch if any(t in k.replace(" ", "") for t in tags)]
    fb = sum(fetch[k] for k in names) * ff * 1024.0
    wb = sum(write.get(k, 0.0) for k in names) * wf * 1024.0
    pts = sum(ps["points_by_family"])
    rec = {"kernels_of": "every refined sweep kernel (the sweep phase of the batches)", "precision": "refined",
           "workload": "serving mix",
           "source_files": SWEEP_SOURCES, "source_sha256_16": _source_digest(SWEEP_SOURCES),
           "kernels": sorted(names), "fetch_factor": ff, "write_factor": wf,
           "fetch_bytes": fb, "write_bytes": wb, "points_swept": pts,
           "hbm_bytes_per_point": (fb + wb) / max(pts, 1),
           "commands": args.traffic_commands or []}
    path = os.path.join(PROFILES, "sweep_serving_traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="serving", choices=["serving"])
    ap.add_argument("--requests", type=int, default=4096, help="requests in the serving mix")
    ap.add_argument("--damped-models", type=int, default=512, help="models of the lightly damped batch")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-secondary", action="store_true", help="only the headline configuration")
    ap.add_argument("--only", choices=["mimo64", "large1024", "damped256", "imdp"],
                    help="run one secondary configuration only (no headline)")
    ap.add_argument("--profile-pass", type=int, default=0,
                    help="counter run: a calibration copy, then this many refined passes of the mix")
    ap.add_argument("--traffic-record", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PASS_JSON"),
                    help="write the HBM-traffic record of a kernel family from two counter runs")
    ap.add_argument("--traffic-commands", nargs="*")
    args = ap.parse_args()
    if args.traffic_record:
        traffic_record(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every request and every frequency is independent, and the "
              "multi-GPU sharding (requests routed per GPU) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    out = {
        "metric": METRIC, "value": None, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c32+f64", "data": "synthetic (seeded models of the stated recipe)",
    }
    if args.profile_pass:
        profile_pass(args)
        return
    if args.only:
        secondary(args, out)
        print(json.dumps(out), flush=True)
        return
    serving_headline(args, out)
    if not args.no_secondary:
        secondary(args, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
