"""Benchmark: PCG map-making with M_2l vs M_BD on one MI355X.

Workload (default): the 256 x 256 patch, 128 detectors x 2^20 samples
(1.34e8 samples), cross-linked rasters, 1/f noise with f_knee ~ U[0.05, 1] Hz
per detector, N^-1 half bandwidth 4,096 applied by FFT over 2^16-sample
intervals, FP64, M_2l with k = 32 Ritz vectors (Arnoldi from M_BD b,
stopped when its own solution of B x = r_0 has a relative residual of 1e-10,
m_max 256) vs M_BD, tolerance 1e-8.  Inputs are seeded and synthetic (see
synth/).

A timed step is one PCG iteration with M_2l: q = A p (P, N^-1, P^T), the
M_2l apply, and the vector updates and reductions.  `value` is the A-apply
rate inside those iterations: samples per second = N_t * steps / time.  The
line also carries the pure A-apply rate, time to a 1e-8 residual for M_2l and
M_BD (with setup costs), the roofline of the dominant kernel and the oracle
timed on the host on a bounded sample.

`--form NAME` measures one form or study instead and prints its own JSON
line.  The latency (c1), batching (c4) and serving (c5) forms carry the
FP64 oracle's timing of the same work as `cpu_baseline` (config 1's solves
on one core; the 64 Monte Carlo solves on all host cores; the serving trace
extrapolated per request from each strategy's measured costs); `--no-cpu`
leaves it out.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1] [--no-solves] [--no-cpu]
    python bench.py --form c1|c3|c4|c5|f1|g1|d1|z1|p1|h1|n1|mf [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TF = 78.6
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per sample per kernel launch, FP64 (index 4 B, angle 8 B,
# TOD 8 B; the weights are formed from the angle in the kernels).  P: map-slot
# index + angle read, y written; P^T: sample index + angle of the sliced
# layout + z gathered (its ~8 % padding entries not counted); direct band:
# y + z.  The FFT's figure depends on the overlap-save geometry and is computed
# by fft_bytes_per_sample.
ALG_BYTES = {"P": 20.0, "PT": 20.0, "Ninv_band": 16.0}


def fft_bytes_per_sample(interval_start, lam: int, n_valid: int, elem: int = 8) -> float:
    """Bytes per sample the overlap-save N^-1 must move: every block reads
    its V valid samples plus lambda on each side, clipped to the interval
    (samples outside it are zero), and writes its valid outputs once."""
    reads = 0
    starts = np.asarray(interval_start, dtype=np.int64)
    for a, e in zip(starts[:-1], starts[1:]):
        t0 = np.arange(a, e, n_valid)
        reads += int(np.sum(np.minimum(e, t0 + n_valid + lam) - np.maximum(a, t0 - lam)))
    n = int(starts[-1] - starts[0])
    return elem * (reads + n) / n


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Files whose text determines each measured kernel group's device code: the
# source that defines it, the device-code headers it includes and the build
# flags.  Host-side declarations (the internal structures, the C API header)
# are left out: they do not change a kernel's code.
KERNEL_SOURCES = {
    "P": ["tod_ops.hip", "pointing.hip", "pol_weights.h", "xcd.h"],
    "PT": ["tod_ops.hip", "pointing.hip", "pol_weights.h", "xcd.h"],
    "Ninv_fft": ["noise_fft_big.hip", "fft_common.h"],
    "Ninv_band": ["tod_ops.hip"],
}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1801_08937_amd")
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(pkg, "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(pkg, "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the kernel's current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("source_hash") != kernel_source_hash(kernel):
        return None
    return k.get("bytes_per_launch")


# Oracle objects shared with forked workers of the all-cores CPU baseline.
_CPU = {}


def _cpu_partial(rng):
    """The oracle's A apply on the intervals [i0, i1) of the sample: N^-1 is
    block diagonal over intervals, so A x is the sum of these partial maps."""
    import dataclasses
    import oracle as O
    i0, i1 = rng
    pt, nz, x = _CPU["pt"], _CPU["nz"], _CPU["x"]
    s0, s1 = int(nz.interval_start[i0]), int(nz.interval_start[i1])
    sub = dataclasses.replace(pt, n_samp=s1 - s0, j=pt.j[s0:s1], cos2=pt.cos2[s0:s1],
                              sin2=pt.sin2[s0:s1])
    snz = O.Noise(nz.interval_start[i0:i1 + 1] - s0, nz.filter_id[i0:i1], nz.band, nz.half_bw)
    return O.apply_A(sub, snz, x, "fft")


def cpu_baseline(p, n_det_sample: int):
    """The FP64 oracle on the host cores, on the first n_det_sample detectors'
    samples of the same inputs (a bounded sample): its A apply (FFT path) on
    one core, and on all the host's cores (at most 16, the GPU's CPU share)
    with a fixed partition of the intervals over forked worker processes and
    the partial maps added in partition order; plus the per-iteration map-
    domain costs (M_BD apply, the PCG vector updates) for the solve-time
    extrapolation.  Runs before the GPU is initialised (workers fork)."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    import oracle as O
    t_all = time.perf_counter()
    spd = p.n_samp // 128 if p.n_samp >= 128 else p.n_samp
    ns = n_det_sample * spd
    n_int = int(np.searchsorted(p.interval_start, ns))
    pt = O.pointing_build(p.pix[:ns], p.psi[:ns], p.n_pix_total, 1)
    nz = O.noise_build(p.interval_start[: n_int + 1], p.filter_id[:n_int], p.band, p.half_bw)
    x = np.random.default_rng(0).standard_normal(pt.n)
    out = {"nproc": os.cpu_count()}
    with threadpool_limits(1):
        ref = None
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            ref = O.apply_A(pt, nz, x, "fft")
            ts.append(time.perf_counter() - t0)
        t1 = min(ts)
        M = O.mbd_build(pt, nz)
        t0 = time.perf_counter()
        for _ in range(5):
            O.mbd_apply(M, x)
        t_mbd = (time.perf_counter() - t0) / 5
        t0 = time.perf_counter()
        for _ in range(5):  # the vector work of one PCG iteration: 3 dots, 3 axpys
            v = x + 0.5 * ref
            _ = float(v @ v) + float(x @ ref) + float(ref @ ref)
            v = ref + 0.25 * v
            v = v - 0.125 * x
        t_vec = (time.perf_counter() - t0) / 5
    W = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, n_int, W + 1).round().astype(int)
    parts = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    _CPU.update(pt=pt, nz=nz, x=x)
    tw = []
    with threadpool_limits(1), mp.get_context("fork").Pool(len(parts)) as pool:
        for _ in range(3):
            t0 = time.perf_counter()
            ys = pool.map(_cpu_partial, parts, chunksize=1)
            acc = np.zeros_like(ref)
            for yv in ys:
                acc += yv
            tw.append(time.perf_counter() - t0)
    _CPU.clear()
    err = float(np.max(np.abs(acc - ref)) / np.max(np.abs(ref)))
    tW = min(tw)
    out.update({
        "value": ns / tW, "unit": "samples/s", "cores": len(parts), "kind": "oracle",
        "sample": f"A apply (numpy FFT path) on the first {n_det_sample} of 128 detectors "
                  f"({ns} samples, {n_int} intervals) of the same inputs; all cores: "
                  f"{len(parts)} forked workers over a fixed partition of the intervals, "
                  f"best of 3 applies; one core: best of 2",
        "single_core": {"value": ns / t1, "unit": "samples/s", "cores": 1, "apply_s": t1},
        "all_cores_apply_s": tW, "all_cores_vs_single_maxrel": err,
        "sample_samples": ns, "mbd_apply_s": t_mbd, "vec_ops_s": t_vec,
        "sample_unknowns": pt.n, "wall_s": time.perf_counter() - t_all})
    return out


def cpu_solve_estimates(cpu, n_samp, n_unknowns, solves, m_max, k):
    """Oracle time to a 1e-8 residual at the full workload, extrapolated: one
    PCG iteration = A apply (the sample's measured time scaled by samples) +
    M_BD apply and vector updates (scaled by unknowns) (+ the M_2l coarse
    terms, 3 n k multiply-adds, counted as three more vector passes per column
    group of 8), times the iteration counts the GPU solves took; M_2l's setup
    = m_max Arnoldi steps at the same per-step cost plus k A applies."""
    if not cpu or not solves:
        return None
    sc_n = n_unknowns / max(cpu["sample_unknowns"], 1)
    res = {"method": "extrapolated from the measured sample costs and the GPU iteration counts"}
    for label, a_rate in (("single_core", cpu["single_core"]["value"]), ("all_cores", cpu["value"])):
        t_a = n_samp / a_rate
        t_map = (cpu["mbd_apply_s"] + cpu["vec_ops_s"]) * sc_n
        t_m2l_extra = cpu["vec_ops_s"] * sc_n * 3 * k / 8
        e = {"A_apply_s": t_a}
        if "mbd" in solves:
            e["mbd_s"] = solves["mbd"]["iters"] * (t_a + t_map)
        if "m2l" in solves:
            e["m2l_solve_s"] = solves["m2l"]["iters"] * (t_a + t_map + t_m2l_extra)
            e["m2l_setup_s"] = m_max * (t_a + t_map) + k * t_a
        res[label] = e
    return res


def _oracle_pcg_cols(rng):
    """Oracle PCG to 1e-8 on the right-hand sides [c0, c1) of the batch held in
    _CPU (a forked worker of oracle_c4): (iterations, true residual) each."""
    import oracle as O
    c0, c1 = rng
    pt, nz, B, apply_M = _CPU["pt"], _CPU["nz"], _CPU["B"], _CPU["apply_M"]
    out = []
    for c in range(c0, c1):
        _, info = O.pcg(lambda v: O.apply_A(pt, nz, v), apply_M, B[:, c], 1e-8, 3000)
        out.append((int(info.iters), float(info.rel_res_true)))
    return out


def oracle_c1():
    """Config 1 on the FP64 oracle, one host core: setup (pointing, noise
    model, M_BD, b), the A apply, PCG to 1e-8 with M_BD, and with M_2l (k = 32,
    Arnoldi with the literal stop rule at 1e-8 and at most 256 steps, as the
    GPU form builds it)."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    import synth
    p = synth.config1()
    res = {"kind": "oracle", "cores": 1, "nproc": os.cpu_count(),
           "sample": f"the whole config-1 problem ({p.n_samp} samples), numpy on one thread"}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
        nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
        M = O.mbd_build(pt, nz)
        b = O.rhs(pt, nz, p.tod)
        res["setup_s"] = time.perf_counter() - t0

        def A(v):
            return O.apply_A(pt, nz, v)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            A(b)
            ts.append(time.perf_counter() - t0)
        res["a_apply_ms"] = 1e3 * float(np.median(ts))
        t0 = time.perf_counter()
        _, info = O.pcg(A, lambda v: O.mbd_apply(M, v), b, 1e-8, 2000)
        res["mbd"] = {"iters": int(info.iters), "rel_res_true": float(info.rel_res_true),
                      "solve_s": time.perf_counter() - t0}
        t0 = time.perf_counter()
        M2 = O.defl_build(pt, nz, M, b, 32, 1e-8, 256)[0]
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, info = O.pcg(A, lambda v: O.m2l_apply(M2, v), b, 1e-8, 2000)
        res["m2l"] = {"iters": int(info.iters), "rel_res_true": float(info.rel_res_true),
                      "solve_s": time.perf_counter() - t0, "setup_s": t_setup}
    res["value"] = 1.0 / res["mbd"]["solve_s"]
    res["unit"] = "M_BD solves/s"
    return res


def oracle_c4():
    """The 64 Monte Carlo solves of the batching form on the FP64 oracle: one
    M_BD solve and M_2l's setup (Z from realization 0, as the GPU form) on one
    core, then the 64 M_BD and the 64 M_2l solves on all host cores (at most
    16, the GPU's CPU share): a fixed partition of the realizations over
    forked single-threaded workers.  Runs before the GPU is initialised."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    import oracle as O
    import synth
    t_all = time.perf_counter()
    reals = [synth.config4_realization(r) for r in range(64)]
    p = reals[0]
    with threadpool_limits(1):
        pt = O.pointing_build(p.pix, p.psi, p.n_pix_total, p.min_hits)
        nz = O.noise_build(p.interval_start, p.filter_id, p.band, p.half_bw)
        M = O.mbd_build(pt, nz)
        B = np.stack([O.rhs(pt, nz, q.tod) for q in reals], axis=1)
        t0 = time.perf_counter()
        O.pcg(lambda v: O.apply_A(pt, nz, v), lambda v: O.mbd_apply(M, v), B[:, 0], 1e-8, 3000)
        t_one = time.perf_counter() - t0
        t0 = time.perf_counter()
        M2 = O.defl_build(pt, nz, M, B[:, 0], 32, 1e-8, 256)[0]
        t_m2l_setup = time.perf_counter() - t0
    W = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, 64, W + 1).round().astype(int)
    parts = [(int(a), int(b_)) for a, b_ in zip(bounds[:-1], bounds[1:]) if b_ > a]
    res = {"kind": "oracle", "cores": len(parts), "nproc": os.cpu_count(),
           "sample": "all 64 realizations of config 4 in FP64; one forked single-threaded "
                     "worker per slice of a fixed partition of the realizations",
           "mbd_one_solve_single_core_s": t_one, "m2l_setup_single_core_s": t_m2l_setup}
    for name, apply_M in (("mbd", lambda v: O.mbd_apply(M, v)),
                          ("m2l", lambda v: O.m2l_apply(M2, v))):
        _CPU.update(pt=pt, nz=nz, B=B, apply_M=apply_M)
        with threadpool_limits(1), mp.get_context("fork").Pool(len(parts)) as pool:
            t0 = time.perf_counter()
            rs = pool.map(_oracle_pcg_cols, parts, chunksize=1)
            t = time.perf_counter() - t0
        its = [i for r in rs for (i, _) in r]
        rr = [x for r in rs for (_, x) in r]
        res[name] = {"solves_64_s": t, "max_iters": max(its), "mean_iters": float(np.mean(its)),
                     "max_rel_res_true": max(rr)}
    _CPU.clear()
    res["value"] = 64 / res["mbd"]["solves_64_s"]
    res["unit"] = "M_BD solves/s"
    res["wall_s"] = time.perf_counter() - t_all
    return res


def oracle_strategy_costs(p):
    """Costs of an oracle M_BD solve for one serving strategy, on one core,
    measured on its first min(2^20, n) samples (whole intervals): the setup
    (pointing, noise model, M_BD), the A apply (FFT path), the M_BD apply and
    one iteration's vector work.  oracle_trace_estimate scales them to the
    strategy's size."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    ns = min(1 << 20, p.n_samp)
    n_int = int(np.searchsorted(p.interval_start, ns))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pt = O.pointing_build(p.pix[:ns], p.psi[:ns], p.n_pix_total, 1)
        nz = O.noise_build(p.interval_start[: n_int + 1], p.filter_id[:n_int], p.band, p.half_bw)
        M = O.mbd_build(pt, nz)
        t_setup = time.perf_counter() - t0
        x = np.random.default_rng(0).standard_normal(pt.n)
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            y = O.apply_A(pt, nz, x, "fft")
            ts.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        for _ in range(5):
            O.mbd_apply(M, x)
        t_mbd = (time.perf_counter() - t0) / 5
        t0 = time.perf_counter()
        for _ in range(5):  # the vector work of one PCG iteration: 3 dots, 3 axpys
            v = x + 0.5 * y
            _ = float(v @ v) + float(x @ y) + float(y @ y)
            v = y + 0.25 * v
            v = v - 0.125 * x
        t_vec = (time.perf_counter() - t0) / 5
    return {"sample_samples": ns, "n_samp": p.n_samp, "sample_unknowns": pt.n,
            "setup_s": t_setup, "a_apply_s": min(ts), "map_ops_s": t_mbd + t_vec}


def oracle_trace_estimate(costs, n_obs, strat, iters):
    """Single-core oracle time of the serving baseline (one request at a time,
    M_BD, nothing cached), extrapolated per request: the strategy's setup and
    A apply scaled by samples, its map-domain work by unknowns, times the
    iteration count the GPU baseline took for that request."""
    per = []
    for s, c in enumerate(costs):
        ss = c["n_samp"] / c["sample_samples"]
        sn = n_obs[s] / max(c["sample_unknowns"], 1)
        per.append({"setup_s": c["setup_s"] * ss,
                    "per_iter_s": c["a_apply_s"] * ss + c["map_ops_s"] * sn,
                    "a_apply_s": c["a_apply_s"] * ss})
    t_req = [per[int(s)]["setup_s"] + it * per[int(s)]["per_iter_s"] for s, it in zip(strat, iters)]
    total = float(np.sum(t_req))
    return {"kind": "oracle", "cores": 1, "nproc": os.cpu_count(),
            "method": "per-strategy costs measured on the first 2^20 samples (one core) and "
                      "scaled; iteration counts from the GPU baseline",
            "per_strategy": per, "trace_s": total, "value": len(t_req) / total,
            "unit": "solves/s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c2", "c1"])
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="setup + timed steps only (for rocprofv3 runs)")
    ap.add_argument("--m-max", type=int, default=256, help="Arnoldi steps for M_2l")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--form", choices=["c1", "c3", "c4", "c5", "f1", "g1", "d1", "z1", "p1", "h1", "n1",
                                       "mf"], default=None,
                    help="measure one form (latency, FP32, batched, serving) instead")
    ap.add_argument("--requests", type=int, default=200, help="requests in the serving trace")
    ap.add_argument("--slots", type=int, default=1, help="columns per serving session")
    ap.add_argument("--rate", type=float, default=4.0, help="serving arrival rate (requests/s)")
    ap.add_argument("--serve-stop", choices=["h", "residual"], default="h",
                    help="Arnoldi stop rule of the serving engine's background M_2l build")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 5, "ms": ms,
                          "GBps_read_plus_write": 2 * src.numel() * 8 / ms / 1e6}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU design (shard by "
              "detector intervals + one map all-reduce per A apply) is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1801_08937_amd import mapmaker as mm

    if args.form:
        # the oracle's legs of the latency and batching forms, before the GPU
        # is initialised (the batching leg forks worker processes)
        pre = None
        if not args.no_cpu and args.form in ("c1", "c4"):
            pre = (oracle_c1 if args.form == "c1" else oracle_c4)()
            log(f"[bench] oracle: {pre}")
        torch.cuda.init()
        ctx = mm.Context(0)
        fn = {"c1": form_c1, "c3": form_c3, "c4": form_c4, "f1": form_f1, "d1": form_d1,
              "z1": form_z1, "g1": lambda m, c: form_f1(m, c, ground=True), "p1": form_p1, "h1": form_h1, "n1": form_n1,
              "mf": form_mf,
              "c5": lambda m, c: form_c5(m, c, n_requests=args.requests,
                                         slots=args.slots, rate=args.rate,
                                         stop=args.serve_stop, cpu=not args.no_cpu)}[args.form]
        res = fn(mm, ctx)
        if pre is not None:
            res["cpu_baseline"] = pre
        print(json.dumps(res), flush=True)
        ctx.close()
        return

    t = time.perf_counter()
    if args.workload == "c2":
        p = synth.config2()
        wl = ("config2: 256x256 patch (65,536 px, 196,608 unknowns), 128 det x 2^20 samples "
              "(1.34e8), 3-orientation cross-linked rasters, HWP psi, 1/f f_knee~U[0.05,1] Hz, "
              "N^-1 half-bandwidth 4096 by FFT over 2^16-sample intervals, FP64, "
              "M_2l k=32 (Arnoldi to a 1e-10 residual) vs M_BD, tol 1e-8")
    else:
        p = synth.config1()
        wl = ("config1: 32x32 patch, 2 det x 65,536 samples, lambda 32 direct band, FP64, "
              "M_BD and M_2l k=32, tol 1e-8")
    log(f"[bench] generated {p.name}: {p.n_samp} samples in {time.perf_counter() - t:.1f} s")
    cpu = None
    if not args.no_cpu and not args.profile_only and args.workload == "c2":
        # before the GPU is initialised: the all-cores leg forks worker processes
        cpu = cpu_baseline(p, 32)
        log(f"[bench] cpu baseline: {cpu}")
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    pix = torch.from_numpy(p.pix).to(dev)
    psi = torch.from_numpy(p.psi).to(dev)
    tod = torch.from_numpy(p.tod).to(dev)
    ctx = mm.Context(0)
    stream = ctx.stream
    setup = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        setup[name] = time.perf_counter() - t0
        log(f"[bench] {name}: {setup[name]:.3f} s")
        return r

    lp = timed("pointing_build_s", lambda: ctx.pointing(pix, psi, p.n_pix_total, p.min_hits))
    lp.set_grid(p.n_side)
    ln = timed("noise_build_s", lambda: ctx.noise(p.interval_start, p.filter_id, p.band,
                                                  p.half_bw))
    Mbd = timed("mbd_build_s", lambda: ctx.mbd(lp, ln))
    b = timed("rhs_s", lambda: ctx.rhs(lp, ln, tod))
    del pix, psi
    # M_2l (k = 32) by Arnoldi stopped when its own solution of B x = r_0 has
    # a relative residual <= 1e-10 (the residual reading of the eps_Arn test;
    # the literal h_{j+1,j} test is timed beside it below)
    M2 = timed("m2l_build_s", lambda: ctx.defl_build(lp, ln, Mbd, b, k=32, eps_arn=1e-10,
                                                      m_max=args.m_max, stop="residual"))
    arn = M2.arnoldi_info
    log(f"[bench] Arnoldi m={arn.m} k={arn.k} h_last={arn.h_last:.2e}")

    solves = {}
    if not args.no_solves and not args.profile_only:
        for name, M in (("m2l", M2), ("mbd", Mbd)):
            # each solve twice: the first in the process also pays one-time
            # costs (code object loads, workspace); the second is reported
            els = []
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = ctx.solve(lp, ln, M, b, tol=1e-8, max_iter=3000, check_every=4,
                                    history=False)
                torch.cuda.synchronize()
                els.append(time.perf_counter() - t0)
            el = els[1]
            solves[name] = {"iters": info["iters"], "converged": info["converged"],
                            "rel_res_true": info["rel_res_true"], "solve_s": el,
                            "first_solve_s": els[0], "s_per_iter": el / max(info["iters"], 1)}
            log(f"[bench] solve {name}: {solves[name]}")
        solves["m2l"]["setup_s"] = setup["m2l_build_s"]
        solves["m2l"]["total_s"] = setup["m2l_build_s"] + solves["m2l"]["solve_s"]
        solves["mbd"]["total_s"] = solves["mbd"]["solve_s"]
        # M_2l whose Z comes from the Ritz vectors of the M_BD solve itself
        # (to 1e-12; the call also returns that solve's map), then M_2l to 1e-8
        xh = torch.empty_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Mh = ctx.defl_build_pcg(lp, ln, Mbd, b, k=32, m_max=500, tol=1e-12, x_out=xh)
        torch.cuda.synchronize()
        t_h = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, info = ctx.solve(lp, ln, Mh, b, tol=1e-8, max_iter=3000, check_every=4,
                            history=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        solves["m2l_from_mbd_solve"] = {
            "iters": info["iters"], "converged": info["converged"],
            "rel_res_true": info["rel_res_true"], "solve_s": el,
            "s_per_iter": el / max(info["iters"], 1), "setup_s": t_h,
            "setup_steps": Mh.arnoldi_info.m, "total_s": t_h + el}
        log(f"[bench] solve m2l_from_mbd_solve: {solves['m2l_from_mbd_solve']}")
        del Mh, xh
        # other Arnoldi stops: the residual reading at 1e-8, and the literal
        # test h_{j+1,j} <= 1e-8, which on this problem runs to m_max
        for key, eps, stop in (("m2l_arnoldi_residual_rule_1e-08", 1e-8, "residual"),
                               ("m2l_arnoldi_h_rule_1e-08", 1e-8, "h")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Mr = ctx.defl_build(lp, ln, Mbd, b, k=32, eps_arn=eps, m_max=args.m_max,
                                stop=stop)
            torch.cuda.synchronize()
            t_r = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, info = ctx.solve(lp, ln, Mr, b, tol=1e-8, max_iter=3000, check_every=4,
                                history=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            solves[key] = {
                "iters": info["iters"], "converged": info["converged"],
                "rel_res_true": info["rel_res_true"], "solve_s": el,
                "s_per_iter": el / max(info["iters"], 1), "setup_s": t_r,
                "setup_steps": Mr.arnoldi_info.m, "total_s": t_r + el}
            log(f"[bench] solve {key}: {solves[key]}")
            del Mr

    # pure A-apply rate
    x = torch.randn(lp.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        ctx.apply_A(lp, ln, x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_apply = 20
    ev0.record(stream)
    for _ in range(n_apply):
        ctx.apply_A(lp, ln, x, y)
    ev1.record(stream)
    ev1.synchronize()
    a_ms = ev0.elapsed_time(ev1) / n_apply
    alg_bytes = dict(ALG_BYTES)
    if ln.method == 2:
        alg_bytes["Ninv_fft"] = fft_bytes_per_sample(p.interval_start, p.half_bw, ln.fft_valid)
    ninv = alg_bytes["Ninv_fft"] if ln.method == 2 else alg_bytes["Ninv_band"]
    a_apply = {"ms": a_ms, "samples_per_s": p.n_samp / (a_ms * 1e-3),
               "design_bytes_per_sample": alg_bytes["P"] + alg_bytes["PT"] + ninv,
               "design_GBps": p.n_samp * (alg_bytes["P"] + alg_bytes["PT"] + ninv)
               / (a_ms * 1e-3) / 1e9,
               "lower_bound_GBps": p.n_samp * 20.0 / (a_ms * 1e-3) / 1e9}
    # the A apply against HBM peak, on the design's bytes per sample and on the
    # 20 B/sample lower bound (P's non-zeros read once)
    a_apply["design_frac_hbm_peak"] = a_apply["design_GBps"] / HBM_PEAK_GBS
    a_apply["lower_bound_frac_hbm_peak"] = a_apply["lower_bound_GBps"] / HBM_PEAK_GBS
    log(f"[bench] A apply: {a_apply}")

    # timed steps: PCG iterations with M_2l
    S = ctx.pcg_session(lp, ln, M2, 1)
    S.start(0, b, 0.0, 10 ** 9)
    S.iterate(args.warmup)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.iterate(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = ctx.profile_read()
    ctx.profile(False)
    ms_step = el * 1e3 / args.steps
    value = p.n_samp * args.steps / el

    # dominant kernel: most event time among the TOD kernels
    tod_stages = {k: v for k, v in stages.items() if k in alg_bytes}
    dom = max(tod_stages, key=lambda k: tod_stages[k][0])
    dom_ms, dom_calls = tod_stages[dom]
    avg_ms = dom_ms / dom_calls
    alg = alg_bytes[dom] * p.n_samp
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_ms": round(avg_ms, 4),
                "alg_bytes_per_launch": alg}

    if cpu is not None:
        cpu["solve_estimates"] = cpu_solve_estimates(cpu, p.n_samp, lp.n, solves, args.m_max, 32)

    line = {
        "metric": "A-apply samples/s (HBM GB/s) + time-to-1e-8 residual, M_2l vs M_BD, 1 GPU",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl, "n_samples": p.n_samp, "n_unknowns": lp.n,
                   "half_bw": p.half_bw, "noise_method": {1: "direct", 2: "fft"}[ln.method],
                   "step": "one PCG iteration with M_2l (A apply + M_2l + vector ops)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "a_apply": a_apply,
        "solves": solves,
        "setup_s": setup,
        "arnoldi": {"m": arn.m, "k": arn.k, "h_last": arn.h_last},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


# ------------------------------------------------------------------ forms
# `--form c1|c3|c4|c5` prints one JSON line for that form of the solver
# instead of the default line: small-problem latency (config 1), the FP32
# precision form, the 64-column batched form and the serving form, each next
# to the plain FP64 solver on the same inputs.

def _sync():
    import torch
    torch.cuda.synchronize()


def _wall(fn, reps=1):
    """(result of the last call, median wall seconds over reps calls)."""
    ts, r = [], None
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        r = fn()
        _sync()
        ts.append(time.perf_counter() - t0)
    return r, float(np.median(ts))


def form_c1(mm, ctx):
    """Config 1 (32x32 patch, 2 x 65,536 samples, lambda 32): everything sits
    in cache, so this is a latency figure: A apply, one PCG iteration eager
    and graph-replayed, and time to 1e-8 for M_BD and M_2l (k = 32)."""
    import torch
    import synth
    p = synth.config1()
    dev = torch.device("cuda", 0)
    lp = ctx.pointing(torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev),
                      p.n_pix_total, p.min_hits)
    ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
    Mbd = ctx.mbd(lp, ln)
    b = ctx.rhs(lp, ln, torch.from_numpy(p.tod).to(dev))
    x = torch.randn(lp.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(5):
        ctx.apply_A(lp, ln, x, y)
    _sync()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(ctx.stream)
    for _ in range(200):
        ctx.apply_A(lp, ln, x, y)
    ev[1].record(ctx.stream)
    ev[1].synchronize()
    a_us = ev[0].elapsed_time(ev[1]) / 200 * 1e3
    (M2, t_m2l) = _wall(lambda: ctx.defl_build(lp, ln, Mbd, b, k=32, eps_arn=1e-8, m_max=256))
    out = {"a_apply_us": a_us}
    for name, M in (("mbd", Mbd), ("m2l", M2)):
        for graph in (False, True):
            (r, t) = _wall(lambda: ctx.solve(lp, ln, M, b, tol=1e-8, max_iter=2000,
                                             check_every=8, history=False, graph=graph), reps=5)
            _, info = r
            out[f"{name}_{'graph' if graph else 'eager'}"] = {
                "iters": info["iters"], "converged": info["converged"],
                "rel_res_true": info["rel_res_true"], "solve_ms": t * 1e3,
                "us_per_iter": t * 1e6 / max(info["iters"], 1)}
    out["m2l_setup_ms"] = t_m2l * 1e3
    # steady-state cost of one iteration inside a session, eager and replayed
    # from captured graphs of 10 iterations
    for name, M in (("mbd", Mbd), ("m2l", M2)):
        for graph in (False, True):
            S = ctx.pcg_session(lp, ln, M, 1)
            if graph:
                S.use_graph(10)
            S.start(0, b, 0.0, 10 ** 7)
            S.iterate(1)
            S.iterate(20)  # graph captured here
            ts = []
            for _ in range(5):
                S.start(0, b, 0.0, 10 ** 7)
                S.iterate(1)
                (_, t) = _wall(lambda: S.iterate(30))
                st, _, _ = S.poll()
                assert st[0] == 1, "column left the running state during the timing"
                ts.append(t)
            out[f"{name}_session_us_per_iter_{'graph' if graph else 'eager'}"] = \
                float(np.median(ts)) * 1e6 / 30
            S.close()
    return {"form": "c1", "workload": "config1: 32x32 patch, 2 det x 65,536 samples, "
            "lambda 32 direct band, FP64, tol 1e-8", **out}


def _config1_oracle_map():
    """The FP64 oracle's config-1 map (PCG to 1e-13), stored by the committed
    script tests/golden/make_config1_solution.py (the bench reads the file;
    it does not run the oracle)."""
    with open(os.path.join(ROOT, "tests", "golden", "config1_solution.json")) as f:
        return np.array(json.load(f)["x"])


def form_c3(mm, ctx):
    """Config 1 in the FP32 form (TOD, weights and N^-1 in FP32; dots, M_BD
    inverses and the coarse solve in FP64): time to a 1e-6 and a 1e-8 FP64
    true residual next to the FP64 solver, plain and with FP64-residual
    iterative refinement (FP32 PCG corrections, one FP64 A apply per outer
    step), each map's error against the FP64 oracle's solution; and the same
    at the config-2 scale."""
    import torch
    import synth
    p = synth.config1()
    dev = torch.device("cuda", 0)
    pix, psi = torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev)
    tod = torch.from_numpy(p.tod).to(dev)
    lp64 = ctx.pointing(pix, psi, p.n_pix_total, p.min_hits)
    ln64 = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
    lp32 = ctx.pointing(pix, psi, p.n_pix_total, p.min_hits, prec=1)
    ln32 = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw, prec=1)
    b64 = ctx.rhs(lp64, ln64, tod)
    b32 = ctx.rhs(lp32, ln32, tod.float())
    M64, M32 = ctx.mbd(lp64, ln64), ctx.mbd(lp32, ln32)
    x_or = _config1_oracle_map()
    bn = float(torch.linalg.norm(b64))

    def true_res(xs):
        r = b64 - ctx.apply_A(lp64, ln64, xs)
        return float(torch.linalg.norm(r)) / bn

    def err(xs):
        xh = xs.cpu().numpy()
        return float(np.linalg.norm(xh - x_or) / np.linalg.norm(x_or))

    out = {"map_reference": "FP64 oracle, PCG to 1e-13 (tests/golden/config1_solution.json)"}
    for tol in (1e-6, 1e-8):
        for name, lp, ln, M, b in (("fp64", lp64, ln64, M64, b64), ("fp32", lp32, ln32, M32, b32)):
            (r, t) = _wall(lambda: ctx.solve(lp, ln, M, b, tol=tol, max_iter=3000, check_every=8,
                                             history=False), reps=5)
            xs, info = r
            out[f"{name}_tol{tol:g}"] = {
                "iters": info["iters"], "converged": info["converged"], "solve_ms": t * 1e3,
                "rel_res_own": info["rel_res_true"], "rel_res_fp64": true_res(xs),
                "map_rel_err_vs_oracle": err(xs)}
        for itol in (1e-4, 1e-5):
            (r, t) = _wall(lambda: ctx.solve_refined(lp32, ln32, lp64, ln64, M64, b64, tol=tol,
                                                     inner_tol=itol), reps=5)
            xs, info = r
            out[f"fp32_refined_inner{itol:g}_tol{tol:g}"] = {
                "outer": info["outer"], "inner_iters": info["inner_iters"],
                "converged": info["converged"], "solve_ms": t * 1e3,
                "rel_res_fp64": true_res(xs), "map_rel_err_vs_oracle": err(xs)}
    # the same precision split at the config-2 scale, where the TOD passes are
    # bandwidth-bound: A apply and PCG(M_BD) to 1e-6 / 1e-8 in both precisions,
    # and the FP32 form refined to 1e-8 against the FP64 residual
    p2 = synth.config2()
    pix2, psi2 = torch.from_numpy(p2.pix).to(dev), torch.from_numpy(p2.psi).to(dev)
    tod2 = torch.from_numpy(p2.tod).to(dev)
    big, H = {}, {}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        lp = ctx.pointing(pix2, psi2, p2.n_pix_total, p2.min_hits, prec=prec)
        lp.set_grid(p2.n_side)
        ln = ctx.noise(p2.interval_start, p2.filter_id, p2.band, p2.half_bw, prec=prec)
        x = torch.randn(lp.n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            ctx.apply_A(lp, ln, x, y)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(ctx.stream)
        for _ in range(10):
            ctx.apply_A(lp, ln, x, y)
        ev[1].record(ctx.stream)
        ev[1].synchronize()
        b = ctx.rhs(lp, ln, tod2 if prec == 0 else tod2.float())
        M = ctx.mbd(lp, ln)
        res = {"a_apply_ms": ev[0].elapsed_time(ev[1]) / 10}
        for tol in (1e-6, 1e-8):
            (r, t) = _wall(lambda: ctx.solve(lp, ln, M, b, tol=tol, max_iter=500, check_every=4,
                                             history=False))
            xs, info = r
            res[f"tol{tol:g}"] = {"iters": info["iters"], "converged": info["converged"],
                                  "solve_s": t, "rel_res_own": info["rel_res_true"]}
            res[f"x_tol{tol:g}"] = xs
        big[name] = res
        H[name] = (lp, ln, M, b)
    lp64b, ln64b, M64b, b64b = H["fp64"]
    lp32b, ln32b, _, _ = H["fp32"]
    (r, t) = _wall(lambda: ctx.solve_refined(lp32b, ln32b, lp64b, ln64b, M64b, b64b, tol=1e-8,
                                             inner_tol=1e-5, max_inner=500))
    xs, info = r
    big["fp32_refined_tol1e-08"] = {
        "outer": info["outer"], "inner_iters": info["inner_iters"], "converged": info["converged"],
        "solve_s": t, "rel_res_fp64": info["rel_res_true"],
        "map_rel_diff_vs_fp64_tol1e-8": float(torch.linalg.norm(xs - big["fp64"]["x_tol1e-08"])
                                              / torch.linalg.norm(big["fp64"]["x_tol1e-08"]))}
    del H
    for tol in (1e-6, 1e-8):
        x64, x32 = big["fp64"].pop(f"x_tol{tol:g}"), big["fp32"].pop(f"x_tol{tol:g}")
        big["fp32"][f"tol{tol:g}"]["map_rel_diff_vs_fp64"] = float(
            torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    out["config2_scale"] = big
    return {"form": "c3", "workload": "config1 in FP32 (TOD, weights, N^-1 FP32; dots, M_BD, "
            "coarse FP64), M_BD, tol 1e-6 and 1e-8, plain and with FP64-residual refinement; "
            "plus the config-2 scan at both precisions", **out}


def form_c4(mm, ctx):
    """64 Monte Carlo realizations on config 1's pointing: one 64-column solve
    (lockstep columns and block CG, eager and graph-replayed) against 64
    sequential single-column solves; M_BD and M_2l (Z from realization 0);
    FP64 and FP32."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    reals = [synth.config4_realization(r) for r in range(64)]
    p = reals[0]
    pix, psi = torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev)
    T = np.stack([q.tod for q in reals], axis=1)  # [n_samp][64]
    out = {}
    for prec in (0, 1):
        tag = "fp64" if prec == 0 else "fp32"
        lp = ctx.pointing(pix, psi, p.n_pix_total, p.min_hits, prec=prec)
        ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw, prec=prec)
        Td = torch.from_numpy(T).to(dev)
        if prec == 1:
            Td = Td.float()
        B = ctx.rhs(lp, ln, Td.reshape(-1), nrhs=64)
        Mbd = ctx.mbd(lp, ln)
        b0 = B.view(-1, 64)[:, 0].contiguous()
        M2 = ctx.defl_build(lp, ln, Mbd, b0, k=32, eps_arn=1e-8, m_max=256)
        cols = [B.view(-1, 64)[:, c].contiguous() for c in range(64)]
        # per-stage autotuner for 64 and 1 columns: the 64-column A apply
        # before and after (results bitwise the same)
        X = torch.randn(lp.n * 64, dtype=torch.float64, device=dev)
        (_, a_before) = _wall(lambda: ctx.apply_A(lp, ln, X, nrhs=64), reps=10)
        tune = {"nrhs64": ctx.autotune(lp, ln, 64), "nrhs1": ctx.autotune(lp, ln, 1)}
        (_, a_after) = _wall(lambda: ctx.apply_A(lp, ln, X, nrhs=64), reps=10)
        out[f"{tag}_autotune"] = {"a64_ms_before": a_before * 1e3, "a64_ms_after": a_after * 1e3,
                                  "report": tune}
        for mname, M in (("mbd", Mbd), ("m2l", M2)):
            res = {}
            # graph chunk length (iterations per captured graph), measured
            chunks = {}
            for ch in (2, 4, 8, 16):
                (_, t) = _wall(lambda: ctx.solve(lp, ln, M, B, tol=1e-8, max_iter=3000, nrhs=64,
                                                 check_every=ch, history=False, graph=True),
                               reps=3)
                chunks[ch] = t * 1e3
            best_ch = min(chunks, key=chunks.get)
            res["graph_chunk_ms"] = chunks
            for mode, kw in (("lockstep", {}), ("lockstep_graph", {"graph": True}),
                             ("block", {"block": True}),
                             ("block_graph", {"block": True, "graph": True})):
                ch = best_ch if mode.endswith("graph") else 8
                (r, t) = _wall(lambda: ctx.solve(lp, ln, M, B, tol=1e-8, max_iter=3000, nrhs=64,
                                                 check_every=ch, history=False, **kw), reps=3)
                _, infos = r
                infos = infos if isinstance(infos, list) else [infos]
                res[mode] = {"solve_ms": t * 1e3, "max_iters": max(i["iters"] for i in infos),
                             "all_converged": all(i["converged"] for i in infos),
                             "check_every": ch}

            def seq():
                its = []
                for c in range(64):
                    _, inf = ctx.solve(lp, ln, M, cols[c], tol=1e-8, max_iter=3000,
                                       check_every=8, history=False)
                    its.append(inf["iters"])
                return its
            (its, t) = _wall(seq)
            res["sequential_64"] = {"solve_ms": t * 1e3, "max_iters": max(its),
                                    "mean_iters": float(np.mean(its))}
            out[f"{tag}_{mname}"] = res
    return {"form": "c4", "workload": "64 realizations (CMB-like sky + noise each) on config 1's "
            "pointing and noise model, tol 1e-8", **out}


def form_mf(mm, ctx, reps=20):
    """The FP64 MFMA products at the path's shapes, each timed with HIP events
    on the context's stream: E = Z^T (A Z) and the Cholesky-QR Gram of the
    coarse build (config 2, k = 32), Z = W_m Y of the Ritz step (m = 256), and
    block PCG's 64 x 64 Gram and update products (config 4's n = 3,072, and
    at config 2's n).  Reported against the 78.6 TFLOP/s FP64 MFMA peak and,
    with the algorithmic bytes (inputs read once, outputs written once),
    against 8 TB/s HBM; the lower of the two bounds the product."""
    import torch
    dev = torch.device("cuda", 0)
    g = torch.Generator(device=dev).manual_seed(0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    n2, n4 = 196608, 3072

    def colmajor(n, k):
        return torch.randn(k, n, dtype=torch.float64, device=dev, generator=g).t()

    def rowmajor(n, k):
        return torch.randn(n, k, dtype=torch.float64, device=dev, generator=g)

    cases = []
    Z, AZ = colmajor(n2, 32), colmajor(n2, 32)
    cases.append(("E = Z^T (AZ), config 2, k = 32", lambda: ctx.dense_gram(Z, AZ),
                  2.0 * n2 * 32 * 32, 8.0 * n2 * 64))
    W, Y = colmajor(n2, 256), torch.randn(256, 32, dtype=torch.float64, device=dev, generator=g)
    Wc, Yc = W.t().contiguous(), Y.t().contiguous()
    Zo = torch.empty(32, n2, dtype=torch.float64, device=dev)
    from paper_1801_08937_amd.mapmaker import lib, _ptr
    cases.append(("Z = W_m Y, config 2, m = 256, k = 32",
                  lambda: lib().mm_dense_tall(ctx.h, n2, 256, 32, _ptr(Wc), _ptr(Yc), _ptr(Zo)),
                  2.0 * n2 * 256 * 32, 8.0 * n2 * (256 + 32)))
    for n, tag in ((n4, "config 4"), (n2, "config-2 size")):
        P_, Q_ = rowmajor(n, 64), rowmajor(n, 64)
        S_ = torch.randn(64, 64, dtype=torch.float64, device=dev, generator=g)
        O_ = rowmajor(n, 64)
        cases.append((f"block CG Gram P^T Q, {tag}, n = {n}, R = 64",
                      lambda P_=P_, Q_=Q_: ctx.dense_gram(P_, Q_), 2.0 * n * 64 * 64,
                      8.0 * n * 128))
        cases.append((f"block CG update X += P S, {tag}, n = {n}, R = 64",
                      lambda P_=P_, S_=S_, O_=O_: ctx.dense_rows(P_, S_, out=O_, beta=1.0),
                      2.0 * n * 64 * 64, 8.0 * n * 64 * 3))
    rows = []
    for name, fn, flops, nbytes in cases:
        for _ in range(3):
            fn()
        ev[0].record(ctx.stream)
        for _ in range(reps):
            fn()
        ev[1].record(ctx.stream)
        ev[1].synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        tf = flops / (ms * 1e-3) / 1e12
        gbs = nbytes / (ms * 1e-3) / 1e9
        bound_tf = min(FP64_PEAK_TF, nbytes and flops / nbytes * HBM_PEAK_GBS / 1e3)
        rows.append({"product": name, "us": ms * 1e3, "TFLOPs": tf,
                     "mfma_util": tf / FP64_PEAK_TF, "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                     "flop_per_byte": flops / nbytes, "roofline_TFLOPs": bound_tf,
                     "frac_of_roofline": tf / bound_tf})
        log(f"[bench] mf {rows[-1]}")
    return {"form": "mf", "workload": "FP64 MFMA products of the coarse build and block PCG at "
            "config-2 and config-4 shapes", "peak_fp64_mfma_TFLOPs": FP64_PEAK_TF,
            "rows": rows}


def form_f1(mm, ctx, ground=False):
    """The paper's own weight on the config-2 scan: white noise and the
    polynomial template filter F = W - W B (B^T W B)^-1 B^T W with quadratic
    Legendre polynomials per subscan (one 256-sample sweep), A = P^T F P;
    with ground=True also the azimuth-binned ground templates of each
    constant-elevation pass (1-pixel bins shared by the detectors), combined
    as F_B W^+ F_G W^+ F_B.  The filter leaves near-null sky modes (Sect. 4):
    M_BD against M_2l."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    p = synth.config2()
    pix, psi = torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev)
    lp = ctx.pointing(pix, psi, p.n_pix_total, p.min_hits)
    lp.set_grid(p.n_side)
    sub = np.arange(0, p.n_samp + 1, 256, dtype=np.int64)
    w = np.ones(p.n_intervals)
    gargs = ()
    if ground:
        gb, nb = synth.raster_ground_bins(p.n_side, (16, 8), p.n_samp // 128)
        gargs = (torch.from_numpy(gb).to(dev), nb)
    (lf, t_build) = _wall(lambda: ctx.polyfilter(lp, p.interval_start, w, sub, 2, *gargs))
    d = synth.signal_tod(p.pix, p.psi, p.signal) + \
        synth.rng_for(2, 0, synth.STREAM_NOISE).standard_normal(p.n_samp)
    y = torch.randn(p.n_samp, dtype=torch.float64, device=dev)
    x = torch.randn(lp.n, dtype=torch.float64, device=dev)
    out = {"filter_build_s": t_build}
    for name, fn in (("F_apply_ms", lambda: ctx.noise_apply(lf, y)),
                     ("A_apply_ms", lambda: ctx.apply_A(lp, lf, x))):
        for _ in range(3):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(ctx.stream)
        for _ in range(20):
            fn()
        ev[1].record(ctx.stream)
        ev[1].synchronize()
        out[name] = ev[0].elapsed_time(ev[1]) / 20
    out["F_GBps_16B_per_sample"] = 16.0 * p.n_samp / (out["F_apply_ms"] * 1e-3) / 1e9
    b = ctx.rhs(lp, lf, torch.from_numpy(d).to(dev))
    Mbd = ctx.mbd(lp, lf)
    (M2, t_m2l) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, b, k=32, eps_arn=1e-8, m_max=256))
    out["m2l_setup_s"] = t_m2l
    for name, M in (("mbd", Mbd), ("m2l", M2)):
        ((xs, info), t) = _wall(lambda: ctx.solve(lp, lf, M, b, tol=1e-8, max_iter=3000,
                                                  check_every=4, history=False))
        out[name] = {"iters": info["iters"], "converged": info["converged"],
                     "rel_res_true": info["rel_res_true"], "solve_s": t}
    if ground:
        out["n_ground_bins"] = gargs[1]
    return {"form": "g1" if ground else "f1",
            "workload": "config-2 scan (1.34e8 samples), white noise, quadratic Legendre "
            "polynomials removed per 256-sample subscan" +
            (" and azimuth-binned ground templates per constant-elevation pass" if ground else "")
            + " (F_T of Sects. 2 and 4), M_BD vs M_2l (k = 32), tol 1e-8", **out}


def form_p1(mm, ctx, orders=(("I", 2), ("QU", 1))):
    """Detector pairs and the sum/difference decomposition (Sect. 4, Eqs. d+
    and d-): 64 pairs on the config-2 scan (a 16 x 4 focal-plane grid, 2^20
    samples per detector, so 1.34e8 samples over both detectors of every
    pair), B's polariser turned by 90 degrees.  White noise, and per 256-sample
    subscan Legendre polynomials up to order 2 removed from d+ and up to order
    1 from d-, as the paper filters its streams.  The intensity map comes
    from the I system on d+, the polarisation map from the QU system on d-;
    each is solved to 1e-8 with M_BD and with M_2l (k = 32).  Two angle
    models: psi iid per sample (the scan's own), and a fixed angle per pair
    (pi k / 64) plus a half-wave plate stepped by 22.5 degrees between passes,
    so that the angle is constant along every subscan."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    p = synth.config2(grid=(16, 4), noiseless=True)
    n = p.n_samp
    spd = n // 64
    k_of_t = np.arange(n) // spd
    m_of_t = (np.arange(n) % spd) // (p.n_side * p.n_side)
    psi_step = np.pi * k_of_t / 64.0 + (m_of_t % 8) * (np.pi / 8.0)
    pix = torch.from_numpy(p.pix).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2024)
    out = {"n_samp_per_stream": n}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sub = np.arange(0, n + 1, 256, dtype=np.int64)
    w = np.ones(p.n_intervals)
    for model, psi_a in (("psi_iid", p.psi), ("psi_stepped", psi_step)):
        psi = torch.from_numpy(psi_a).to(dev)
        d_a = torch.from_numpy(synth.signal_tod(p.pix, psi_a, p.signal)).to(dev) + \
            torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
        d_b = torch.from_numpy(synth.signal_tod(p.pix, psi_a + 0.5 * np.pi, p.signal)).to(dev) + \
            torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
        res = {}
        if model == "psi_iid":
            for _ in range(3):
                ctx.pair_sum_diff(d_a, d_b)
            ev[0].record(ctx.stream)
            for _ in range(20):
                ctx.pair_sum_diff(d_a, d_b)
            ev[1].record(ctx.stream)
            ev[1].synchronize()
            out["sum_diff_ms"] = ev[0].elapsed_time(ev[1]) / 20
        dp, dm = ctx.pair_sum_diff(d_a, d_b)
        del d_a, d_b
        for stokes, order in orders:
            if stokes == "I" and model != "psi_iid":
                continue  # the intensity system does not see the angles
            d = dp if stokes == "I" else dm
            (lp, t_pt) = _wall(lambda: ctx.pointing(pix, None if stokes == "I" else psi,
                                                    p.n_pix_total, p.min_hits, stokes=stokes))
            lp.set_grid(p.n_side)
            lf = ctx.polyfilter(lp, p.interval_start, w, sub, order)
            x = torch.randn(lp.n, dtype=torch.float64, device=dev, generator=gen)
            for _ in range(3):
                ctx.apply_A(lp, lf, x)
            ev[0].record(ctx.stream)
            for _ in range(20):
                ctx.apply_A(lp, lf, x)
            ev[1].record(ctx.stream)
            ev[1].synchronize()
            r = {"order": order, "n": lp.n, "pointing_build_s": t_pt,
                 "A_apply_ms": ev[0].elapsed_time(ev[1]) / 20}
            b = ctx.rhs(lp, lf, d)
            Mbd = ctx.mbd(lp, lf)
            (M2, t_m2l) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, b, k=32, eps_arn=1e-8,
                                                       m_max=256))
            r["m2l_setup_s"] = t_m2l
            for name, M in (("mbd", Mbd), ("m2l", M2)):
                ((xs, info), t) = _wall(lambda: ctx.solve(lp, lf, M, b, tol=1e-8, max_iter=3000,
                                                          check_every=4, history=False))
                r[name] = {"iters": info["iters"], "converged": info["converged"],
                           "rel_res_true": info["rel_res_true"], "solve_s": t}
            res[stokes] = r
            del lp, lf, b, Mbd, M2
        out[model] = res
    return {"form": "p1", "workload": "64 detector pairs on the config-2 scan (2 x 6.7e7 "
            "samples), white noise, sum/difference streams: I from d+ (Legendre order <= 2 "
            "removed per 256-sample subscan), QU from d- (order <= 1), M_BD vs M_2l (k = 32), "
            "tol 1e-8; angles iid per sample, or fixed per pair with a stepped half-wave plate",
            **out}


def form_h1(mm, ctx, tols=(1e-8, 1e-10, 1e-12), k=32):
    """Config 2's "Ritz vectors from a prior M_BD solve" taken literally: the
    Lanczos tridiagonal of an M_BD PCG solve of the system itself to
    tolerance tol (mm_defl_build_pcg) against the default Arnoldi build
    (mm_defl_build, m = 256, CGS2), each followed by an M_2l solve to 1e-8."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    p = synth.config2()
    lp = ctx.pointing(torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev),
                      p.n_pix_total, p.min_hits)
    lp.set_grid(p.n_side)
    ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
    b = ctx.rhs(lp, ln, torch.from_numpy(p.tod).to(dev))
    Mbd = ctx.mbd(lp, ln)
    out = {}
    ((_, i0), t0) = _wall(lambda: ctx.solve(lp, ln, Mbd, b, tol=1e-8, max_iter=3000,
                                            check_every=4, history=False))
    out["mbd"] = {"iters": i0["iters"], "solve_s": t0}
    builds = [("arnoldi_m256", lambda: ctx.defl_build(lp, ln, Mbd, b, k=k, eps_arn=1e-8,
                                                      m_max=256))]
    builds += [(f"pcg_tol{t:.0e}", (lambda t=t: ctx.defl_build_pcg(lp, ln, Mbd, b, k=k,
                                                                    m_max=500, tol=t)))
               for t in tols]
    for name, fn in builds:
        (M2, t_set) = _wall(fn)
        ((_, info), t) = _wall(lambda: ctx.solve(lp, ln, M2, b, tol=1e-8, max_iter=3000,
                                                 check_every=4, history=False))
        out[name] = {"setup_s": t_set, "steps": M2.arnoldi_info.m, "k": M2.arnoldi_info.k,
                     "iters": info["iters"], "solve_s": t, "rel_res_true": info["rel_res_true"]}
        del M2
    return {"form": "h1", "workload": "config 2, M_2l (k = 32) from Arnoldi vs from the "
            "Lanczos tridiagonal of a prior M_BD PCG solve to tol, then M_2l to 1e-8", **out}


def form_n1(mm, ctx, lams=(16, 32, 64, 128, 256, 512, 1024, 2048, 4096),
            sizes=(1 << 20, 1 << 23, 1 << 27), L=1 << 16):
    """N^-1 method by measured time: the direct band and the overlap-save FFT
    on a config-2-sized stream (1.34e8 samples in 2^16-sample intervals, one
    1/f filter) for a range of half bandwidths, each against its own bound:
    the band against FP64 vector peak (2 (2 lambda + 1) flops per sample),
    the FFT against HBM (its algorithmic bytes per sample)."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rows = []
    for n_samp in sizes:
        rows += _n1_size(mm, ctx, lams, n_samp, L, dev, ev)
    return {"form": "n1", "workload": "2^20, 2^23 and 2^27 samples in 2^16-sample intervals, one "
            "1/f filter; direct band vs overlap-save FFT per half bandwidth", "rows": rows}


def _n1_size(mm, ctx, lams, n_samp, L, dev, ev):
    import torch
    import synth
    istart = np.arange(0, n_samp + 1, L, dtype=np.int64)
    fid = np.zeros(istart.shape[0] - 1, dtype=np.int32)
    y = torch.randn(n_samp, dtype=torch.float64, device=dev)
    z = torch.empty_like(y)
    rows = []
    for lam in lams:
        band = synth.band_from_psd(L, lam, 0.5)[None, :]
        row = {"n_samp": n_samp, "half_bw": lam}
        for name, method in (("direct", 1), ("fft", 2)):
            try:
                ln = ctx.noise(istart, fid, band, lam, method)
            except mm.MapmakerError:
                continue
            reps = 3 if (method == 1 and lam >= 1024) else 20
            ctx.noise_apply(ln, y, z)
            ev[0].record(ctx.stream)
            for _ in range(reps):
                ctx.noise_apply(ln, y, z)
            ev[1].record(ctx.stream)
            ev[1].synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            if method == 1:
                tf = n_samp * 2.0 * (2 * lam + 1) / (ms * 1e-3) / 1e12
                row[name] = {"ms": ms, "TFLOPs": tf, "frac_fp64_peak": tf / FP64_PEAK_TF}
            else:
                bps = fft_bytes_per_sample(istart, lam, ln.fft_valid)
                gbs = n_samp * bps / (ms * 1e-3) / 1e9
                row[name] = {"ms": ms, "GBps": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                             "fft_n": ln.fft_n}
            ln.close()
        picked = ctx.noise(istart, fid, band, lam, 0)
        row["auto_picks"] = {1: "direct", 2: "fft"}[picked.method]
        picked.close()
        rows.append(row)
        log(f"[bench] n1 {row}")
    return rows


def _stats(v):
    """median, 16th and 84th percentiles and (p84 - p16) / 2 (the spread the
    paper tabulates)."""
    v = np.asarray(v, dtype=np.float64)
    p16, p50, p84 = np.percentile(v, [16, 50, 84])
    return {"median": float(p50), "p16": float(p16), "p84": float(p84),
            "half_spread": float((p84 - p16) / 2), "n": int(v.size)}


def form_d1(mm, ctx, n_sub=64, full_m2l=8):
    """Divide and conquer with the "simplified" two-level preconditioner
    (Sect. 7.3, tab. stats and fig. histos2D on synthetic data): the config-2
    scan split by detectors into n_sub subsets over the same patch (two
    detectors, 2^21 samples each at n_sub = 64), each filtered as in form f1
    (white noise, quadratic polynomials per 256-sample subscan).  Z (k = 32)
    is built once, by Arnoldi on subset 0, and moved to every other subset
    with A Z and E rebuilt there (mm_defl_transfer).  Every subset is solved
    to 1e-8 with M_BD and with the transferred M_2l, and the first full_m2l
    with their own M_2l; per solve the iterations to 1e-8 and the residual
    after 100 iterations, then their statistics and histograms."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    p = synth.config2()
    per = p.n_samp // n_sub
    ipd = p.n_intervals // n_sub
    rows, src = [], None
    for k in range(n_sub):
        sl = slice(k * per, (k + 1) * per)
        pix = torch.from_numpy(p.pix[sl]).to(dev)
        psi = torch.from_numpy(p.psi[sl]).to(dev)
        lp = ctx.pointing(pix, psi, p.n_pix_total, p.min_hits)
        lp.set_grid(p.n_side)
        istart = p.interval_start[k * ipd:(k + 1) * ipd + 1] - k * per
        lf = ctx.polyfilter(lp, istart, np.ones(ipd), np.arange(0, per + 1, 256), 2)
        d = synth.signal_tod(p.pix[sl], p.psi[sl], p.signal) + \
            synth.rng_for(2, 10 + k, synth.STREAM_NOISE).standard_normal(per)
        b = ctx.rhs(lp, lf, torch.from_numpy(d).to(dev))
        Mbd = ctx.mbd(lp, lf)
        row = {"subset": k, "n_obs": lp.n_obs}

        def run(M):
            ((_, info), t) = _wall(lambda: ctx.solve(lp, lf, M, b, tol=1e-8, max_iter=3000,
                                                     check_every=1, history=True))
            h = info["history"]
            r100 = float(h[100]) if len(h) > 100 and h[100] >= 0 else float(info["rel_res_true"])
            return {"iters": info["iters"], "converged": info["converged"],
                    "rel_res_true": info["rel_res_true"], "res_at_100": r100, "solve_s": t}
        row["mbd"] = run(Mbd)
        if k == 0:
            (M2, t) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, b, k=32, eps_arn=1e-8, m_max=256))
            row["m2l_own"] = run(M2)
            row["m2l_own"]["setup_s"] = t
            src = (lp, M2)
        else:
            (Ms, t) = _wall(lambda: ctx.defl_transfer(src[0], src[1], lp, lf, Mbd))
            row["m2l_transferred"] = run(Ms)
            row["m2l_transferred"]["setup_s"] = t
            del Ms
            if k < full_m2l:
                (M2, t) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, b, k=32, eps_arn=1e-8,
                                                       m_max=256))
                row["m2l_own"] = run(M2)
                row["m2l_own"]["setup_s"] = t
                del M2
        rows.append(row)
        log(f"[bench] subset {k}: " + json.dumps({kk: vv for kk, vv in row.items()}))
        if k > 0:
            del lp
        del lf, Mbd, b
    summary, hist = {}, {}
    edges = [0, 20, 30, 40, 50, 60, 80, 100, 125, 150, 200, 300, 3000]
    for name in ("mbd", "m2l_transferred", "m2l_own"):
        its = [r[name]["iters"] for r in rows if name in r]
        res = [r[name]["res_at_100"] for r in rows if name in r]
        if not its:
            continue
        summary[name] = {"iters_to_1e-8": _stats(its), "residual_after_100": _stats(res),
                         "all_converged": all(r[name]["converged"] for r in rows if name in r),
                         "setup_s_median": float(np.median([r[name].get("setup_s", 0.0)
                                                            for r in rows if name in r]))}
        counts, _ = np.histogram(its, bins=edges)
        hist[name] = {f"[{a},{b_})": int(c) for a, b_, c in zip(edges[:-1], edges[1:], counts)}
    return {"form": "d1", "workload": f"config-2 scan split by detectors into {n_sub} subsets "
            f"({128 // n_sub} detectors, {per} samples each), quadratic polynomial filter per "
            "256-sample subscan, white noise; Z (k = 32) from subset 0 moved to the others, "
            "tol 1e-8", "summary": summary, "iteration_histograms": hist, "subsets": rows}


def form_z1(mm, ctx):
    """The eps_Arn x dim Z study of Sect. 6 (figs. eigenspectrum, binned_ritz
    and arntol_vs_dimZ) on a problem in the paper's regime: a 64 x 64 patch
    scanned by rasters whose passes are only 5 degrees apart (weak cross-
    linking, as constant-elevation scans give) and filtered by offset + slope
    per sweep (one 64-sample subscan), white noise.  Such a filter leaves a
    few tens of eigenvalues of M_BD A between ~1e-5 and 0.1, the rest near 1.
    One long Arnoldi run gives, per step, h_{j+1,j} and the relative residual
    of the Arnoldi solution of B x = r_0, hence the step at which each eps_Arn
    stops it under either reading of the stop test; for each eps_Arn, under
    the residual reading (the literal h_{j+1,j} test does not act here), the
    Ritz values of H_m (the library's host eigensolver), binned, and the PCG
    iterations to 1e-8 for several dim Z."""
    import torch
    import synth
    dev = torch.device("cuda", 0)
    p = synth.config2(n_side=64, grid=(4, 4), samp_per_det=1 << 16, L=1 << 14, half_bw=10,
                      angles_deg=(0.0, 5.0, -5.0))
    lp = ctx.pointing(torch.from_numpy(p.pix).to(dev), torch.from_numpy(p.psi).to(dev),
                      p.n_pix_total, p.min_hits)
    lp.set_grid(p.n_side)
    sub_len, order = p.n_side, 1
    lf = ctx.polyfilter(lp, p.interval_start, np.ones(p.n_intervals),
                        np.arange(0, p.n_samp + 1, sub_len), order)
    n_tmpl = (p.n_samp // sub_len) * (order + 1)
    d = synth.signal_tod(p.pix, p.psi, p.signal) + \
        synth.rng_for(2, 30, synth.STREAM_NOISE).standard_normal(p.n_samp)
    b = ctx.rhs(lp, lf, torch.from_numpy(d).to(dev))
    Mbd = ctx.mbd(lp, lf)
    ((_, i0), t0) = _wall(lambda: ctx.solve(lp, lf, Mbd, b, tol=1e-8, max_iter=3000,
                                           check_every=4, history=False))
    m_max = 500
    # Arnoldi starts from the initial residual r_0 = M_BD (b - A x_0) of a
    # seeded random guess x_0: with x_0 = 0 on white noise, M_BD b lies almost
    # wholly in the eigenvalue-1 eigenspace and h_21 is already below 1e-2
    x0 = torch.from_numpy(synth.rng_for(2, 31, synth.STREAM_SIGNAL).standard_normal(lp.n)).to(dev)
    seed = b - ctx.apply_A(lp, lf, x0)
    del x0
    # one long run: h_{j+1,j} and the Arnoldi solution's residual per step
    Mfull = ctx.defl_build(lp, lf, Mbd, seed, k=8, eps_arn=0.0, m_max=m_max)
    h = np.array(Mfull.h_history)
    fom = np.array(Mfull.res_history)
    del Mfull
    eps_list = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12)

    def first(a, eps):
        idx = np.flatnonzero(a <= eps)
        return int(idx[0]) + 1 if idx.size else None
    bins = np.array([0.0, 1e-4, 1e-3, 1e-2, 0.1, 0.3, 0.6, 0.9, 0.99, 1.01, 2.0, np.inf])
    rows = []
    for eps in eps_list:
        row = {"eps_arn": eps, "steps_residual_rule": first(fom, eps),
               "steps_h_rule": first(h, eps)}
        (M8, ts) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, seed, k=8, eps_arn=eps,
                                                m_max=m_max, stop="residual"))
        W, H = M8.arnoldi()
        m = H.shape[1]
        theta, _ = mm.hessenberg_eig(H[:m, :m])
        th = np.sort(theta.real)
        row["ritz_count"] = int(m)
        row["ritz_smallest"] = [float(v) for v in th[:8]]
        row["ritz_binned"] = {f"[{lo:g},{hi:g})": int(np.sum((th >= lo) & (th < hi)))
                              for lo, hi in zip(bins[:-1], bins[1:])}
        del W, M8
        row["dimZ"] = {}
        for k in (2, 5, 10, 15, 25, 35, 50):
            if k > m:
                continue
            (M2, ts) = _wall(lambda: ctx.defl_build(lp, lf, Mbd, seed, k=k, eps_arn=eps,
                                                    m_max=m_max, stop="residual"))
            ((_, info), t) = _wall(lambda: ctx.solve(lp, lf, M2, b, tol=1e-8, max_iter=3000,
                                                     check_every=4, history=False))
            row["dimZ"][k] = {"iters": info["iters"], "converged": info["converged"],
                              "solve_s": t, "setup_s": ts}
            del M2
        log(f"[bench] z1 {row}")
        rows.append(row)
    return {"form": "z1", "workload": f"64x64 patch, 16 detectors x 2^16 samples (2^20), raster "
            f"passes at 0/+5/-5 degrees, white noise, offset + slope per {sub_len}-sample sweep "
            f"({n_tmpl} templates), "
            "tol 1e-8; Arnoldi from r_0 = M_BD (b - A x_0), x_0 seeded N(0,1), stopped by the "
            "Arnoldi-solution residual <= eps_Arn (the h_{j+1,j} rule's step reported beside it), "
            "k smallest Ritz vectors",
            "n_unknowns": lp.n, "templates": n_tmpl,
            "mbd": {"iters": i0["iters"], "solve_s": t0},
            "h_history": {str(j): float(h[j - 1]) for j in [1, 5, 10] + list(range(25, m_max + 1, 25))
                          if j <= len(h)},
            "residual_history": {str(j): float(fom[j - 1])
                                 for j in [1, 5, 10] + list(range(25, m_max + 1, 25)) if j <= len(fom)},
            "rows": rows}


def form_c5(mm, ctx, n_requests=200, slots=1, rate=4.0, stop="h", cpu=True):
    """Serving: a Poisson trace (`rate` requests/s) over four recurring strategies
    of uneven size (2^20 to 2^27 samples, lambda 1,024 to 8,192), tolerance
    1e-6 or 1e-8.  Served by mm_server_* (cached pointing, M_BD and M_2l per
    strategy, continuous batching over `slots` columns) and, as the baseline,
    one request at a time with plain FP64 M_BD and no cache (pointing, noise
    model and M_BD built per request)."""
    import torch
    import synth
    import synth.gpu as sg
    from paper_1801_08937_amd import serving
    dev = torch.device("cuda", 0)
    arrivals, strat, tol = synth.poisson_arrivals(n_requests, rate, seed=0)
    S = []
    for s in range(4):
        t0 = time.perf_counter()
        p = synth.serve_strategy(s, 0, noiseless=True)
        n_det = synth.SERVE_STRATEGIES[s][1][0] * synth.SERVE_STRATEGIES[s][1][1]
        fk = synth.rng_for(50 + s, 0, synth.STREAM_FKNEE).uniform(0.05, 1.0, n_det)
        S.append({"p": p, "pix": torch.from_numpy(p.pix).to(dev),
                  "psi": torch.from_numpy(p.psi).to(dev), "fk": fk[p.filter_id]})
        if cpu:
            S[-1]["oracle"] = oracle_strategy_costs(p)
        p.pix = p.psi = p.tod = None
        log(f"[bench] strategy {s}: {S[-1]['pix'].numel()} samples "
            f"({time.perf_counter() - t0:.1f} s)")

    def make_tod(i):
        s = int(strat[i])
        st = S[s]
        sky = synth.white_sky(synth.rng_for(50 + s, 1000 + i, synth.STREAM_SIGNAL),
                              st["p"].n_pix_total)
        d = sg.signal(st["pix"], st["psi"], sky, dev)
        d += sg.noise_1f(50 + s, 1000 + i, synth.STREAM_NOISE, 1 << 16, st["fk"], dev)
        return d

    n_obs = []
    for s in range(4):
        lp = ctx.pointing(S[s]["pix"], S[s]["psi"], S[s]["p"].n_pix_total, S[s]["p"].min_hits)
        n_obs.append(lp.n)
        lp.close() if hasattr(lp, "close") else None
        del lp
    def serve(prebuild):
        srv = mm.Server(0, hbm_budget_bytes=240 << 30, slots=slots, defl_k=32, iters_per_step=4,
                        prebuild=prebuild,
                        arnoldi=None if stop == "h" else ("residual", 1e-10, 256))
        t0 = time.perf_counter()
        for s in range(4):
            p = S[s]["p"]
            srv.add_strategy(s, S[s]["pix"], S[s]["psi"], p.n_pix_total, p.interval_start,
                             p.filter_id, p.band, p.half_bw, grid_width=p.n_side)
        t_reg = time.perf_counter() - t0
        xs = {}

        def req(i):
            d = make_tod(i)
            _sync()
            x = torch.zeros(n_obs[int(strat[i])], dtype=torch.float64, device=dev)
            xs[i] = x
            return int(strat[i]), d, x, float(tol[i])
        log(f"[bench] serving trace (M_2l {'at registration' if prebuild else 'in background'}) ...")
        ready = {"t": None}

        def on_step(el):
            if ready["t"] is None and all(srv.strategy_state(s_) in (2, 3) for s_ in range(4)):
                ready["t"] = el
        infos, wall = serving.run_trace(srv, arrivals, req, on_step=on_step)
        served = serving.latency_stats(infos, wall)
        served["all_m2l_ready_at_s"] = ready["t"]
        steady = [i for i in range(n_requests)
                  if ready["t"] is not None and arrivals[i] >= ready["t"]]
        served["iters_mean"] = float(np.mean([d["iters"] for d in infos]))
        served["register_s"] = t_reg
        lat_s = np.array([d["latency_seconds"] for d in infos])
        served["per_strategy_p50_p99_s"] = {
            int(s_): [float(np.percentile(lat_s[strat == s_], 50)),
                      float(np.percentile(lat_s[strat == s_], 99))] for s_ in range(4)}
        if steady:
            served["steady_state"] = {"n": len(steady),
                                      "p50_s": float(np.percentile(lat_s[steady], 50)),
                                      "p99_s": float(np.percentile(lat_s[steady], 99)),
                                      "mean_s": float(lat_s[steady].mean())}
        slow = np.argsort(-lat_s)[:5]
        served["slowest"] = [{"i": int(i), "strategy": int(strat[i]), "tol": float(tol[i]),
                              "precond": int(infos[i]["precond"]),
                              "iters": int(infos[i]["iters"]),
                              "queue_s": float(infos[i]["queue_seconds"]),
                              "latency_s": float(lat_s[i])} for i in slow]
        log(f"[bench] served: {served}")
        srv.close()
        return served, xs, steady

    served, xs_srv, steady = serve(False)
    served_pre, _, _ = serve(True)
    # baseline: one at a time, FP64 M_BD, nothing cached
    log("[bench] baseline trace ...")
    lat, iters, diffs = [], [], []
    t_start = time.perf_counter()
    for i in range(n_requests):
        now = time.perf_counter() - t_start
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        s = int(strat[i])
        p = S[s]["p"]
        tg = time.perf_counter()
        d = make_tod(i)
        _sync()
        g = time.perf_counter() - tg
        lp = ctx.pointing(S[s]["pix"], S[s]["psi"], p.n_pix_total, p.min_hits)
        ln = ctx.noise(p.interval_start, p.filter_id, p.band, p.half_bw)
        M = ctx.mbd(lp, ln)
        b = ctx.rhs(lp, ln, d)
        x, info = ctx.solve(lp, ln, M, b, tol=float(tol[i]), max_iter=3000, check_every=4,
                            history=False)
        _sync()
        done = time.perf_counter() - t_start
        lat.append(done - arrivals[i] - g)
        iters.append(info["iters"])
        if i < 8:
            xa = xs_srv[i]
            diffs.append(float(torch.linalg.norm(xa - x) / torch.linalg.norm(x)))
        del lp, ln, M, b, x, d
    wall_b = time.perf_counter() - t_start
    lat = np.array(lat)
    if steady:
        steady_b = {"n": len(steady), "p50_s": float(np.percentile(lat[steady], 50)),
                    "p99_s": float(np.percentile(lat[steady], 99)),
                    "mean_s": float(lat[steady].mean())}
    else:
        steady_b = None
    per_b = {int(s_): [float(np.percentile(lat[strat == s_], 50)),
                       float(np.percentile(lat[strat == s_], 99))] for s_ in range(4)}
    base = {"per_strategy_p50_p99_s": per_b, "steady_state": steady_b, "n": n_requests, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "solves_per_s": n_requests / wall_b, "wall_s": wall_b,
            "iters_mean": float(np.mean(iters))}
    log(f"[bench] baseline: {base}")
    extra = {}
    if cpu:
        extra["cpu_baseline"] = oracle_trace_estimate([st["oracle"] for st in S], n_obs, strat,
                                                      iters)
    return {**extra, "form": "c5", "workload": f"Poisson {rate:g} req/s, 4 strategies: 64^2/16 det x 2^16 "
            "(lambda 1024), 128^2/32 x 2^18 (2048), 256^2/64 x 2^20 (4096), 256^2/128 x 2^20 "
            "(8192); tol 1e-6 or 1e-8; slots %d; background Arnoldi stop rule %s" % (slots, stop),
            "served": served,
            "served_m2l_at_registration": served_pre,
            "one_at_a_time_mbd_no_cache": base,
            "served_vs_baseline_map_rel_diff_first8": diffs}


if __name__ == "__main__":
    main()
