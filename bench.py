"""Benchmark: PCG map-making with M_2l vs M_BD on one MI355X.

Workload (default): the 256 x 256 patch, 128 detectors x 2^20 samples
(1.34e8 samples), cross-linked rasters, 1/f noise with f_knee ~ U[0.05, 1] Hz
per detector, N^-1 half bandwidth 4,096 applied by FFT over 2^16-sample
intervals, FP64, M_2l with k = 32 Ritz vectors (Arnoldi from M_BD b,
eps_Arn 1e-8, m_max 256) vs M_BD, tolerance 1e-8.  Inputs are seeded and
synthetic (see synth/).

A timed step is one PCG iteration with M_2l: q = A p (P, N^-1, P^T), the
M_2l apply, and the vector updates and reductions.  `value` is the A-apply
rate inside those iterations: samples per second = N_t * steps / time.  The
line also carries the pure A-apply rate, time to a 1e-8 residual for M_2l and
M_BD (with setup costs), the roofline of the dominant kernel and the oracle
timed on the host on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1] [--no-solves] [--no-cpu]
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

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per sample per kernel launch, FP64 (weights 16 B, index 4 B,
# TOD 8 B).  P: pixel index + weights + y written; P^T: permutation + sorted
# weights + z gathered; direct band: y + z.  The FFT's figure depends on the
# overlap-save geometry and is computed by fft_bytes_per_sample.
ALG_BYTES = {"P": 28.0, "PT": 28.0, "Ninv_band": 16.0}


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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1801_08937_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1801_08937_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(p, n_det_sample: int):
    """The FP64 oracle's A apply (FFT path) on the first n_det_sample
    detectors' samples of the same inputs, single process on the host."""
    import oracle as O
    spd = p.n_samp // 128 if p.n_samp >= 128 else p.n_samp
    ns = n_det_sample * spd
    n_int = int(np.searchsorted(p.interval_start, ns))
    pt = O.pointing_build(p.pix[:ns], p.psi[:ns], p.n_pix_total, 1)
    nz = O.noise_build(p.interval_start[: n_int + 1], p.filter_id[:n_int], p.band, p.half_bw)
    x = np.random.default_rng(0).standard_normal(pt.n)
    reps, t0 = 0, time.perf_counter()
    while True:
        O.apply_A(pt, nz, x, "fft")
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 5:
            break
    return {"value": ns * reps / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"A apply (numpy FFT path) on the first {n_det_sample} of 128 detectors "
                      f"({ns} samples) of the same inputs, {reps} applies in {el:.1f} s"}


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

    t = time.perf_counter()
    if args.workload == "c2":
        p = synth.config2()
        wl = ("config2: 256x256 patch (65,536 px, 196,608 unknowns), 128 det x 2^20 samples "
              "(1.34e8), 3-orientation cross-linked rasters, HWP psi, 1/f f_knee~U[0.05,1] Hz, "
              "N^-1 half-bandwidth 4096 by FFT over 2^16-sample intervals, FP64, "
              "M_2l k=32 vs M_BD, tol 1e-8")
    else:
        p = synth.config1()
        wl = ("config1: 32x32 patch, 2 det x 65,536 samples, lambda 32 direct band, FP64, "
              "M_BD and M_2l k=32, tol 1e-8")
    log(f"[bench] generated {p.name}: {p.n_samp} samples in {time.perf_counter() - t:.1f} s")
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
    M2 = timed("m2l_build_s", lambda: ctx.defl_build(lp, ln, Mbd, b, k=32, eps_arn=1e-8,
                                                      m_max=args.m_max))
    arn = M2.arnoldi_info
    log(f"[bench] Arnoldi m={arn.m} k={arn.k} h_last={arn.h_last:.2e}")

    solves = {}
    if not args.no_solves and not args.profile_only:
        for name, M in (("m2l", M2), ("mbd", Mbd)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = ctx.solve(lp, ln, M, b, tol=1e-8, max_iter=3000, check_every=4,
                                history=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            solves[name] = {"iters": info["iters"], "converged": info["converged"],
                            "rel_res_true": info["rel_res_true"], "solve_s": el,
                            "s_per_iter": el / max(info["iters"], 1)}
            log(f"[bench] solve {name}: {solves[name]}")
        solves["m2l"]["setup_s"] = setup["m2l_build_s"]
        solves["m2l"]["total_s"] = setup["m2l_build_s"] + solves["m2l"]["solve_s"]
        solves["mbd"]["total_s"] = solves["mbd"]["solve_s"]

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

    cpu = None
    if not args.no_cpu and not args.profile_only and args.workload == "c2":
        cpu = cpu_baseline(p, 32)
        log(f"[bench] cpu baseline: {cpu}")

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


if __name__ == "__main__":
    main()
