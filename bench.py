"""Benchmark: colour-summed |M|^2 events/s for gg -> 4g (n = 6 gluons).

Workload: 2^20 RAMBO points at sqrt(s) = 1 TeV with p_T > 20 GeV and
Delta R > 0.4, one uniformly sampled helicity configuration per event,
colour-ordered recursion over the 24 orderings plus the 24 x 24 colour-matrix
contraction (matrix cores).  One step = one bg_me2 call over the whole batch
with inputs resident in HBM.  The headline path is FP32 complex currents with
FP64 invariants and FP64 contraction; the plain FP64 path is timed beside it.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nonvanishing(hel):
    """Helicity configurations with a non-zero tree amplitude (>= 2 of each sign)."""
    m = np.sum(hel < 0, axis=0)
    return (m >= 2) & (m <= hel.shape[0] - 2)


def rel_err_stats(got, ref):
    rel = np.abs(got - ref) / np.abs(ref)
    return {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)), "max": float(rel.max())}


def time_calls(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps  # ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="events of the same workload timed on the oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the events are "
              "independent and a multi-GPU run would shard them by range.", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        ms = time_calls(lambda: dst.copy_(src), max(1, args.steps), 1)
        print(json.dumps({"copy_probe_bytes": nbytes, "ms": ms,
                          "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return
    from bg_inputs import workload
    from paper_2106_06507_amd import api, workmodel as wm

    n = 6
    log(f"generating gg -> 4g inputs: {args.events} events")
    ev = workload("gg_4g_n6", n_events=args.events)
    E = ev["mom"].shape[2]
    mom = torch.from_numpy(ev["mom"]).cuda()
    hel = torch.from_numpy(ev["hel"]).cuda()
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    ctx = api.default_context()

    def step32():
        api.me2(mom, hel, precision="fp32", out=out, ctx=ctx)

    def step64():
        api.me2(mom, hel, precision="fp64", out=out, ctx=ctx)

    # headline: FP32-recursion / FP64-contraction path, K timed steps
    log("timing fp32/mixed path")
    step32()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms32 = time_calls(step32, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    me2_32 = out.cpu().numpy().copy()
    log("timing fp64 path")
    ms64 = time_calls(step64, max(3, args.steps // 2), 1)
    me2_64 = out.cpu().numpy().copy()

    # dominant kernel (recursion) alone, same launch shape, on the current stream
    amp = torch.empty((2, 24, E), dtype=torch.float64, device="cuda")
    from paper_2106_06507_amd._lib import lib, check
    import ctypes

    def rec32():
        check(lib().bg_currents(ctx.handle, n, E, ctypes.c_void_p(mom.data_ptr()),
                                ctypes.c_void_p(hel.data_ptr()), 1, ctypes.c_void_p(amp.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "bg_currents")

    def rec64():
        check(lib().bg_currents(ctx.handle, n, E, ctypes.c_void_p(mom.data_ptr()),
                                ctypes.c_void_p(hel.data_ptr()), 0, ctypes.c_void_p(amp.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "bg_currents")

    kms32 = time_calls(rec32, args.steps, 1)
    kms64 = time_calls(rec64, max(3, args.steps // 2), 1)
    amp_t = amp.clone()

    def contr():
        api.color_contract(amp_t, n, out=out, ctx=ctx)

    cms = time_calls(contr, args.steps, 1)

    # accuracy against the FP64 oracle on a sample of events
    from oracle.me2 import me2_cobg
    idx = np.sort(np.random.default_rng(7).choice(E, min(E, 256), replace=False))
    ref = me2_cobg(ev["mom"][:, :, idx], ev["hel"][:, idx])
    scale = me2_cobg(ev["mom"][:, :, idx], None) / 2 ** n  # helicity-averaged |M|^2
    nz = nonvanishing(ev["hel"][:, idx])
    err32 = rel_err_stats(me2_32[idx][nz], ref[nz])
    err64 = rel_err_stats(me2_64[idx][nz], ref[nz])
    err32["scale_relative_max"] = float((np.abs(me2_32[idx] - ref) / scale)[nz].max())
    err64["scale_relative_max"] = float((np.abs(me2_64[idx] - ref) / scale)[nz].max())
    nz_all = nonvanishing(ev["hel"])
    err32_vs64 = rel_err_stats(me2_32[nz_all], me2_64[nz_all])

    flop_ev = wm.cobg_flops_per_event(n)
    achieved32 = flop_ev * E / (kms32 * 1e-3) / 1e12
    achieved64 = flop_ev * E / (kms64 * 1e-3) / 1e12
    cflop = wm.contraction_flops_per_event(n) * E / (cms * 1e-3) / 1e12

    cpu = None
    if not args.no_cpu:
        S = min(args.cpu_sample, E)
        log(f"timing the oracle on {S} events (1 thread)")
        t0 = time.perf_counter()
        me2_cobg(ev["mom"][:, :, :S], ev["hel"][:, :S])
        dt = time.perf_counter() - t0
        cpu = {"value": S / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": f"first {S} of the {E} gg->4g events, numpy FP64 oracle, single thread"}

    value = E / (ms32 * 1e-3)
    rec = {
        "metric": "|M|^2 events/sec per n-gluon multiplicity at stated rel. error vs FP64; % roofline",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 recursion + f64 contraction",
        "data": "synthetic: seeded RAMBO + cuts, sampled helicities",
        "config": {"workload": "gg->4g n=6 COBG 24 orderings + 24x24 colour matrix (MFMA)",
                   "n": n, "events": E, "sqrt_s_GeV": 1000.0, "cuts": "pT>20 GeV, dR>0.4",
                   "helicity": "sampled", "parallelism": "single GPU"},
        "rel_err_vs_oracle": {"events": int(nz.sum()), "fp32_mixed": err32, "fp64": err64,
                              "fp32_vs_fp64_all_nonvanishing": err32_vs64,
                              "note": "per-event |d|/|ref| and scale-relative |d|/S_e with S_e the "
                                      "helicity-averaged |M|^2 of the event; configurations with a "
                                      "vanishing tree amplitude excluded"},
        "fp64_path": {"value": E / (ms64 * 1e-3), "ms_per_step": ms64},
        "kernels_ms": {"recursion_fp32": kms32, "recursion_fp64": kms64, "contraction_mfma": cms},
        "roofline": {"bound": "alu", "kernel": "cobg_amp_kernel<6,float>", "achieved": achieved32,
                     "peak": wm.PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved32 / wm.PEAK_FP32_VALU_TFLOPS, "traffic": None,
                     "flops_per_event": flop_ev},
        "roofline_fp64": {"bound": "alu", "kernel": "cobg_amp_kernel<6,double>", "achieved": achieved64,
                          "peak": wm.PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                          "frac": achieved64 / wm.PEAK_FP64_VALU_TFLOPS},
        "roofline_contraction": {"bound": "mfma", "achieved": cflop, "peak": wm.PEAK_FP64_MFMA_TFLOPS,
                                 "unit": "TFLOP/s", "frac": cflop / wm.PEAK_FP64_MFMA_TFLOPS,
                                 "hbm_GBs": wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9},
        "cpu_baseline": cpu,
        "timed_wall_s": wall,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
