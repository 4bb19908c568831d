"""Benchmark: colour-summed |M|^2 events/s for gg -> 4g (n = 6 gluons), FP64.

Headline workload: 2^20 RAMBO points at sqrt(s) = 1 TeV with p_T > 20 GeV and
Delta R > 0.4, one uniformly sampled helicity configuration per event,
colour-ordered recursion over the 24 orderings and the 24 x 24 colour sum,
all in FP64 (the paper's arithmetic).  One step = one bg_me2 call over the
whole batch with inputs resident in HBM; bg_me2 runs the recursion and the
colour sum in one fused kernel.

Beside it, on the same line: the FP32 recursion with FP64 re-evaluation of
the events its error bound lists (and the plain FP32 recursion), with their
per-event error against the FP64 path; the two-stage path (amplitudes
through memory, matrix-core contraction); gg -> gg with all helicities summed
(1024 points); the colour-dressed gg -> 6g workload (n = 8, sampled colour
flows); the adjoint d|M|^2/dp for gg -> 4g (2^18 events); the mixed-
multiplicity batch (n = 4..9) in one persistent launch replayed from a
recorded graph; phase space generated on the device ahead of the
evaluation; and events/s per gluon multiplicity n = 4..9.  Every kernel row
carries its algorithmic FLOP rate against the vector peak of its arithmetic
(paper_2106_06507_amd.workmodel).  The oracle is timed on the host on one
core and on all cores.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CSRC = os.path.join(ROOT, "paper_2106_06507_amd", "csrc")
# sources whose change invalidates the committed counter readings of the
# fused colour-ordered kernels
FUSED_SOURCES = ["bg_device.h", "bg_pair.h", "cobg_pair_impl.h", "cobg_path_impl.h", "cdbg_impl.h",
                 "fused_impl.h", "batch_impl.h", "batch.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
HEADLINE_KERNEL = "cobg_fused_kernel<6,double,false>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fused_source_hash():
    return source_hash(FUSED_SOURCES)


def stored_traffic(kernel, units):
    """HBM bytes per launch (FETCH + WRITE, calibrated) recorded for `kernel`
    in profiles/hbm_traffic.json, or None when there is no record for this
    unit count or the kernel's sources changed since it was measured."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("events") != units:
        return None
    if rec.get("source_hash") != source_hash(rec.get("sources", FUSED_SOURCES)):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def nonvanishing(hel):
    """Helicity configurations with a non-zero tree amplitude (>= 2 of each sign)."""
    m = np.sum(hel < 0, axis=0)
    return (m >= 2) & (m <= hel.shape[0] - 2)


def rel_err_stats(got, ref):
    rel = np.abs(got - ref) / np.abs(ref)
    return {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
            "max": float(rel.max()), "events": int(rel.size)}


def dressed_keep(hel, ref):
    """Valid flows, non-vanishing helicities, excluding flows that cancel to
    rounding (far below the median, where a relative error is undefined)."""
    keep = nonvanishing(hel) & (ref != 0.0)
    if keep.any():
        keep &= np.abs(ref) > 1e-8 * np.median(np.abs(ref[keep]))
    return keep


def time_events(fn, steps, warmup):
    """Average ms per call from HIP events recorded on the current stream
    (the stream every entry point is given)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(s)
    for _ in range(steps):
        fn()
    stop.record(s)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def roofline(kernel, flops_per_unit, units, ms, peak, what, **extra):
    """Algorithmic FLOP rate of a launch against a vector peak."""
    achieved = flops_per_unit * units / (ms * 1e-3) / 1e12
    row = {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak, "flops_per_unit": flops_per_unit,
           "units": units, "what": what, "traffic": stored_traffic(kernel, units)}
    row.update(extra)
    return row


def section_headline(args, api, wm, torch):
    from bg_inputs import workload
    from oracle.me2 import me2_cobg
    from oracle.numeric import extended
    n = 6
    log(f"gg->4g inputs: {args.events} events")
    ev = workload("gg_4g_n6", n_events=args.events)
    E = ev["mom"].shape[2]
    mom = torch.from_numpy(ev["mom"]).cuda()
    hel = torch.from_numpy(ev["hel"]).cuda()
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    ctx = api.default_context()

    def step(prec):
        return lambda: api.me2(mom, hel, precision=prec, out=out, ctx=ctx)

    log("timing the fused FP64 path (headline)")
    for _ in range(args.warmup):
        step("fp64")()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step("fp64")()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # the step is one kernel launch: its average duration from HIP events
    kms64 = time_events(step("fp64"), args.steps, 1)
    me2_64 = out.cpu().numpy().copy()
    log("timing the checked FP32 path and the plain FP32 recursion")
    kms32 = time_events(step("fp32"), args.steps, 1)
    me2_32 = out.cpu().numpy().copy()
    kms32u = time_events(step("fp32_unchecked"), args.steps, 1)
    me2_32u = out.cpu().numpy().copy()

    log("timing the two-stage path (amplitudes through memory, matrix-core contraction)")
    amp = torch.empty((2, 24, E), dtype=torch.float64, device="cuda")
    import ctypes
    from paper_2106_06507_amd._lib import check, lib

    def rec64():
        check(lib().bg_currents(ctx.handle, n, E, ctypes.c_void_p(mom.data_ptr()),
                                ctypes.c_void_p(hel.data_ptr()), 0, ctypes.c_void_p(amp.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
              "bg_currents")

    rms64 = time_events(rec64, max(3, args.steps // 2), 1)
    amp_t = amp.clone()
    cms = time_events(lambda: api.color_contract(amp_t, n, out=out, ctx=ctx), args.steps, 1)
    two_stage = out.cpu().numpy().copy()

    # FP64 against the long-double oracle on a sample (the per-event bar of
    # the tests: max(1e-12 |ref|, 12 (n - 2) u m))
    from oracle.conditioning import me2_cobg_magnitude
    idx = np.sort(np.random.default_rng(7).choice(E, min(E, 256), replace=False))
    m_s, h_s = ev["mom"][:, :, idx], ev["hel"][:, idx]
    ref = me2_cobg(extended(m_s), h_s).astype(np.float64)
    _, mag = me2_cobg_magnitude(m_s, h_s)
    nz = nonvanishing(h_s)
    allow = np.maximum(1e-12 * np.abs(ref), 12 * (n - 2) * 2.0 ** -53 * mag)
    err64 = rel_err_stats(me2_64[idx][nz], ref[nz])
    err64["max_over_bar"] = float(np.max(np.abs(me2_64[idx] - ref)[nz] / allow[nz]))
    err64_32 = rel_err_stats(me2_32[idx][nz], ref[nz])
    nz_all = nonvanishing(ev["hel"])
    e32 = rel_err_stats(me2_32[nz_all], me2_64[nz_all])
    e32u = rel_err_stats(me2_32u[nz_all], me2_64[nz_all])
    relisted = float(np.mean((me2_32 == me2_64)[nz_all] & (me2_32u != me2_64)[nz_all]))
    two_vs = rel_err_stats(two_stage[nz_all], me2_64[nz_all])

    rec_flops = wm.cobg_flops_per_event(n)
    col_flops = wm.colour_sum_flops_per_event(n)
    flops = rec_flops + col_flops
    traffic = stored_traffic(HEADLINE_KERNEL, E)

    rf = roofline(HEADLINE_KERNEL, flops, E, kms64, wm.PEAK_FP64_VALU_TFLOPS,
                  "recursion (prefix-shared walk) + fused colour sum, FP64 flops per event",
                  traffic=traffic, algorithmic_bytes=wm.cobg_bytes_per_event(n, amp_out=False) + 8,
                  hbm_GBs=(wm.cobg_bytes_per_event(n, amp_out=False) + 8) * E / (kms64 * 1e-3) / 1e9)
    row = {
        "value": E / (ms_step * 1e-3), "ms_per_step": ms_step, "wall_s": wall, "events": E,
        "kernel_ms": kms64,
        "rel_err_fp64_vs_long_double_oracle": dict(err64, note=(
            "256 sampled events; per-event bar max(1e-12 |ref|, 12 (n-2) u m) with m the "
            "oracle's magnitude: max_over_bar <= 1 means every event is within it")),
        "roofline": rf,
        "fp32_checked": {
            "value": E / (kms32 * 1e-3), "kernel_ms": kms32, "speedup_vs_fp64": kms64 / kms32,
            "rel_err_vs_fp64_all_events": e32, "rel_err_vs_long_double_oracle": err64_32,
            "reevaluated_fraction": relisted,
            "roofline": roofline("cobg_fused_kernel<6,float,false,true> + cobg_fix_kernel<6,false>",
                                 rec_flops + col_flops + relisted * (rec_flops + col_flops), E,
                                 kms32, wm.PEAK_FP32_VALU_NOPK_TFLOPS,
                                 "FP32 recursion + FP64 colour sum for every event, plus the FP64 "
                                 "evaluation of the re-evaluated fraction; peak: FP32 without "
                                 "packed instructions (= FP64 rate)",
                                 peak_published_fp32=wm.PEAK_FP32_VALU_TFLOPS),
            "note": "FP32 recursion; events whose running error bound is large against their "
                    "amplitudes are listed on the device and evaluated again in FP64"},
        "fp32_unchecked": {"value": E / (kms32u * 1e-3), "kernel_ms": kms32u,
                           "rel_err_vs_fp64_all_events": e32u},
        "two_stage_fp64": {
            "value": E / ((rms64 + cms) * 1e-3), "recursion_ms": rms64, "contraction_mfma_ms": cms,
            "rel_diff_vs_fused": two_vs,
            "roofline_contraction": dict(
                roofline("contract_mfma_kernel<24>", wm.contraction_flops_per_event(n), E, cms,
                         wm.PEAK_FP64_MFMA_TFLOPS, "A^dagger C A, K = 24, 4K^2 + 4K flops"),
                bound="mfma",
                hbm_GBs=wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9,
                hbm_frac=wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9 / wm.PEAK_HBM_GBS)},
    }
    return row, ev


def section_cfg1(args, api, wm, torch):
    """gg -> gg, 1024 points without cuts, all 16 helicities summed, FP64."""
    from bg_inputs import workload
    from oracle.me2 import me2_cobg
    from oracle.numeric import extended
    ev = workload("gg_gg_n4_sumhel")
    mom = torch.from_numpy(ev["mom"]).cuda()
    E = mom.shape[2]
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    log("timing gg->gg helicity sum")
    ms = time_events(lambda: api.me2(mom, None, precision="fp64", out=out), max(5, args.steps), 2)
    got = out.cpu().numpy()
    ref = me2_cobg(extended(ev["mom"]), None).astype(np.float64)
    flops = 16 * (wm.cobg_flops_per_event(4) + wm.colour_sum_flops_per_event(4))
    return {"workload": "gg->gg n=4, 1024 points without cuts, 16 helicities summed, FP64",
            "events": E, "ms": ms, "value": E / (ms * 1e-3),
            "rel_err_vs_long_double_oracle": rel_err_stats(got, ref),
            "roofline": roofline("cobg_fused_kernel<4,double,true>", flops, E, ms,
                                 wm.PEAK_FP64_VALU_TFLOPS,
                                 "16 x (recursion + colour sum); 1024 events fill 32 of the "
                                 "256 compute units: launch- and occupancy-bound by design")}


def section_cdbg(args, api, wm, torch):
    from bg_inputs import workload
    from oracle import cdbg as ocdbg
    from oracle.numeric import extended
    n = 8
    log("gg->6g colour-dressed inputs")
    ev = workload("gg_6g_n8_colour", n_events=args.events)
    E = ev["mom"].shape[2]
    mom, hel, col = (torch.from_numpy(ev[k]).cuda() for k in ("mom", "hel", "col"))
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    steps = max(2, args.steps // 4)
    ms, res = {}, {}
    for p in ("fp64", "fp32", "fp32_unchecked"):
        log(f"timing colour-dressed {p}")
        ms[p] = time_events(lambda: api.me2(mom, hel, col, mode="cdbg", precision=p, out=out),
                            steps, 1)
        res[p] = out.cpu().numpy().copy()
    valid = res["fp64"] != 0.0
    smp = np.random.default_rng(17).choice(E, min(E, 1 << 15), replace=False)
    flops_event = float(np.mean(wm.cdbg_flops_per_event(ev["col"][:, :, smp])))
    keep = dressed_keep(ev["hel"], res["fp64"])
    idx = np.nonzero(valid & nonvanishing(ev["hel"]))[0]
    idx = np.sort(np.random.default_rng(13).choice(idx, min(8, idx.size), replace=False))
    ref = (np.abs(ocdbg.flow_amplitude(extended(ev["mom"][:, :, idx]), ev["hel"][:, idx],
                                       ev["col"][:, :, idx])) ** 2).astype(np.float64)
    out_row = {
        "workload": "gg->6g n=8 colour-dressed, sampled helicities and colour flows",
        "events": E, "valid_fraction": float(valid.mean()),
        "flops_per_event": flops_event,
        "flops_per_valid_event": flops_event / max(float(valid.mean()), 1e-12),
    }
    for p, kern, peak in (("fp64", "cdbg_event_kernel<8,double,64>", wm.PEAK_FP64_VALU_TFLOPS),
                          ("fp32", "cdbg_event_kernel<8,float,64,true> + FP64 re-evaluation",
                           wm.PEAK_FP32_VALU_NOPK_TFLOPS),
                          ("fp32_unchecked", "cdbg_event_kernel<8,float,64>",
                           wm.PEAK_FP32_VALU_NOPK_TFLOPS)):
        r = {"value": E / (ms[p] * 1e-3), "ms": ms[p],
             "valid_events_per_s": valid.sum() / (ms[p] * 1e-3),
             "roofline": roofline(kern, flops_event, E, ms[p], peak,
                                  "contributing unordered splits (colour commutator) of the "
                                  "dressed recursion per sampled event "
                                  "(workmodel.cdbg_flops_per_event, mean over 2^15 events; "
                                  "invalid flows cost 0)")}
        if p == "fp64":
            r["rel_err_vs_long_double_oracle"] = rel_err_stats(res[p][idx], ref)
        else:
            r["rel_err_vs_fp64_valid_events"] = rel_err_stats(res[p][keep], res["fp64"][keep])
        out_row[p] = r
    return out_row


def section_adjoint(args, api, wm, torch):
    from bg_inputs import workload
    log("gg->4g adjoint inputs")
    ev = workload("gg_4g_n6_adjoint")
    E = ev["mom"].shape[2]
    mom, hel = torch.from_numpy(ev["mom"]).cuda(), torch.from_numpy(ev["hel"]).cuda()
    steps = max(2, args.steps // 4)
    flops = wm.adjoint_flops_per_event(6)
    row = {"workload": "gg->4g n=6, d|M|^2/dp for every momentum component", "events": E,
           "flops_per_event": flops}
    for p in ("fp64", "fp32"):
        log(f"timing adjoint {p}")
        ms = time_events(lambda: api.me2_grad(mom, hel, precision=p), steps, 1)
        row[p] = {"value": E / (ms * 1e-3), "ms": ms,
                  "roofline": roofline(f"cobg_amplitudes + contract_y + cobg_adj_kernel<6,{p}>",
                                       flops, E, ms,
                                       wm.PEAK_FP64_VALU_TFLOPS if p == "fp64"
                                       else wm.PEAK_FP32_VALU_NOPK_TFLOPS,
                                       "forward amplitudes + C A + per ordering recomputation "
                                       "and reverse sweep (workmodel.adjoint_flops_per_event)"),
                  "note": "one call = recursion, FP64 colour vector C A, reverse sweep"}
    return row


def section_batch(args, api, wm, torch):
    from bg_inputs import mixed_workload
    log("mixed batch inputs (n = 4..9)")
    ev = mixed_workload()
    segs = []
    flops = 0.0
    for n, e in sorted(ev.items()):
        segs.append({"mom": torch.from_numpy(e["mom"]).cuda(), "hel": torch.from_numpy(e["hel"]).cuda(),
                     "col": torch.from_numpy(e["col"]).cuda() if n >= 8 else None, "mode": "auto"})
        En = e["mom"].shape[2]
        if n <= 7:
            flops += En * (wm.cobg_flops_per_event(n) + wm.colour_sum_flops_per_event(n))
        else:
            smp = np.random.default_rng(n).choice(En, min(En, 1 << 14), replace=False)
            flops += En * float(np.mean(wm.cdbg_flops_per_event(e["col"][:, :, smp])))
    total = sum(s["mom"].shape[2] for s in segs)
    steps = max(2, args.steps // 4)
    row = {"workload": "mixed n=4..9, log-uniform counts in [2^10, 2^20], COBG n<=7, CDBG n>=8",
           "counts": {str(n): int(e["mom"].shape[2]) for n, e in sorted(ev.items())},
           "events": total, "flops_total": flops}
    for p in ("fp64", "fp32"):
        log(f"autotuning the batch kernel ({p})")
        cfg, tune_ms = api.batch_tune(segs, p)
        g = api.BatchGraph(segs, p)
        log("timing graph replays")
        ms = time_events(g.replay, steps, 1)
        single = []
        for s in segs:
            single.append(time_events(lambda s=s: api.me2(s["mom"], s["hel"], s["col"], mode="auto",
                                                          precision=p), steps, 1))
        kern = ("batch_kernel<double,W,plain>" if p == "fp64" else
                "batch_kernel<float,W,check> + fix_tiles_kernel + batch_kernel<double,W,fix>")
        row[p] = {"value": total / (ms * 1e-3), "ms": ms, "tuned_config": cfg,
                  "tune_best_ms": tune_ms,
                  "single_requests_ms": dict(zip([str(n) for n in sorted(ev)], single)),
                  "single_requests_total_ms": float(sum(single)),
                  "roofline": roofline(kern, flops / total, total, ms,
                                       wm.PEAK_FP64_VALU_TFLOPS if p == "fp64"
                                       else wm.PEAK_FP32_VALU_NOPK_TFLOPS,
                                       "sum over segments of the colour-ordered and colour-dressed "
                                       "work models")}
    return row


def section_pipeline(args, api, torch):
    """Phase space generated on the device (RAMBO + cuts + helicities) and fed
    to the fused evaluation: the whole Monte Carlo step with no host data."""
    n, E = 6, args.events
    steps = max(2, args.steps // 4)
    attempts = int(1.5 * E)  # acceptance of the cuts at n = 6 is ~0.86
    out = api.generate(n, E, 2106065070 + 11, n_attempts=attempts)
    me2 = torch.empty(E, dtype=torch.float64, device="cuda")

    def gen():
        api.generate(n, E, 2106065070 + 11, n_attempts=attempts)

    def both(prec):
        o = api.generate(n, E, 2106065070 + 11, n_attempts=attempts)
        api.me2(o["mom"], o["hel"], precision=prec, out=me2)

    log("timing device phase space + fused evaluation")
    gms = time_events(gen, steps, 1)
    pms = time_events(lambda: both("fp64"), steps, 1)
    torch.cuda.synchronize()
    return {"workload": "gg->4g n=6: RAMBO + cuts + sampled helicities on the device, then the "
                        "fused FP64 evaluation", "events": int(out["n_generated"]),
            "attempts": attempts, "generate_ms": gms, "pipeline_ms": pms,
            "value": E / (pms * 1e-3)}


def two_stage_row(api, wm, torch, n, mom, hel, steps):
    """Colour-ordered FP64 |M|^2 as two calls: the amplitudes of every ordering
    to memory (bg_currents), then the colour sum A^dagger C A (bg_color_contract:
    matrix cores with C in LDS for K = 24 and 120; for K = 720 C is rebuilt
    from its first row by relabelling)."""
    E = mom.shape[2]
    K = math.factorial(n - 2)
    amp = torch.empty((2, K, E), dtype=torch.float64, device="cuda")
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    log(f"timing n={n} two-stage: amplitudes, then the colour sum (K = {K})")
    rms = time_events(lambda: api.currents(mom, hel, "fp64", out=amp), steps, 1)
    cms = time_events(lambda: api.color_contract(amp, n, out=out), steps, 1)
    kern = ("relabel_contract_kernel<6> + relabel_reduce_kernel" if K == 720
            else f"contract_mfma_kernel<{K}>" if K in (24, 120) else f"contract_valu<{K}>")
    row = {"events": E, "K": K, "value": E / ((rms + cms) * 1e-3), "recursion_ms": rms,
           "contraction_ms": cms,
           "roofline_recursion": roofline({7: "cobg_path_kernel<7,double>", 8: "cobg_path_kernel_q<8>"}
                                          .get(n, f"cobg_pair_kernel<{n},double>"),
                                          wm.cobg_flops_per_event(n),
                                          E, rms, wm.PEAK_FP64_VALU_TFLOPS,
                                          "colour-ordered recursion, FP64 flops per event"),
           "roofline_contraction": dict(
               roofline(kern, wm.contraction_flops_per_event(n), E, cms, wm.PEAK_FP64_MFMA_TFLOPS,
                        f"A^dagger C A, K = {K}, 4K^2 + 4K flops"),
               bound="mfma",
               hbm_GBs=wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9,
               hbm_frac=wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9 / wm.PEAK_HBM_GBS)}
    if n == 8:
        me = torch.empty(E, dtype=torch.float64, device="cuda")
        row["me2_call_ms"] = time_events(lambda: api.me2(mom, hel, mode="cobg", out=me), steps, 1)
        row["me2_equals_two_stage"] = bool(torch.equal(me, out))
    return row


def section_two_stage(args, api, wm, torch):
    """Only the two-stage colour-ordered path (amplitudes to memory, then the
    colour sum) at n = 6, 7, 8: K = 24 and 120 on matrix cores, K = 720 from
    the first row of C.  Device-generated inputs; used for kernel profiles."""
    rows = {}
    steps = max(2, args.steps // 4)
    for n, E in ((6, args.events), (7, 1 << 18), (8, 1 << 16)):
        out = api.generate(n, E, 2106065070 + 40 + n, n_attempts=3 * E)
        torch.cuda.synchronize()
        if int(out["n_generated"]) < E:
            raise RuntimeError(f"device generator produced too few events at n={n}")
        rows[str(n)] = two_stage_row(api, wm, torch, n, out["mom"], out["hel"], steps)
    return rows


def section_per_n(args, api, wm, torch):
    """Events/s and roofline fraction per gluon multiplicity, FP64 and FP32
    (checked), with the FP32 error relative to the FP64 evaluation of the same
    events.  Inputs are generated on the device (RAMBO + cuts, sampled
    helicities; sampled colour flows and the colour-dressed recursion for
    n >= 8)."""
    rows = {}
    steps = max(2, args.steps // 4)
    for n in (4, 5, 6, 7, 8, 9):
        E = (1 << 18) if n == 7 else args.events
        cd = n >= 8
        out = api.generate(n, E, 2106065070 + 20 + n, n_attempts=3 * E, sample_col=True)
        torch.cuda.synchronize()
        got = int(out["n_generated"])
        if got < E:
            raise RuntimeError(f"device generator produced {got} < {E} events at n={n}")
        mom, hel, col = out["mom"], out["hel"], out["col"]
        mode = "cdbg" if cd else "cobg"
        h = hel.cpu().numpy()
        if cd:
            c = col.cpu().numpy()
            smp = np.random.default_rng(n).choice(E, min(E, 1 << 15), replace=False)
            flops = float(np.mean(wm.cdbg_flops_per_event(c[:, :, smp])))
        else:
            flops = wm.cobg_flops_per_event(n) + wm.colour_sum_flops_per_event(n)
        res, ms = {}, {}
        for p in ("fp64", "fp32", "fp32_unchecked"):
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            log(f"timing n={n} {mode} {p}")
            ms[p] = time_events(lambda: api.me2(mom, hel, col, mode=mode, precision=p, out=buf),
                                steps, 1)
            res[p] = buf.cpu().numpy()
        keep = dressed_keep(h, res["fp64"]) if cd else nonvanishing(h)
        row = {"mode": mode, "events": E, "flops_per_event": flops}
        for p in ("fp64", "fp32", "fp32_unchecked"):
            peak = wm.PEAK_FP64_VALU_TFLOPS if p == "fp64" else wm.PEAK_FP32_VALU_NOPK_TFLOPS
            r = {"events_per_s": E / (ms[p] * 1e-3), "ms": ms[p],
                 "tflops": flops * E / (ms[p] * 1e-3) / 1e12,
                 "roofline_frac": flops * E / (ms[p] * 1e-3) / 1e12 / peak}
            if p != "fp64":
                r["rel_err_vs_fp64"] = rel_err_stats(res[p][keep], res["fp64"][keep])
            row[p] = r
        # colour-sampled colour-ordered mode on the same sampled colour flows
        dres = res["fp64"] if cd else None
        if dres is None:
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            api.me2(mom, hel, col, mode="cdbg", precision="fp64", out=buf)
            dres = buf.cpu().numpy()
        co = {}
        ck = dressed_keep(h, dres)
        for p in ("fp32", "fp64"):
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            log(f"timing n={n} comc {p}")
            cms = time_events(lambda: api.me2(mom, hel, col, mode="comc", precision=p, out=buf),
                              steps, 1)
            co[p] = {"events_per_s": E / (cms * 1e-3), "ms": cms,
                     "rel_dev_from_dressed_fp64": rel_err_stats(buf.cpu().numpy()[ck], dres[ck])}
        row["colour_sampled_ordered"] = co
        row["valid_fraction"] = float((dres != 0.0).mean())
        if n in (7, 8):
            # full colour through memory: K = 120 on matrix cores, and K = 720
            # with the colour matrix held as its first row
            E2 = E if n == 7 else 1 << 16
            row["full_colour_ordered_two_stage_fp64"] = two_stage_row(
                api, wm, torch, n, mom[:, :, :E2].contiguous(), hel[:, :E2].contiguous(), steps)
        if not cd:
            # leading-colour mode on the same events: all (n-1)! orderings,
            # no colour matrix; its deviation from the full colour sum
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            lms = time_events(lambda: api.me2(mom, hel, mode="lc", precision="fp64", out=buf),
                              steps, 1)
            lc64 = buf.cpu().numpy()
            row["leading_colour_fp64"] = {
                "events_per_s": E / (lms * 1e-3), "ms": lms,
                "rel_dev_from_full_colour": rel_err_stats(lc64[keep], res["fp64"][keep])}
            buf32 = torch.empty(E, dtype=torch.float64, device="cuda")
            lms32 = time_events(lambda: api.me2(mom, hel, mode="lc", precision="fp32", out=buf32),
                                steps, 1)
            row["leading_colour_fp32_checked"] = {
                "events_per_s": E / (lms32 * 1e-3), "ms": lms32,
                "rel_err_vs_fp64": rel_err_stats(buf32.cpu().numpy()[keep], lc64[keep])}
        if args.continuous:
            Ec = min(E, 1 << (22 - n))
            phi_c, eta_c = api.generate_continuous(n, Ec, 2106065070 + 60 + n)
            mom_c = mom[:, :, :Ec].contiguous()
            cflops = wm.continuous_flops_per_event(n)
            cr = {}
            for p in ("fp32", "fp64"):
                buf = torch.empty(Ec, dtype=torch.float64, device="cuda")
                cms = time_events(lambda: api.me2_continuous(mom_c, phi_c, eta_c, precision=p,
                                                             out=buf), steps, 1)
                cr[p] = {"events_per_s": Ec / (cms * 1e-3), "ms": cms,
                         "tflops": cflops * Ec / (cms * 1e-3) / 1e12}
            row["continuous_colour_polarization"] = dict(cr, events=Ec, flops_per_event=cflops)
        rows[str(n)] = row
    return rows


def _oracle_chunk(args):
    from threadpoolctl import threadpool_limits
    from bg_inputs import workload
    from oracle.me2 import me2_cobg
    a, b, n_events = args
    ev = workload("gg_4g_n6", n_events=n_events)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        me2_cobg(ev["mom"][:, :, a:b], ev["hel"][:, a:b])
        return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(args, ev):
    """The oracle (numpy FP64, BLAS pools limited to one thread per process)
    on the headline events: one core on the first --cpu-sample events, then
    all cores the box gives this process (a process pool over 2^15-event
    chunks, at most 16 workers) on twice as many."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle.me2 import me2_cobg
    E = ev["mom"].shape[2]
    S = min(args.cpu_sample, E)
    log(f"timing the oracle on {S} events (1 core)")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for a in range(0, S, 1 << 15):
            b = min(S, a + (1 << 15))
            me2_cobg(ev["mom"][:, :, a:b], ev["hel"][:, a:b])
        dt1 = time.perf_counter() - t0
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(16, avail))
    S2 = min(E, 2 * S)
    chunks = [(a, min(S2, a + (1 << 15)), E) for a in range(0, S2, 1 << 15)]
    log(f"timing the oracle on {S2} events ({workers} processes)")
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_chunk, chunks[:workers])  # start-up and inputs, untimed
        t0 = time.perf_counter()
        pool.map(_oracle_chunk, chunks)
        dtn = time.perf_counter() - t0
    return {"value": S / dt1, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {S} of the {E} gg->4g events, numpy FP64 oracle, one thread "
                      f"({dt1:.1f} s)",
            "all_cores": {"value": S2 / dtn, "cores": workers, "seconds": dtn,
                          "sample": f"first {S2} events, {len(chunks)} chunks of 2^15 over "
                                    f"{workers} processes (one thread each)"},
            "nproc": os.cpu_count(), "cpus_available": avail, "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=1 << 20)
    ap.add_argument("--sections", default="cfg1,cdbg,adjoint,batch,pipeline,per_n",
                    help="extra rows beside the headline: any of cfg1, cdbg, adjoint, batch, "
                         "pipeline, per_n, two_stage (profiling only), or none")
    ap.add_argument("--continuous", action="store_true",
                    help="also time the continuous colour/polarization variant per n")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18,
                    help="events of the headline workload timed on the oracle (one core)")
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
        ms = time_events(lambda: dst.copy_(src), max(1, args.steps), 1)
        print(json.dumps({"copy_probe_bytes": nbytes, "ms": ms,
                          "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return
    from paper_2106_06507_amd import api, workmodel as wm

    head, ev = section_headline(args, api, wm, torch)
    sections = [s for s in args.sections.split(",") if s and s != "none"]
    extra = {}
    if "cfg1" in sections:
        extra["gg_gg_helicity_sum"] = section_cfg1(args, api, wm, torch)
    if "cdbg" in sections:
        extra["cdbg_gg_6g"] = section_cdbg(args, api, wm, torch)
    if "adjoint" in sections:
        extra["adjoint_gg_4g"] = section_adjoint(args, api, wm, torch)
    if "batch" in sections:
        extra["mixed_batch"] = section_batch(args, api, wm, torch)
    if "pipeline" in sections:
        extra["device_phase_space_pipeline"] = section_pipeline(args, api, torch)
    if "per_n" in sections:
        extra["per_multiplicity"] = section_per_n(args, api, wm, torch)
    if "two_stage" in sections:
        extra["two_stage_colour_ordered"] = section_two_stage(args, api, wm, torch)
    cpu = None if args.no_cpu else cpu_baseline(args, ev)

    rec = {
        "metric": "|M|^2 events/sec per n-gluon multiplicity at stated rel. error vs FP64; % roofline",
        "value": head["value"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded RAMBO + cuts, sampled helicities",
        "config": {"workload": "gg->4g n=6 COBG 24 orderings + 24x24 colour sum, fused kernel, FP64",
                   "n": 6, "events": head["events"], "sqrt_s_GeV": 1000.0,
                   "cuts": "pT>20 GeV, dR>0.4", "helicity": "sampled", "parallelism": "single GPU"},
        "kernel_ms": head["kernel_ms"],
        "rel_err_fp64_vs_long_double_oracle": head["rel_err_fp64_vs_long_double_oracle"],
        "roofline": head["roofline"],
        "fp32_checked": head["fp32_checked"],
        "fp32_unchecked": head["fp32_unchecked"],
        "two_stage_fp64": head["two_stage_fp64"],
        "cpu_baseline": cpu,
        "timed_wall_s": head["wall_s"],
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
