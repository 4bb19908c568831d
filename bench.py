"""Benchmark: colour-summed |M|^2 events/s for gg -> 4g (n = 6 gluons).

Headline workload: 2^20 RAMBO points at sqrt(s) = 1 TeV with p_T > 20 GeV and
Delta R > 0.4, one uniformly sampled helicity configuration per event,
colour-ordered recursion over the 24 orderings and the 24 x 24 colour sum.
One step = one bg_me2 call over the whole batch with inputs resident in HBM;
bg_me2 runs the recursion and the colour sum in one fused kernel.  The
headline path is FP32 complex currents with FP64 invariants and FP64 colour
sum; the plain FP64 path is timed beside it.

Further rows (same JSON line): the two-stage path with amplitudes through
memory and the matrix-core contraction, the colour-dressed gg -> 6g workload
(n = 8, sampled colour flows), the adjoint d|M|^2/dp for gg -> 4g (2^18
events), the mixed-multiplicity batch (n = 4..9) in one persistent launch
replayed from a recorded graph, phase space generated on the device ahead
of the evaluation, and events/s per gluon multiplicity n = 4..9 (FP32 and
FP64, with the FP32 error relative to FP64, and the colour-sampled
colour-ordered and leading-colour modes on the same events), and the
statistical efficiency of the colour treatments (colour sum, sampled flows,
continuous colours and polarizations) on shared phase-space points.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CSRC = os.path.join(ROOT, "paper_2106_06507_amd", "csrc")
# sources whose change invalidates the committed HBM counter readings of the
# fused colour-ordered kernel
FUSED_SOURCES = ["bg_device.h", "bg_pair.h", "cobg_pair_impl.h", "cdbg_impl.h", "fused_impl.h",
                 "batch.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused_source_hash():
    h = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def nonvanishing(hel):
    """Helicity configurations with a non-zero tree amplitude (>= 2 of each sign)."""
    m = np.sum(hel < 0, axis=0)
    return (m >= 2) & (m <= hel.shape[0] - 2)


def rel_err_stats(got, ref):
    rel = np.abs(got - ref) / np.abs(ref)
    return {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
            "max": float(rel.max())}


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


def section_headline(args, api, wm, torch):
    from bg_inputs import workload
    n = 6
    log(f"gg->4g inputs: {args.events} events")
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

    log("timing the fused FP32-recursion path (headline)")
    for _ in range(args.warmup):
        step32()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step32()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # the step is one kernel launch: its average duration from HIP events
    kms32 = time_events(step32, args.steps, 1)
    me2_32 = out.cpu().numpy().copy()
    log("timing the fused FP64 path")
    kms64 = time_events(step64, max(3, args.steps // 2), 1)
    me2_64 = out.cpu().numpy().copy()

    log("timing the two-stage path (amplitudes through memory, matrix-core contraction)")
    amp = torch.empty((2, 24, E), dtype=torch.float64, device="cuda")
    import ctypes
    from paper_2106_06507_amd._lib import check, lib

    def rec32():
        check(lib().bg_currents(ctx.handle, n, E, ctypes.c_void_p(mom.data_ptr()),
                                ctypes.c_void_p(hel.data_ptr()), 1, ctypes.c_void_p(amp.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
              "bg_currents")

    rms32 = time_events(rec32, args.steps, 1)
    amp_t = amp.clone()
    cms = time_events(lambda: api.color_contract(amp_t, n, out=out, ctx=ctx), args.steps, 1)
    two_stage = out.cpu().numpy().copy()

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
    two_vs_fused = rel_err_stats(two_stage[nz_all], me2_32[nz_all])

    rec_flops = wm.cobg_flops_per_event(n)
    col_flops = wm.colour_sum_flops_per_event(n)
    eq32 = rec_flops + 2 * col_flops  # FP32-equivalent: an FP64 flop costs two
    achieved32 = eq32 * E / (kms32 * 1e-3) / 1e12
    achieved64 = (rec_flops + col_flops) * E / (kms64 * 1e-3) / 1e12
    cflop = wm.contraction_flops_per_event(n) * E / (cms * 1e-3) / 1e12

    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        k = t.get("cobg_fused_kernel<6,float,false>")
        if k and k.get("source_hash") == fused_source_hash() and k.get("events") == E:
            traffic = k["fetch_bytes"] + k["write_bytes"]
    except (OSError, ValueError, KeyError):
        traffic = None

    row = {
        "value": E / (ms_step * 1e-3), "ms_per_step": ms_step, "wall_s": wall,
        "events": E, "kernel_ms": kms32,
        "fp64_path": {"value": E / (kms64 * 1e-3), "kernel_ms": kms64},
        "two_stage_fp32": {"value": E / ((rms32 + cms) * 1e-3), "recursion_ms": rms32,
                           "contraction_mfma_ms": cms,
                           "rel_diff_vs_fused_nonvanishing": two_vs_fused},
        "rel_err_vs_oracle": {
            "events": int(nz.sum()), "fp32_mixed": err32, "fp64": err64,
            "fp32_vs_fp64_all_nonvanishing": err32_vs64,
            "note": "per-event |d|/|ref| and scale-relative |d|/S_e with S_e the "
                    "helicity-averaged |M|^2 of the event; configurations with a "
                    "vanishing tree amplitude excluded"},
        "roofline": {"bound": "alu", "kernel": "cobg_fused_kernel<6,float,false>",
                     "achieved": achieved32, "peak": wm.PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved32 / wm.PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
                     "flops_per_event": eq32,
                     "peak_without_packed_fp32": wm.PEAK_FP32_VALU_NOPK_TFLOPS,
                     "frac_without_packed_fp32": achieved32 / wm.PEAK_FP32_VALU_NOPK_TFLOPS,
                     "note": "FP32 recursion flops + 2 x FP64 colour-sum flops per event "
                             "(FP64 vector rate is half the FP32 rate); the published FP32 "
                             "peak counts packed FP32 instructions, which this build does not "
                             "emit.  The flops are those of the vertex formulas as written per "
                             "vertex; the kernel shares the dot products of a range's splits "
                             "(coefficient collection) and fuses every product into a "
                             "multiply-add, so it executes fewer operations than counted and "
                             "frac_without_packed_fp32 can exceed 1"},
        "roofline_fp64": {"bound": "alu", "kernel": "cobg_fused_kernel<6,double,false>",
                          "achieved": achieved64, "peak": wm.PEAK_FP64_VALU_TFLOPS,
                          "unit": "TFLOP/s", "frac": achieved64 / wm.PEAK_FP64_VALU_TFLOPS},
        "roofline_contraction": {
            "bound": "mfma", "kernel": "contract_mfma_kernel<32>", "achieved": cflop,
            "peak": wm.PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": cflop / wm.PEAK_FP64_MFMA_TFLOPS,
            "hbm_GBs": wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9,
            "hbm_frac": wm.contraction_bytes_per_event(n) * E / (cms * 1e-3) / 1e9 / wm.PEAK_HBM_GBS},
    }
    return row, ev


def section_cdbg(args, api, torch):
    from bg_inputs import workload
    from oracle import cdbg as ocdbg
    n = 8
    log("gg->6g colour-dressed inputs")
    ev = workload("gg_6g_n8_colour", n_events=args.events)
    E = ev["mom"].shape[2]
    mom, hel, col = (torch.from_numpy(ev[k]).cuda() for k in ("mom", "hel", "col"))
    out = torch.empty(E, dtype=torch.float64, device="cuda")
    steps = max(2, args.steps // 4)
    ms = {}
    res = {}
    for p in ("fp32", "fp64"):
        log(f"timing colour-dressed {p}")
        ms[p] = time_events(lambda: api.me2(mom, hel, col, mode="cdbg", precision=p, out=out),
                            steps, 1)
        res[p] = out.cpu().numpy().copy()
    valid = res["fp64"] != 0.0
    idx = np.nonzero(valid & nonvanishing(ev["hel"]))[0]
    idx = np.sort(np.random.default_rng(13).choice(idx, min(6, idx.size), replace=False))
    ref = np.abs(ocdbg.flow_amplitude(ev["mom"][:, :, idx], ev["hel"][:, idx],
                                      ev["col"][:, :, idx])) ** 2
    return {
        "workload": "gg->6g n=8 colour-dressed, sampled helicities and colour flows",
        "events": E, "valid_fraction": float(valid.mean()),
        "fp32": {"value": E / (ms["fp32"] * 1e-3), "ms": ms["fp32"],
                 "valid_events_per_s": valid.sum() / (ms["fp32"] * 1e-3),
                 "rel_err_vs_oracle": rel_err_stats(res["fp32"][idx], ref)},
        "fp64": {"value": E / (ms["fp64"] * 1e-3), "ms": ms["fp64"],
                 "rel_err_vs_oracle": rel_err_stats(res["fp64"][idx], ref)},
    }


def section_adjoint(args, api, torch):
    from bg_inputs import workload
    log("gg->4g adjoint inputs")
    ev = workload("gg_4g_n6_adjoint")
    E = ev["mom"].shape[2]
    mom, hel = torch.from_numpy(ev["mom"]).cuda(), torch.from_numpy(ev["hel"]).cuda()
    steps = max(2, args.steps // 4)
    row = {"workload": "gg->4g n=6, d|M|^2/dp for every momentum component", "events": E}
    for p in ("fp32", "fp64"):
        log(f"timing adjoint {p}")
        ms = time_events(lambda: api.me2_grad(mom, hel, precision=p), steps, 1)
        row[p] = {"value": E / (ms * 1e-3), "ms": ms,
                  "note": "one call = recursion, FP64 colour vector C A, reverse sweep"}
    return row


def section_batch(args, api, torch):
    from bg_inputs import mixed_workload
    log("mixed batch inputs (n = 4..9)")
    ev = mixed_workload()
    segs = []
    for n, e in sorted(ev.items()):
        segs.append({"mom": torch.from_numpy(e["mom"]).cuda(), "hel": torch.from_numpy(e["hel"]).cuda(),
                     "col": torch.from_numpy(e["col"]).cuda() if n >= 8 else None, "mode": "auto"})
    total = sum(s["mom"].shape[2] for s in segs)
    log("autotuning the batch kernel")
    cfg, tune_ms = api.batch_tune(segs, "fp32")
    g = api.BatchGraph(segs, "fp32")
    steps = max(2, args.steps // 4)
    log("timing graph replays")
    ms = time_events(g.replay, steps, 1)
    single = []
    for s in segs:
        single.append(time_events(lambda s=s: api.me2(s["mom"], s["hel"], s["col"], mode="auto",
                                                      precision="fp32"), steps, 1))
    return {"workload": "mixed n=4..9, log-uniform counts in [2^10, 2^20], COBG n<=7, CDBG n>=8, FP32",
            "counts": {str(n): int(e["mom"].shape[2]) for n, e in sorted(ev.items())},
            "events": total, "value": total / (ms * 1e-3), "ms": ms, "tuned_config": cfg,
            "tune_best_ms": tune_ms, "single_requests_ms": dict(zip([str(n) for n in sorted(ev)], single)),
            "single_requests_total_ms": float(sum(single))}


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

    def both():
        o = api.generate(n, E, 2106065070 + 11, n_attempts=attempts)
        api.me2(o["mom"], o["hel"], precision="fp32", out=me2)

    log("timing device phase space + fused evaluation")
    gms = time_events(gen, steps, 1)
    pms = time_events(both, steps, 1)
    torch.cuda.synchronize()
    return {"workload": "gg->4g n=6: RAMBO + cuts + sampled helicities on the device, then the "
                        "fused FP32 evaluation", "events": int(out["n_generated"]),
            "attempts": attempts, "generate_ms": gms, "pipeline_ms": pms,
            "value": E / (pms * 1e-3)}


def section_per_n(args, api, torch):
    from paper_2106_06507_amd import workmodel as wm
    """Events/s per gluon multiplicity, FP32 recursion and FP64, with the
    FP32 error relative to the FP64 evaluation of the same events.  Inputs are
    generated on the device (RAMBO + cuts, sampled helicities; sampled colour
    flows and the colour-dressed recursion for n >= 8)."""
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
        res, ms = {}, {}
        for p in ("fp32", "fp64"):
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            log(f"timing n={n} {mode} {p}")
            ms[p] = time_events(lambda: api.me2(mom, hel, col, mode=mode, precision=p, out=buf),
                                steps, 1)
            res[p] = buf.cpu().numpy()
        h = hel.cpu().numpy()
        keep = nonvanishing(h) & (res["fp64"] != 0.0)
        err = rel_err_stats(res["fp32"][keep], res["fp64"][keep])
        # against the typical size of |M|^2 at this n: cancelling helicity or
        # colour configurations make the per-event ratio meaningless
        typical = float(np.median(np.abs(res["fp64"][keep])))
        err["scale_relative_max"] = float(np.max(np.abs(res["fp32"][keep] - res["fp64"][keep])) / typical)
        rows[str(n)] = {
            "mode": mode, "events": E,
            "fp32": {"events_per_s": E / (ms["fp32"] * 1e-3), "ms": ms["fp32"]},
            "fp64": {"events_per_s": E / (ms["fp64"] * 1e-3), "ms": ms["fp64"]},
            "fp32_rel_err_vs_fp64": err,
            "note": "per-event |d|/|fp64| on non-vanishing helicities; scale_relative_max = "
                    "max |d| / median |fp64|",
        }
        # colour-sampled colour-ordered mode on the same sampled colour flows:
        # the orderings whose colour chain closes, each by the colour-ordered
        # recursion; deviation from the dressed recursion in FP64
        dres = res["fp64"] if cd else None
        if dres is None:
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            api.me2(mom, hel, col, mode="cdbg", precision="fp64", out=buf)
            dres = buf.cpu().numpy()
        co = {}
        for p in ("fp32", "fp64"):
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            log(f"timing n={n} comc {p}")
            cms = time_events(lambda: api.me2(mom, hel, col, mode="comc", precision=p, out=buf),
                              steps, 1)
            got_c = buf.cpu().numpy()
            ck = nonvanishing(h) & (dres != 0.0)
            ck &= np.abs(dres) > 1e-8 * np.median(np.abs(dres[ck]))
            co[p] = {"events_per_s": E / (cms * 1e-3), "ms": cms,
                     "rel_dev_from_dressed_fp64": rel_err_stats(got_c[ck], dres[ck])}
        rows[str(n)]["colour_sampled_ordered"] = co
        # continuous colours and real polarizations (all-real dressed
        # recursion) on the first Ec of these points
        Ec = min(E, 1 << (22 - n))
        phi_c, eta_c = api.generate_continuous(n, Ec, 2106065070 + 60 + n)
        mom_c = mom[:, :, :Ec].contiguous()
        cres, cms = {}, {}
        for p in ("fp32", "fp64"):
            buf = torch.empty(Ec, dtype=torch.float64, device="cuda")
            log(f"timing n={n} continuous {p}")
            cms[p] = time_events(lambda: api.me2_continuous(mom_c, phi_c, eta_c, precision=p, out=buf),
                                 steps, 1)
            cres[p] = buf.cpu().numpy()
        flops = wm.continuous_flops_per_event(n)
        ck = cres["fp64"] > 1e-3 * np.median(cres["fp64"])
        cerr = rel_err_stats(cres["fp32"][ck], cres["fp64"][ck])
        cerr["max_abs_over_max"] = float(np.max(np.abs(cres["fp32"] - cres["fp64"])) / np.max(cres["fp64"]))
        rows[str(n)]["continuous_colour_polarization"] = {
            "events": Ec, "flops_per_event": flops,
            "fp32": {"events_per_s": Ec / (cms["fp32"] * 1e-3), "ms": cms["fp32"],
                     "tflops": flops * Ec / (cms["fp32"] * 1e-3) / 1e12,
                     "frac_of_fp32_without_packed": flops * Ec / (cms["fp32"] * 1e-3) / 1e12
                     / wm.PEAK_FP32_VALU_NOPK_TFLOPS},
            "fp64": {"events_per_s": Ec / (cms["fp64"] * 1e-3), "ms": cms["fp64"],
                     "tflops": flops * Ec / (cms["fp64"] * 1e-3) / 1e12,
                     "frac_of_fp64": flops * Ec / (cms["fp64"] * 1e-3) / 1e12 / wm.PEAK_FP64_VALU_TFLOPS},
            "fp32_rel_err_vs_fp64": cerr}
        rows[str(n)]["valid_fraction"] = float((dres != 0.0).mean())
        if not cd:
            # leading-colour mode on the same events: all (n-1)! orderings,
            # no colour matrix; its deviation from the full colour sum
            buf = torch.empty(E, dtype=torch.float64, device="cuda")
            lms = time_events(lambda: api.me2(mom, hel, mode="lc", precision="fp32", out=buf),
                              steps, 1)
            lc = buf.cpu().numpy()
            rows[str(n)]["leading_colour_fp32"] = {
                "events_per_s": E / (lms * 1e-3), "ms": lms,
                "rel_dev_from_full_colour": rel_err_stats(lc[keep], res["fp64"][keep])}
    return rows


def section_sampling(args, api, torch):
    """Statistical efficiency of the colour treatments.  Each method gives an
    unbiased per-event estimate w of the colour- and helicity-summed |M|^2:
      colour-summed colour-ordered, sampled helicity:   2^n |M_h|^2 (n <= 7)
      colour-dressed or colour-sampled colour-ordered,
        uniform colour flow and helicity:               2^n 9^n |A_flow,h|^2
      continuous colours and polarizations:             9^n A^2
    To separate the colour/helicity variance from the phase-space variance,
    64 device-generated phase-space points are each repeated 4096 times with
    independent colour and helicity samples.  Per point the relative variance
    var(w)/mean(w)^2 is taken; reported: its median over the points, the
    events/s of the method (FP32) and the effective rate events/s /
    (1 + median relative variance), i.e. colour- and helicity-exact
    equivalent events per second at a fixed phase-space point."""
    out = {}
    steps = max(2, args.steps // 8)
    P, R = 64, 4096
    E = P * R
    for n in (6, 8):
        g = api.generate(n, E, 2106065070 + 40 + n, n_attempts=3 * E, sample_col=True)
        torch.cuda.synchronize()
        if int(g["n_generated"]) < E:
            raise RuntimeError(f"device generator produced too few events at n={n}")
        mom = g["mom"][:, :, :P].repeat_interleave(R, dim=2).contiguous()
        hel, col = g["hel"], g["col"]
        phi, eta = api.generate_continuous(n, E, 2106065070 + 50 + n)
        buf = torch.empty(E, dtype=torch.float64, device="cuda")
        runs = []
        if n <= 7:
            runs.append(("colour_summed_ordered", 2.0 ** n,
                         lambda: api.me2(mom, hel, precision="fp32", out=buf)))
        runs.append(("colour_dressed_flow", 2.0 ** n * 9.0 ** n,
                     lambda: api.me2(mom, hel, col, mode="cdbg", precision="fp32", out=buf)))
        runs.append(("colour_sampled_ordered_flow", 2.0 ** n * 9.0 ** n,
                     lambda: api.me2(mom, hel, col, mode="comc", precision="fp32", out=buf)))
        runs.append(("continuous_colour_polarization", 9.0 ** n,
                     lambda: api.me2_continuous(mom, phi, eta, precision="fp32", out=buf)))
        row = {"points": P, "samples_per_point": R}
        exact = None
        if n <= 7:
            exact = api.me2(g["mom"][:, :, :P].contiguous(), None, precision="fp64").cpu().numpy()
        for name, scale, fn in runs:
            log(f"timing sampling n={n} {name}")
            ms = time_events(fn, steps, 1)
            w = (scale * buf.cpu().numpy()).reshape(P, R)
            mean = w.mean(axis=1)
            rv = w.var(axis=1) / mean ** 2
            rate = E / (ms * 1e-3)
            r = {"ms": ms, "events_per_s": rate,
                 "rel_variance_median": float(np.median(rv)),
                 "rel_variance_mean": float(np.mean(rv)),
                 "effective_events_per_s": rate / (1.0 + float(np.median(rv)))}
            if exact is not None:
                # per-point sample mean against the exact colour and helicity sum
                pull = (mean - exact) / (w.std(axis=1) / np.sqrt(R))
                r["pull_vs_exact_sum"] = {"median_abs": float(np.median(np.abs(pull))),
                                          "max_abs": float(np.max(np.abs(pull)))}
            row[name] = r
        out[str(n)] = row
    return out


def cpu_baseline(args, ev):
    """The oracle on the first --cpu-sample headline events, one thread (BLAS
    pools limited to 1), in chunks of 2^15 events to bound memory."""
    from threadpoolctl import threadpool_limits
    from oracle.me2 import me2_cobg
    E = ev["mom"].shape[2]
    S = min(args.cpu_sample, E)
    log(f"timing the oracle on {S} events (1 thread)")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for a in range(0, S, 1 << 15):
            b = min(S, a + (1 << 15))
            me2_cobg(ev["mom"][:, :, a:b], ev["hel"][:, a:b])
        dt = time.perf_counter() - t0
    return {"value": S / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {S} of the {E} gg->4g events (numpy FP64 oracle, one thread, "
                      f"{dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=1 << 20)
    ap.add_argument("--sections", default="cdbg,adjoint,batch,pipeline,per_n,sampling",
                    help="extra rows beside the headline: any of cdbg, adjoint, batch, "
                         "pipeline, per_n, sampling, or none")
    ap.add_argument("--cpu-sample", type=int, default=1 << 19,
                    help="events of the headline workload timed on the oracle")
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
    if "cdbg" in sections:
        extra["cdbg_gg_6g"] = section_cdbg(args, api, torch)
    if "adjoint" in sections:
        extra["adjoint_gg_4g"] = section_adjoint(args, api, torch)
    if "batch" in sections:
        extra["mixed_batch"] = section_batch(args, api, torch)
    if "pipeline" in sections:
        extra["device_phase_space_pipeline"] = section_pipeline(args, api, torch)
    if "per_n" in sections:
        extra["per_multiplicity"] = section_per_n(args, api, torch)
    if "sampling" in sections:
        extra["sampling_efficiency"] = section_sampling(args, api, torch)
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
        "dtype": "f32 recursion + f64 colour sum",
        "data": "synthetic: seeded RAMBO + cuts, sampled helicities",
        "config": {"workload": "gg->4g n=6 COBG 24 orderings + 24x24 colour sum, fused kernel",
                   "n": 6, "events": head["events"], "sqrt_s_GeV": 1000.0,
                   "cuts": "pT>20 GeV, dR>0.4", "helicity": "sampled", "parallelism": "single GPU"},
        "kernel_ms": head["kernel_ms"],
        "fp64_path": head["fp64_path"],
        "two_stage_fp32": head["two_stage_fp32"],
        "rel_err_vs_oracle": head["rel_err_vs_oracle"],
        "roofline": head["roofline"],
        "roofline_fp64": head["roofline_fp64"],
        "roofline_contraction": head["roofline_contraction"],
        "cpu_baseline": cpu,
        "timed_wall_s": head["wall_s"],
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
