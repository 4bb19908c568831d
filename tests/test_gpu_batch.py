"""Persistent mixed-multiplicity batch on the GPU.

The batch kernel evaluates every event with fused colour-ordered tiles for
n <= 7 and colour-dressed chunks for n >= 8.  Colour-ordered segments in FP64
with n <= 6 equal bg_me2 on each segment alone bit for bit (the same tile
routine); bg_me2 evaluates n = 7 in FP64 in two stages (one straight path per
ordering, matrix-core colour sum), so there and otherwise the two agree
within the sum of their error bars (see _same).  Within the batch kernel the result does
not depend on tile or grid shape (bit for bit).  A few events of each segment
are also checked against the oracle directly.
"""
import numpy as np
import pytest

from bg_inputs import make_events, mixed_workload
from oracle import cdbg as ocdbg
from oracle import me2 as ome2
from oracle.conditioning import flow_amplitude_magnitude, me2_cobg_magnitude
from oracle.numeric import extended
from tests.helpers import U64, fp64_allowance, nonvanishing, reference_cobg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_06507_amd import api as a
    return a


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(*a):
    print(*a, flush=True)


def _segments(events):
    segs = []
    for n, ev in sorted(events.items()):
        col = _dev(ev["col"]) if n >= 8 else None
        segs.append({"n": n, "mom": _dev(ev["mom"]), "hel": _dev(ev["hel"]), "col": col,
                     "mode": "auto"})
    return segs


def _single(api, segs, precision):
    return [api.me2(s["mom"], s["hel"], s["col"], mode="auto", precision=precision) for s in segs]


FP32_MAX = 3e-4


def _same(segs, got, ref, precision, label=""):
    """Colour-ordered segments in FP64 with n <= 6: bit-identical.  Otherwise
    the two kernels may round differently (FP64 n = 7: bg_me2's two-stage
    path forms 1/P^2 from prefix sums and sums the colours in another order;
    FP32: multiply-add contraction, and an event near the check's threshold
    may be re-evaluated in FP64 by one path only; colour-dressed: the batch
    evaluates an event on 256 lanes, the single request on 64, 128 or 256, which
    splits the vertex sums differently).  Both sides meet their per-event
    bars, so they differ by at most twice a bar: FP32 2 FP32_MAX = 6e-4
    (median 1e-6); FP64 2e-12 relative, or for events above that twice the
    running error bound 12 (n - 2) u m of the oracle's magnitude (median
    1e-13).  For colour-dressed segments the zeros of invalid colour flows
    coincide."""
    for s, g, r in zip(segs, got, ref):
        g, r = g.cpu().numpy(), r.cpu().numpy()
        n = s["n"]
        if precision == "fp64" and n <= 6:
            assert np.array_equal(g, r), f"{label} n={n}"
            continue
        keep = nonvanishing(s["hel"].cpu().numpy())
        if n >= 8:
            # flows whose amplitude cancels to rounding may give an exact 0 on
            # one side only
            typical = np.median(np.abs(r[r != 0.0])) if (r != 0.0).any() else 0.0
            noise = (np.abs(r) < 1e-8 * typical) & (np.abs(g) < 1e-8 * typical)
            assert np.array_equal((g == 0.0) | noise, (r == 0.0) | noise), f"{label} n={n}"
            keep &= (np.abs(r) >= 1e-8 * typical) & (r != 0.0)
        if not keep.any():
            continue
        d = np.abs(g - r)
        rel = d[keep] / np.abs(r[keep])
        _say(f"  {label} n={n}: events differing {(g != r).sum()} of {g.size}, "
             f"rel diff median {np.median(rel):.1e} max {rel.max():.1e}")
        if precision == "fp32":
            assert np.median(rel) <= 1e-6 and rel.max() <= 2 * FP32_MAX, f"{label} n={n}"
            continue
        assert np.median(rel) <= 1e-13, f"{label} n={n}"
        over = np.nonzero(keep & (d > 2e-12 * np.abs(r)))[0][:40]
        if over.size:
            mom = s["mom"].cpu().numpy()[:, :, over]
            hel = s["hel"].cpu().numpy()[:, over]
            if n <= 7:
                _, m = me2_cobg_magnitude(mom, hel)
                allow = 2 * 12 * (n - 2) * U64 * m
            else:
                col = s["col"].cpu().numpy()[:, :, over]
                _, mA = flow_amplitude_magnitude(mom, hel, col)
                allow = 2 * 12 * (n - 2) * U64 * 2.0 * np.sqrt(np.abs(r[over])) * mA
            _say(f"  {over.size} events above 2e-12: max |d| / allowance "
                 f"{np.max(d[over] / allow):.2e}")
            assert np.all(d[over] <= allow), f"{label} n={n}"


def _small_mix():
    sizes = {4: 300, 5: 257, 6: 130, 7: 40, 8: 700, 9: 260}
    return {n: make_events(n, E, seed=7000 + n, cuts=True, sample_col=n >= 8)
            for n, E in sizes.items()}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_requests(api, precision):
    segs = _segments(_small_mix())
    _say(f"bg_me2_batch small mix {precision}: " + ", ".join(f"n={s['n']} E={s['mom'].shape[2]}" for s in segs))
    got = api.me2_batch(segs, precision)
    ref = _single(api, segs, precision)
    torch.cuda.synchronize()
    _same(segs, got, ref, precision, "batch vs single")


def test_batch_spot_checks_against_oracle(api):
    """FP64 batch against the long-double oracle, per event: within
    max(1e-12 |ref|, 12 (n - 2) u m) (helpers.fp64_allowance)."""
    ev = _small_mix()
    segs = _segments(ev)
    got = [g.cpu().numpy() for g in api.me2_batch(segs, "fp64")]
    for s, g in zip(segs, got):
        n = s["n"]
        e = ev[n]
        if n <= 7:
            idx = np.nonzero(nonvanishing(e["hel"]))[0][:4]
            ref, mag = reference_cobg(e["mom"][:, :, idx], e["hel"][:, idx])
        else:
            valid = ocdbg.is_valid_flow(e["col"])
            assert np.all(g[~valid] == 0.0)
            idx = np.nonzero(valid & nonvanishing(e["hel"]))[0][:3]
            m, h, c = e["mom"][:, :, idx], e["hel"][:, idx], e["col"][:, :, idx]
            ref = (np.abs(ocdbg.flow_amplitude(extended(m), h, c)) ** 2).astype(np.float64)
            _, mA = flow_amplitude_magnitude(m, h, c)
            mag = 2.0 * np.sqrt(ref) * mA
        d = np.abs(g[idx] - ref)
        _say(f"  n={n} oracle spot check max rel {np.max(d / np.abs(ref)):.2e}")
        assert np.all(d <= fp64_allowance(n, ref, mag))


@pytest.mark.parametrize("cfg", [
    dict(blocks_per_cu=1, cobg_tile_events=128, cdbg_tile_events=256, waves_per_simd=1),
    dict(blocks_per_cu=2, cobg_tile_events=256, cdbg_tile_events=512, waves_per_simd=2),
    dict(blocks_per_cu=0, cobg_tile_events=128, cdbg_tile_events=64, waves_per_simd=2),
    dict(blocks_per_cu=0, cobg_tile_events=8192, cdbg_tile_events=8192, waves_per_simd=1),
    dict(blocks_per_cu=0, cobg_tile_events=256, cdbg_tile_events=256, waves_per_simd=2,
         split_kinds=0),
    dict(blocks_per_cu=0, cobg_tile_events=128, cdbg_tile_events=256, waves_per_simd=1,
         split_kinds=0),
])
def test_batch_result_independent_of_config(api, cfg):
    """Other tiles and grid: bit-identical results; another kernel instance
    (the other register-budget variant, or one launch for every segment kind
    instead of one per kind): the same up to multiply-add contraction (FP32
    rounding)."""
    segs = _segments(_small_mix())
    ref = [r.clone() for r in api.me2_batch(segs, "fp32")]
    old = api.batch_config("fp32")
    try:
        api.set_batch_config("fp32", **cfg)
        _say(f"bg_me2_batch config {cfg}")
        got = api.me2_batch(segs, "fp32")
        torch.cuda.synchronize()
    finally:
        api.set_batch_config("fp32", **old)
    if cfg["waves_per_simd"] == 2 and cfg.get("split_kinds", 1) == old["split_kinds"]:
        for g, r in zip(got, ref):
            assert torch.equal(g, r)
    else:
        _same(segs, got, ref, "fp32", "other register budget")


def test_batch_rejects_bad_requests(api):
    from paper_2106_06507_amd._lib import BGError
    segs = _segments(_small_mix())
    with pytest.raises(ValueError):
        api.me2_batch([{"mom": segs[0]["mom"], "hel": None}], "fp32")
    with pytest.raises(BGError):  # colour-ordered mode above n = 7
        api.me2_batch([dict(segs[4], mode="cobg")], "fp32")
    with pytest.raises(BGError):  # colour-dressed without colours
        api.me2_batch([dict(segs[4], col=None, mode="cdbg")], "fp32")
    with pytest.raises(BGError):
        api.set_batch_config("fp32", cobg_tile_events=48)
    with pytest.raises(BGError):  # leading colour is not a batch mode
        api.me2_batch([dict(segs[0], mode="lc")], "fp32")
    with pytest.raises(BGError):  # nor the colour-sampled colour-ordered one (it synchronises)
        api.me2_batch([dict(segs[4], mode="comc")], "fp32")
    assert api.me2_batch([], "fp32") == []


def test_batch_fp32_against_oracle(api):
    """FP32 recursion in the batch kernel (with the FP64 re-evaluation of the
    listed events) against the FP64 oracle on a few events per segment
    (per-event relative error, non-vanishing helicities): within FP32_MAX."""
    ev = _small_mix()
    segs = _segments(ev)
    got = [g.cpu().numpy() for g in api.me2_batch(segs, "fp32")]
    for s, g in zip(segs, got):
        n = s["n"]
        e = ev[n]
        if n <= 7:
            idx = np.nonzero(nonvanishing(e["hel"]))[0][:8]
            ref = ome2.me2_cobg(e["mom"][:, :, idx], e["hel"][:, idx])
        else:
            idx = np.nonzero(ocdbg.is_valid_flow(e["col"]) & nonvanishing(e["hel"]))[0][:3]
            ref = np.abs(ocdbg.flow_amplitude(e["mom"][:, :, idx], e["hel"][:, idx],
                                              e["col"][:, :, idx])) ** 2
        rel = np.abs(g[idx] - ref) / np.abs(ref)
        _say(f"  n={n} fp32 oracle spot check median {np.median(rel):.1e} max {rel.max():.1e}")
        assert np.median(rel) < 1e-6 and rel.max() <= FP32_MAX


def test_batch_empty_and_tiny_segments(api):
    ev = {4: make_events(4, 1, seed=7100), 8: make_events(8, 3, seed=7101, sample_col=True),
          6: make_events(6, 33, seed=7102)}
    segs = _segments(ev)
    empty = {"n": 5, "mom": torch.empty((5, 4, 0), dtype=torch.float64, device="cuda"),
             "hel": torch.empty((5, 0), dtype=torch.int8, device="cuda"), "col": None}
    got = api.me2_batch(segs + [empty], "fp64")
    ref = _single(api, segs, "fp64")
    _same(segs, got, ref, "fp64", "tiny")
    assert got[-1].numel() == 0


def test_batch_graph_replays(api):
    """Recorded launch replayed several times, with eager work and
    synchronisation between replays; every replay equals the eager result."""
    segs = _segments(_small_mix())
    ref = [r.clone() for r in api.me2_batch(segs, "fp32")]
    single = api.me2(segs[2]["mom"], segs[2]["hel"], precision="fp32").clone()
    g = api.BatchGraph(segs, "fp32")
    for k in range(4):
        for o in g.outs:
            o.fill_(-1.0)
        outs = g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), f"replay {k}"
        # unrelated eager work between replays
        other = api.me2(segs[2]["mom"], segs[2]["hel"], precision="fp32")
        torch.cuda.synchronize()
        assert torch.equal(other, single)


def test_batch_autotune(api):
    segs = _segments(_small_mix())
    ref = [r.clone() for r in api.me2_batch(segs, "fp32")]
    old = api.batch_config("fp32")
    try:
        cfg, ms = api.batch_tune(segs, "fp32")
        _say(f"  tuned {cfg} {ms:.3f} ms")
        assert ms > 0
        assert api.batch_config("fp32") == cfg
        got = api.me2_batch(segs, "fp32")
        torch.cuda.synchronize()
    finally:
        api.set_batch_config("fp32", **old)
    # the same kernel instances (register budget, one launch per kind or for
    # all) give the same results bit for bit; other instances round
    # differently (see test_batch_result_independent_of_config)
    if (cfg["waves_per_simd"], cfg["split_kinds"]) == (old["waves_per_simd"], old["split_kinds"]):
        for g, r in zip(got, ref):
            assert torch.equal(g, r)
    else:
        _same(segs, got, ref, "fp32", "tuned config")


def test_full_size_mixed_batch(api):
    """The mixed workload at full size (n = 4..9, log-uniform counts in
    [2^10, 2^20]) in one launch, FP32 recursion: equal to the single-request
    results on every event."""
    ev = mixed_workload()
    segs = _segments(ev)
    _say("bg_me2_batch full mix: " + ", ".join(f"n={s['n']} E={s['mom'].shape[2]}" for s in segs))
    got = api.me2_batch(segs, "fp32")
    ref = _single(api, segs, "fp32")
    torch.cuda.synchronize()
    for g in got:
        assert torch.isfinite(g).all()
    _same(segs, got, ref, "fp32", "full mix")
