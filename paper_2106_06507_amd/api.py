"""Torch-facing wrappers around the C ABI.

PyTorch provides device memory and the current HIP stream; every step of the
computation runs in the library's kernels.  Inputs follow include/bg.h:
mom float64 [n, 4, E], hel int8 [n, E], col int8 [2, n, E], all on the GPU.
"""
import ctypes
import math
import threading

import torch

from . import _lib
from ._lib import bg_batch_config, bg_gen_params, bg_request, check, lib

_PREC = {"fp64": _lib.PREC_FP64, "fp32": _lib.PREC_FP32_MIXED, "mixed": _lib.PREC_FP32_MIXED,
         "fp32_unchecked": _lib.PREC_FP32_MIXED}
# precision names that add request flags: the plain FP32 recursion without the
# FP64 re-evaluation of ill-conditioned events
_PREC_FLAGS = {"fp32_unchecked": _lib.FLAG_FP32_UNCHECKED}
_MODE = {"cobg": _lib.MODE_COBG, "cdbg": _lib.MODE_CDBG, "auto": _lib.MODE_AUTO,
         "lc": _lib.MODE_LC, "comc": _lib.MODE_COMC}


class Context:
    """Owns a bg_context (colour matrices, workspace) on one device; flags
    (FLAG_* of the library) apply to every request made through it."""

    def __init__(self, device=None, flags=0):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        check(lib().bg_context_create(ctypes.byref(h), self.device, int(flags)), "bg_context_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().bg_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctx_lock = threading.Lock()
_contexts = {}


def default_context(device=None):
    if device is None:
        device = torch.cuda.current_device()
    with _ctx_lock:
        c = _contexts.get(device)
        if c is None:
            c = _contexts[device] = Context(device)
        return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_mom(mom):
    if not (mom.is_cuda and mom.dtype == torch.float64 and mom.dim() == 3 and mom.shape[1] == 4):
        raise ValueError("mom must be a CUDA float64 tensor [n, 4, E]")
    if not mom.is_contiguous():
        raise ValueError("mom must be contiguous")
    return mom.shape[0], mom.shape[2]


def _check_i8(t, shape, name):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.int8 and tuple(t.shape) == tuple(shape) and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA int8 tensor of shape {tuple(shape)}")
    return t


def num_orderings(n):
    return math.factorial(n - 2)


def colour_matrix(n):
    """Host-generated exact colour matrix C(n) (float64 CPU tensor [K, K])."""
    K = num_orderings(n)
    out = torch.empty((K, K), dtype=torch.float64)
    check(lib().bg_color_matrix(n, ctypes.c_void_p(out.data_ptr()), K * K), "bg_color_matrix")
    return out


def currents(mom, hel, precision="fp64", ctx=None, out=None):
    """Partial amplitudes A(1, sigma, n): float64 [2, K, E] (real, imaginary planes)."""
    n, E = _check_mom(mom)
    _check_i8(hel, (n, E), "hel")
    ctx = ctx or default_context(mom.device.index)
    shape = (2, num_orderings(n), E)
    amp = out if out is not None else torch.empty(shape, dtype=torch.float64, device=mom.device)
    if not (amp.is_cuda and amp.dtype == torch.float64 and tuple(amp.shape) == shape and amp.is_contiguous()):
        raise ValueError(f"out must be a contiguous CUDA float64 tensor {shape}")
    check(lib().bg_currents(ctx.handle, n, E, _ptr(mom), _ptr(hel), _PREC[precision], _ptr(amp),
                            _stream(mom.device)), "bg_currents")
    return amp


def color_contract(amp, n, out=None, accumulate=False, ctx=None):
    """|M|^2 = A^dagger C A per event from amp [2, K, E] (FP64)."""
    K = num_orderings(n)
    if not (amp.is_cuda and amp.dtype == torch.float64 and amp.shape[:2] == (2, K) and amp.is_contiguous()):
        raise ValueError(f"amp must be a contiguous CUDA float64 tensor [2, {K}, E]")
    E = amp.shape[2]
    ctx = ctx or default_context(amp.device.index)
    if out is None:
        out = torch.empty(E, dtype=torch.float64, device=amp.device)
    check(lib().bg_color_contract(ctx.handle, n, E, _ptr(amp), _ptr(out), int(accumulate),
                                  _stream(amp.device)), "bg_color_contract")
    return out


def _request(mom, hel, col, mode, precision, me2, validate=False):
    n, E = _check_mom(mom)
    _check_i8(hel, (n, E), "hel")
    _check_i8(col, (2, n, E), "col")
    r = bg_request()
    r.n = n
    r.mode = _MODE[mode]
    r.precision = _PREC[precision]
    r.flags = _PREC_FLAGS.get(precision, 0) | (_lib.FLAG_VALIDATE if validate else 0)
    r.n_events = E
    r.mom = mom.data_ptr()
    r.hel = hel.data_ptr() if hel is not None else None
    r.col = col.data_ptr() if col is not None else None
    r.me2 = me2.data_ptr() if me2 is not None else None
    return r


def me2(mom, hel=None, col=None, mode="cobg", precision="fp64", out=None, ctx=None,
        validate=False):
    """Per-event |M|^2 (float64 [E]); hel None sums over helicities (COBG).
    precision: "fp64", "fp32" (FP32 recursion with FP64 re-evaluation of
    ill-conditioned events) or "fp32_unchecked" (FP32 recursion only).
    validate: check the hel and col values on the device first."""
    n, E = _check_mom(mom)
    ctx = ctx or default_context(mom.device.index)
    if out is None:
        out = torch.empty(E, dtype=torch.float64, device=mom.device)
    r = _request(mom, hel, col, mode, precision, out, validate)
    check(lib().bg_me2(ctx.handle, ctypes.byref(r), _stream(mom.device)), "bg_me2")
    return out


def fp32_check(n, tau=None, mode="cobg", ctx=None):
    """Threshold of the FP32 accuracy check of `mode` ("cobg", "cdbg", "comc" or "lc") at n
    (bg_fp32_check_get/set): returns the current value; sets it first if tau
    is given."""
    ctx = ctx or default_context()
    m = _MODE[mode]
    if tau is not None:
        check(lib().bg_fp32_check_set(ctx.handle, m, n, ctypes.c_float(tau)), "bg_fp32_check_set")
    t = ctypes.c_float()
    check(lib().bg_fp32_check_get(ctx.handle, m, n, ctypes.byref(t)), "bg_fp32_check_get")
    return t.value


def me2_grad(mom, hel, grad_me2=None, precision="fp64", ctx=None, want_me2=True):
    """(me2 [E], grad [n, 4, E]) with grad = grad_me2 * d me2 / d mom."""
    n, E = _check_mom(mom)
    ctx = ctx or default_context(mom.device.index)
    out = torch.empty(E, dtype=torch.float64, device=mom.device) if want_me2 else None
    grad = torch.empty_like(mom)
    r = _request(mom, hel, None, "cobg", precision, out)
    if grad_me2 is not None:
        if not (grad_me2.is_cuda and grad_me2.dtype == torch.float64 and grad_me2.shape == (E,)):
            raise ValueError("grad_me2 must be a CUDA float64 tensor [E]")
        grad_me2 = grad_me2.contiguous()
    check(lib().bg_me2_grad(ctx.handle, ctypes.byref(r), _ptr(grad_me2), _ptr(grad),
                            _stream(mom.device)), "bg_me2_grad")
    return out, grad


class ME2(torch.autograd.Function):
    """Differentiable colour-summed |M|^2 (COBG, one helicity per event)."""

    @staticmethod
    def forward(ctx, mom, hel, precision="fp64"):
        ctx.save_for_backward(mom, hel)
        ctx.precision = precision
        return me2(mom, hel, precision=precision)

    @staticmethod
    def backward(ctx, grad_out):
        mom, hel = ctx.saved_tensors
        _, g = me2_grad(mom, hel, grad_me2=grad_out.contiguous(), precision=ctx.precision,
                        want_me2=False)
        return g, None, None


# ---------------------------------------------------------------- batches


def _segment(seg):
    """(mom, hel, col, mode) from a dict with keys mom, hel, col (optional), mode
    (optional, default "auto") or from such a tuple."""
    if isinstance(seg, dict):
        return seg["mom"], seg["hel"], seg.get("col"), seg.get("mode", "auto")
    mom, hel = seg[0], seg[1]
    col = seg[2] if len(seg) > 2 else None
    mode = seg[3] if len(seg) > 3 else "auto"
    return mom, hel, col, mode


def _batch_requests(segments, precision, outs):
    segs = [_segment(s) for s in segments]
    if len(segs) > _lib.BATCH_MAX_SEGS:
        raise ValueError(f"at most {_lib.BATCH_MAX_SEGS} segments per batch")
    if outs is None:
        outs = [torch.empty(m.shape[2], dtype=torch.float64, device=m.device) for m, _, _, _ in segs]
    arr = (bg_request * max(1, len(segs)))()
    for i, ((mom, hel, col, mode), out) in enumerate(zip(segs, outs)):
        if hel is None:
            raise ValueError("batch segments need helicities")
        arr[i] = _request(mom, hel, col, mode, precision, out)
    return arr, outs


def me2_batch(segments, precision="fp32", outs=None, ctx=None):
    """|M|^2 of several segments (mixed n, uneven sizes) in one persistent
    launch; returns one float64 [E_i] tensor per segment."""
    if not segments:
        return []
    dev = _segment(segments[0])[0].device
    ctx = ctx or default_context(dev.index)
    arr, outs = _batch_requests(segments, precision, outs)
    check(lib().bg_me2_batch(ctx.handle, arr, len(outs), _stream(dev)), "bg_me2_batch")
    return outs


def batch_config(precision="fp32", ctx=None):
    ctx = ctx or default_context()
    c = bg_batch_config()
    check(lib().bg_batch_config_get(ctx.handle, _PREC[precision], ctypes.byref(c)), "bg_batch_config_get")
    return {"blocks_per_cu": c.blocks_per_cu, "cobg_tile_events": c.cobg_tile_events,
            "cdbg_tile_events": c.cdbg_tile_events, "waves_per_simd": c.waves_per_simd,
            "split_kinds": c.split_kinds}


def set_batch_config(precision="fp32", ctx=None, **cfg):
    ctx = ctx or default_context()
    cur = batch_config(precision, ctx)
    cur.update(cfg)
    c = bg_batch_config(cur["blocks_per_cu"], cur["cobg_tile_events"], cur["cdbg_tile_events"],
                        cur["waves_per_simd"], cur["split_kinds"])
    check(lib().bg_batch_config_set(ctx.handle, _PREC[precision], ctypes.byref(c)), "bg_batch_config_set")


def batch_tune(segments, precision="fp32", ctx=None):
    """Run the library's autotuner on these segments; returns (config, ms)."""
    dev = _segment(segments[0])[0].device
    ctx = ctx or default_context(dev.index)
    arr, outs = _batch_requests(segments, precision, None)
    c = bg_batch_config()
    ms = ctypes.c_double()
    check(lib().bg_me2_batch_tune(ctx.handle, arr, len(outs), ctypes.byref(c), ctypes.byref(ms),
                                  _stream(dev)), "bg_me2_batch_tune")
    return {"blocks_per_cu": c.blocks_per_cu, "cobg_tile_events": c.cobg_tile_events,
            "cdbg_tile_events": c.cdbg_tile_events, "waves_per_simd": c.waves_per_simd,
            "split_kinds": c.split_kinds}, ms.value


class BatchGraph:
    """One bg_me2_batch launch recorded into a torch.cuda.CUDAGraph.

    The call is made once eagerly first, which builds the tile table and the
    workspace, so the recorded call only enqueues kernels.  replay() re-runs
    the batch on the same input tensors and writes the same output tensors
    (self.outs)."""

    def __init__(self, segments, precision="fp32", ctx=None):
        self.segments = list(segments)
        dev = _segment(self.segments[0])[0].device
        self.ctx = ctx or default_context(dev.index)
        self.outs = me2_batch(self.segments, precision, ctx=self.ctx)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            me2_batch(self.segments, precision, outs=self.outs, ctx=self.ctx)

    def replay(self):
        self.graph.replay()
        return self.outs


# ---------------------------------------------------------------- phase space


def me2_continuous(mom, phi, eta, precision="fp64", out=None, ctx=None):
    """A^2 per event (float64 [E]) for real polarization angles phi [n, E]
    and colour vectors eta [2, n, 3, E] (float64, CUDA); 9^n times its mean
    over uniform phi and sphere vectors is the colour- and helicity-summed
    |M|^2."""
    n, E = _check_mom(mom)
    if not (phi.is_cuda and phi.dtype == torch.float64 and tuple(phi.shape) == (n, E)):
        raise ValueError("phi must be a CUDA float64 tensor [n, E]")
    if not (eta.is_cuda and eta.dtype == torch.float64 and tuple(eta.shape) == (2, n, 3, E)):
        raise ValueError("eta must be a CUDA float64 tensor [2, n, 3, E]")
    phi = phi.contiguous()
    eta = eta.contiguous()
    ctx = ctx or default_context(mom.device.index)
    if out is None:
        out = torch.empty(E, dtype=torch.float64, device=mom.device)
    check(lib().bg_me2_continuous(ctx.handle, n, _PREC[precision], E, mom.data_ptr(), phi.data_ptr(),
                                  eta.data_ptr(), out.data_ptr(), _stream(mom.device)),
          "bg_me2_continuous")
    return out


def generate_continuous(n, n_events, seed, first_event=0, device=None, ctx=None):
    """(phi [n, E], eta [2, n, 3, E]) drawn on the device for bg_me2_continuous."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    ctx = ctx or default_context(dev.index)
    phi = torch.empty((n, n_events), dtype=torch.float64, device=dev)
    eta = torch.empty((2, n, 3, n_events), dtype=torch.float64, device=dev)
    check(lib().bg_generate_continuous(ctx.handle, n, seed, first_event, n_events, phi.data_ptr(),
                                       eta.data_ptr(), _stream(dev)), "bg_generate_continuous")
    return phi, eta


def generate(n, n_events, seed, n_attempts=None, first_attempt=0, cuts=True, sample_hel=True,
             sample_col=False, sqrt_s=1000.0, pt_min=20.0, dr_min=0.4, with_attempts=False,
             device=None, ctx=None):
    """Events generated on the device (RAMBO + cuts, helicities, colours).

    Tries n_attempts attempts from first_attempt (default: 2 n_events, or
    n_events without cuts) and returns a dict with mom [n, 4, E], hel, col,
    attempt (int64 [E], if with_attempts) and n_generated (a 0-d device
    tensor: min(accepted, n_events); slots beyond it are undefined).  Nothing
    is synchronised."""
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or default_context(device.index)
    if n_attempts is None:
        n_attempts = 2 * n_events if cuts else n_events
    E = int(n_events)
    mom = torch.empty((n, 4, E), dtype=torch.float64, device=device)
    hel = torch.empty((n, E), dtype=torch.int8, device=device) if sample_hel else None
    col = torch.empty((2, n, E), dtype=torch.int8, device=device) if sample_col else None
    att = torch.empty(E, dtype=torch.int64, device=device) if with_attempts else None
    ngen = torch.zeros((), dtype=torch.int64, device=device)
    p = bg_gen_params()
    p.n = n
    p.flags = (_lib.GEN_CUTS if cuts else 0) | (_lib.GEN_HEL if sample_hel else 0) | \
        (_lib.GEN_COL if sample_col else 0)
    p.sqrt_s, p.pt_min, p.dr_min = sqrt_s, pt_min, dr_min
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.first_attempt = first_attempt
    check(lib().bg_generate(ctx.handle, ctypes.byref(p), int(n_attempts), E, _ptr(mom), _ptr(hel),
                            _ptr(col), _ptr(att), _ptr(ngen), _stream(device)), "bg_generate")
    return {"mom": mom, "hel": hel, "col": col, "attempt": att, "n_generated": ngen}
