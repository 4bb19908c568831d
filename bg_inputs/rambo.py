"""RAMBO phase space, kinematic cuts and the sampled quantum numbers.

Phase-space points follow RAMBO (Kleiss, Stirling, Ellis, Comput. Phys.
Commun. 40 (1986) 359), massless case: each outgoing momentum is first drawn
isotropically with an energy from -log(r3 r4), then the set is boosted and
scaled so that the total four-momentum is (sqrt(s), 0, 0, 0).  The paper uses
RAMBO for all its methods (Section 3) with cuts p_T > 20 GeV and Delta R > 0.4
between outgoing gluons (Section 5); the workloads here keep those two cuts,
drop the pseudo-rapidity cut and run at sqrt(s) = 1 TeV.

Convention: all momenta are outgoing.  The two incoming beam gluons with
physical momenta (sqrt(s)/2)(1, 0, 0, +-1) enter as their negatives, as
gluons 1 and 2.  Arrays are structure-of-arrays with the event index fastest:
    mom [n][4][E] float64 (GeV), hel [n][E] int8 in {-1, +1},
    col [2][n][E] int8 with col[0] = i_k, col[1] = j_k in {0, 1, 2}.

Random numbers come from the keyed SplitMix64 stream of ``rng``; event
attempt t uses counter t.  Draw slots per attempt: 4 per outgoing gluon for
RAMBO, then one per gluon for the helicity, then two per gluon for the
colour-flow pair.  Accepted events are the first E attempts that pass the cuts,
so the result does not depend on how attempts are chunked.
"""
import math

import numpy as np

from .rng import splitmix64_uniform

SQRT_S_DEFAULT = 1000.0
PT_MIN = 20.0
DR_MIN = 0.4
BASE_SEED = 2106065070


def rambo_massless(u, sqrt_s):
    """Massless RAMBO for n_out particles.

    u: float64 [E, 4 * n_out] uniforms.  Returns p [E, n_out, 4] with the
    total momentum (sqrt_s, 0, 0, 0).
    """
    E = u.shape[0]
    n_out = u.shape[1] // 4
    r = u[:, : 4 * n_out].reshape(E, n_out, 4)
    c = 2.0 * r[..., 0] - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    f = 2.0 * math.pi * r[..., 1]
    q0 = -np.log(r[..., 2] * r[..., 3])
    q = np.stack([q0, q0 * s * np.cos(f), q0 * s * np.sin(f), q0 * c], axis=-1)
    Q = q.sum(axis=1)  # [E, 4]
    M = np.sqrt(Q[:, 0] ** 2 - Q[:, 1] ** 2 - Q[:, 2] ** 2 - Q[:, 3] ** 2)
    b = -Q[:, 1:] / M[:, None]
    x = sqrt_s / M
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    bq = np.einsum("ej,eij->ei", b, q[..., 1:])
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gam[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:]
        + b[:, None, :] * q[..., 0:1]
        + (a[:, None] * bq)[..., None] * b[:, None, :]
    )
    return p


def passes_cuts(p, pt_min=PT_MIN, dr_min=DR_MIN):
    """p_T > pt_min for each outgoing gluon and Delta R > dr_min for each pair.

    p: [E, n_out, 4].  Rapidity of a massless particle equals its
    pseudo-rapidity; Delta phi is wrapped into [-pi, pi].
    """
    pt = np.hypot(p[..., 1], p[..., 2])
    ok = np.all(pt > pt_min, axis=1)
    eta = np.arcsinh(p[..., 3] / pt)
    phi = np.arctan2(p[..., 2], p[..., 1])
    n_out = p.shape[1]
    for i in range(n_out):
        for j in range(i + 1, n_out):
            dphi = np.abs(phi[:, i] - phi[:, j])
            dphi = np.where(dphi > math.pi, 2.0 * math.pi - dphi, dphi)
            deta = eta[:, i] - eta[:, j]
            ok &= (deta * deta + dphi * dphi) > dr_min * dr_min
    return ok


def make_events(n, n_events, seed, sqrt_s=SQRT_S_DEFAULT, cuts=True,
                sample_hel=True, sample_col=False, chunk=1 << 16):
    """Generate n-gluon events.

    Returns dict with mom [n][4][E] float64, hel [n][E] int8 (or None),
    col [2][n][E] int8 (or None), and 'attempts' (RAMBO points drawn).
    """
    if n < 4:
        raise ValueError("need n >= 4 gluons")
    n_out = n - 2
    n_draw = 4 * n_out + n + 2 * n
    moms, hels, cols = [], [], []
    got = 0
    t0 = 0
    while got < n_events:
        need = n_events - got
        batch = max(chunk, int(need * 1.3) + 64) if cuts else need
        ctr = np.arange(t0, t0 + batch, dtype=np.uint64)
        u = splitmix64_uniform(seed, ctr, n_draw)
        p = rambo_massless(u[:, : 4 * n_out], sqrt_s)
        ok = passes_cuts(p) if cuts else np.ones(batch, dtype=bool)
        idx = np.nonzero(ok)[0][:need]
        moms.append(p[idx])
        uh = u[idx, 4 * n_out: 4 * n_out + n]
        hels.append(np.where(uh < 0.5, 1, -1).astype(np.int8))
        uc = u[idx, 4 * n_out + n:]
        cols.append(np.minimum((uc * 3.0).astype(np.int64), 2).astype(np.int8))
        got += idx.size
        if got >= n_events:
            t0 = t0 + int(idx[-1]) + 1 if idx.size else t0
            break
        t0 += batch
    p = np.concatenate(moms, axis=0)[:n_events]  # [E, n_out, 4]
    E = p.shape[0]
    mom = np.empty((n, 4, E), dtype=np.float64)
    half = 0.5 * sqrt_s
    mom[0, 0], mom[0, 1], mom[0, 2], mom[0, 3] = -half, 0.0, 0.0, -half
    mom[1, 0], mom[1, 1], mom[1, 2], mom[1, 3] = -half, 0.0, 0.0, half
    mom[2:] = np.transpose(p, (1, 2, 0))
    hel = np.ascontiguousarray(np.concatenate(hels, axis=0)[:n_events].T) if sample_hel else None
    col = None
    if sample_col:
        c = np.concatenate(cols, axis=0)[:n_events]  # [E, 2n]: (i_k, j_k) pairs
        col = np.empty((2, n, E), dtype=np.int8)
        col[0] = c[:, 0::2].T
        col[1] = c[:, 1::2].T
    return {"mom": np.ascontiguousarray(mom), "hel": hel, "col": col,
            "attempts": t0, "n": n, "sqrt_s": sqrt_s}


def mixed_counts(seed, ns=(4, 5, 6, 7, 8, 9), lo=10, hi=20):
    """Per-multiplicity event counts floor(2**(lo + (hi-lo) u_n))."""
    u = splitmix64_uniform(seed, np.arange(len(ns), dtype=np.uint64), 1)[:, 0]
    return {n: int(math.floor(2.0 ** (lo + (hi - lo) * ui))) for n, ui in zip(ns, u)}


# The five workloads: gluon multiplicity, events, cuts, what is sampled.
_WORKLOADS = {
    "gg_gg_n4_sumhel": dict(n=4, n_events=1024, cuts=False, sample_hel=False, sample_col=False, offset=0),
    "gg_4g_n6": dict(n=6, n_events=1 << 20, cuts=True, sample_hel=True, sample_col=False, offset=1),
    "gg_6g_n8_colour": dict(n=8, n_events=1 << 20, cuts=True, sample_hel=True, sample_col=True, offset=2),
    "gg_4g_n6_adjoint": dict(n=6, n_events=1 << 18, cuts=True, sample_hel=True, sample_col=False, offset=3),
}


def mixed_workload(seed=None, ns=(4, 5, 6, 7, 8, 9), scale=1.0):
    """Mixed-multiplicity batch: for each n, floor(scale * count) events with
    counts log-uniform in [2^10, 2^20] (mixed_counts), RAMBO at 1 TeV with the
    pT/dR cuts, sampled helicities, and sampled colour flows for n >= 8."""
    s = BASE_SEED + 4 if seed is None else seed
    counts = mixed_counts(s, ns)
    out = {}
    for k, n in enumerate(ns):
        E = max(1, int(math.floor(counts[n] * scale)))
        out[n] = make_events(n, E, seed=s + 100 * (k + 1), cuts=True, sample_hel=True,
                             sample_col=n >= 8)
    return out


def workload(name, n_events=None, seed=None):
    """Events of one named workload; n_events/seed override the defaults."""
    w = dict(_WORKLOADS[name])
    off = w.pop("offset")
    if n_events is not None:
        w["n_events"] = n_events
    s = BASE_SEED + off if seed is None else seed
    return make_events(seed=s, **w)
