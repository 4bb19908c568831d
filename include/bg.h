/*
 * bg.h -- C ABI of the MI355X (gfx950) n-gluon tree-amplitude library.
 *
 * The library evaluates tree-level n-gluon squared matrix elements |M|^2 with
 * the Berends-Giele recursion of "Many-gluon tree amplitudes on modern GPUs"
 * (Bothmann, Giele, Hoeche, Isaacson, Knobbe, arXiv:2106.06507), one event per
 * GPU lane, in two forms:
 *   - colour-ordered (COBG, Section 2.3 eq. cobg): partial amplitudes for the
 *     (n-2)! orderings A(1, sigma, n) of the adjoint decomposition (Section 2.2
 *     eq. color_decomposition_adjoint), then |M|^2 = A^dagger C A
 *     (eq. color_summed_analytic) with the colour matrix of
 *     eq. color_coefficient_adjoint;
 *   - colour-dressed (CDBG, Section 2.3 eq. color_dressed_currents) for one
 *     sampled colour-flow assignment per event (eq. color_decomposition_colorflow).
 * Beside these: the same flow amplitude as a sum over the colour-ordered
 * amplitudes whose colour chain closes (BG_MODE_COMC), the leading-colour sum
 * (BG_MODE_LC), the gradient of the colour-summed |M|^2 (bg_me2_grad), many
 * multiplicities in one launch (bg_me2_batch), continuous colour and real
 * polarization sampling (bg_me2_continuous), and phase space and sampled
 * quantum numbers drawn on the device (bg_generate, bg_generate_continuous).
 *
 * Conventions shared by every entry point
 *   - Pointers named mom/hel/col/amp/me2/grad are DEVICE pointers owned by the
 *     caller; the library never frees them and never retains them past the call.
 *   - mom   : double [n][4][E], E fastest.  All momenta outgoing (incoming beams
 *             negated), metric (+,-,-,-), any unit (GeV in the tests).
 *   - hel   : int8 [n][E], each +1 or -1 (all-outgoing helicity labels).  A gluon
 *             with label h and physical momentum k = sign(p^0) p uses the external
 *             current (eps^h(k))* with eps^+-(k) = (e1 +- i e2)/sqrt2 in the
 *             light-cone gauge with gauge vector (|k|, -k) (Section 2.1 eq.
 *             tensor_axial): e1 = (r|k|^2 - (r.k)k)/|..|, e2 = (k x e1)/|k|,
 *             e1^0 = e2^0 = 0, r = (3, -6, 2)/7.
 *   - col   : int8 [2][n][E]: col[0][k] = i_k, col[1][k] = j_k in {0,1,2}, the
 *             colour-flow pair of gluon k (3x3 unit matrix e_{j_k i_k}).
 *   - amp   : double [2][K][E] (real plane then imaginary plane), K = (n-2)!,
 *             sigma in lexicographic order of (sigma_2..sigma_{n-1}).
 *   - me2   : double [E].  No spin/colour averaging, no symmetry factor.
 *   - Couplings: g_s = sqrt(4 pi 0.118) (alpha_s of Section 5), SU(3), generators
 *     normalised as Tr(T^a T^b) = delta^ab.
 *   - stream: a hipStream_t passed as void*; NULL is the legacy default stream.
 *     Every call is stream-ordered and asynchronous: host-detectable errors are
 *     returned before anything is enqueued; device faults surface on a later
 *     synchronisation.
 *   - A context is bound to one device and is not thread-safe; use one per host
 *     thread.  It owns the colour matrices and a reusable workspace.  Calls on
 *     one context that use its workspace (bg_me2, bg_me2_grad, bg_me2_batch,
 *     bg_generate, bg_me2_continuous) are ordered even when they are issued on
 *     different streams: each such call records a context-owned event on its
 *     stream, and the next such call on another stream waits for it first.
 *     Work recorded into a graph is not ordered this way (the wait is skipped
 *     while a stream captures); the caller orders graph replays.
 */
#ifndef BG_H_
#define BG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BG_OK            0
#define BG_EINVAL       -1   /* null pointer, bad enum, n or E out of range */
#define BG_ERANGE       -2   /* size overflow or workspace too small */
#define BG_ENODEV       -3   /* no usable gfx950 device */
#define BG_EDEVICE      -4   /* a HIP runtime call failed */
#define BG_ENOMEM       -5   /* device allocation failed */
#define BG_EUNSUPPORTED -6   /* valid request the library does not implement */

/* evaluation mode */
#define BG_MODE_COBG 0       /* colour-ordered recursion + colour matrix (n <= 8) */
#define BG_MODE_CDBG 1       /* colour-dressed recursion, colours sampled (col required) */
#define BG_MODE_AUTO 2       /* COBG for n <= 7, CDBG for n >= 8 */
#define BG_MODE_LC   3       /* leading colour: N^(n-2)(N^2-1) sum over the (n-1)! orderings
                                (1, rho) of |A(1, rho)|^2 (Section 3.1, exact for n <= 5),
                                n <= 7, hel required; bg_me2 only */
#define BG_MODE_COMC 4       /* colour-sampled colour-ordered: the same |A|^2 as CDBG for the
                                given colour flow, as the sum of A(1, sigma) over the orderings
                                whose delta chain closes (Section 2.2); col and hel required;
                                bg_me2 only; synchronises the stream once per call (item count)
                                and the device when its item buffers grow; refused (BG_EINVAL)
                                while the stream is being captured; BG_ERANGE beyond 2^31
                                (event, ordering) items per call */

/* arithmetic of the recursion; contraction and |M|^2 sums are always FP64 */
#define BG_PREC_FP64       0
#define BG_PREC_FP32_MIXED 1 /* FP32 complex currents, FP64 invariants/contraction, and
                                FP64 re-evaluation of the events whose FP32 evaluation is
                                ill-conditioned (see bg_fp32_check_set) */

/* request and context flags */
#define BG_FLAG_VALIDATE       1u  /* check before any launch that every hel is +1 or -1 and
                                      every col entry is 0, 1 or 2 (BG_EINVAL otherwise);
                                      reads the inputs once and synchronises the stream;
                                      refused (BG_EINVAL) while the stream captures */
#define BG_FLAG_FP32_UNCHECKED 2u  /* BG_PREC_FP32_MIXED without the FP64 re-evaluation of
                                      ill-conditioned events (plain FP32 recursion) */

#define BG_N_MIN 4
#define BG_N_MAX 9

typedef struct bg_context bg_context;

/* Create a context on HIP device `device`.  Returns BG_ENODEV if the device is
 * missing or not gfx950, BG_EINVAL for unknown flags.  `flags` (BG_FLAG_*) are
 * applied to every request made through the context, in addition to the
 * request's own.  *out is set only on success. */
int bg_context_create(bg_context** out, int device, uint32_t flags);
void bg_context_destroy(bg_context* ctx);

/* Static message for a status code (never NULL). */
const char* bg_status_string(int status);

/* Number of colour-ordered amplitudes K = (n-2)! for n in [BG_N_MIN, BG_N_MAX], else 0. */
int64_t bg_num_orderings(int n);

/* Host function, no device needed.  Writes the colour matrix C(n) of
 * eq. color_coefficient_adjoint (Section 2.2), K x K row-major doubles, into
 * HOST memory `out` of capacity `cap` doubles.  Entries are exact integers
 * (N = 3).  n in [4, 8].  BG_ERANGE if cap < K*K. */
int bg_color_matrix(int n, double* out, int64_t cap);

/* Partial amplitudes A(1, sigma, n) for every sigma of the adjoint basis
 * (Section 2.3 eqs. cobg and cobg_full_amplitude; the printed p^2_{1,n} is read
 * as the inverse propagator of J(1..n-1), i.e. the top current is amputated).
 * One helicity configuration per event (hel required).  precision selects the
 * recursion arithmetic (BG_PREC_FP32_MIXED: plain FP32 recursion, no
 * accuracy check).  Output amp [2][K][E] as above.  n in [4, 8]
 * (BG_EUNSUPPORTED for n = 9). */
int bg_currents(bg_context* ctx, int n, int64_t n_events, const double* mom,
                const int8_t* hel, int precision, double* amp, void* stream);

/* me2[e] = sum_{s,t} C_st Re(A_s conj(A_t)) (eq. color_summed_analytic) for
 * amp [2][K][E] from bg_currents, in FP64 (matrix cores for K = 24 and 120).
 * For n = 8 (K = 720) C is held as its first row only, C_st = C_{0, r(s,t)}
 * with r(s,t) the ordering t after renaming gluons 2..n-1 so that s becomes
 * the identity (the colour factor is invariant under renaming summed colour
 * indices); the entries are rebuilt on the fly from K doubles, not the K^2 of
 * the full matrix.  n = 8 needs context workspace of 96 bytes per event
 * (allocated on first use of a size, with a device synchronisation).
 * If accumulate != 0 the result is added to me2 instead of stored.  n in [4, 8]. */
int bg_color_contract(bg_context* ctx, int n, int64_t n_events, const double* amp,
                      double* me2, int accumulate, void* stream);

typedef struct bg_request {
    int n;               /* gluons, BG_N_MIN..BG_N_MAX */
    int mode;            /* BG_MODE_* */
    int precision;       /* BG_PREC_* */
    uint32_t flags;      /* BG_FLAG_* (0 for none) */
    int64_t n_events;    /* E >= 0 (0 is a no-op) */
    const double* mom;   /* [n][4][E] */
    const int8_t* hel;   /* [n][E], or NULL = sum over all 2^n helicities (COBG only) */
    const int8_t* col;   /* [2][n][E] for CDBG, NULL for COBG */
    double* me2;         /* [E] out */
} bg_request;

/* |M|^2 per event.  COBG: colour-summed (eq. color_summed_analytic), for one
 * helicity per event or summed over helicities (hel NULL).  For n <= 6, and
 * for n = 7 in FP32, the recursion and the colour sum run in one kernel and
 * the partial amplitudes never reach device memory outside a small
 * per-block scratch (FP64 colour sum in VALU).  For n = 7 in FP64 and for
 * n = 8 (BG_PREC_FP64 only, BG_EUNSUPPORTED otherwise) it runs as
 * bg_currents followed by bg_color_contract (one straight path per ordering,
 * then the matrix-core colour sum) over chunks of 2^18 (n = 7, 0.5 GB of
 * context workspace) or 2^17 events (n = 8, 1.5 GB), once per helicity
 * configuration (accumulated) when hel is NULL; the FP32 check at n = 7
 * re-evaluates its listed events through the same two stages.  CDBG: |A|^2 of the
 * colour-flow amplitude of the given assignment (eq. color_decomposition_colorflow
 * via eq. color_dressed_currents); assignments without a closed colour chain
 * give exactly 0.  May allocate context workspace on first use of a size. */
int bg_me2(bg_context* ctx, const bg_request* req, void* stream);

/* bg_me2 for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * request, kernels and results (bit for bit) as bg_me2, but every piece of
 * device memory beyond the caller's inputs and outputs (check lists,
 * counters, colour-dressed event lists, per-block scratch and two-stage
 * amplitude chunks of the n = 7 paths, in chunks of at most 16,930 events)
 * comes from a file-scope device array of BG_NOALLOC_SCRATCH_BYTES
 * that each GPU holds until the process ends; its address is looked up once
 * per device when the first context on it is created, and the colour
 * matrices it needs are uploaded then.  The call itself calls no hipMalloc
 * or hipFree.  Modes: BG_MODE_COBG (n <= 7), BG_MODE_CDBG, BG_MODE_AUTO,
 * BG_MODE_LC (BG_MODE_COMC and COBG at n = 8 need growing buffers:
 * BG_EUNSUPPORTED).  At most
 * BG_NOALLOC_MAX_EVENTS events (BG_ERANGE beyond).  Every call on a GPU
 * shares that GPU's array, whatever its context: calls that overlap in time
 * on one GPU (other streams, other contexts, other host threads) race and
 * must be ordered by the caller.  Counters are cleared on the stream at the
 * start of each call. */
#define BG_NOALLOC_SCRATCH_BYTES (64u << 20)
#define BG_NOALLOC_MAX_EVENTS ((int64_t)1 << 22)
int bg_me2_noalloc(bg_context* ctx, const bg_request* req, void* stream);

/* FP32 accuracy control (BG_PREC_FP32_MIXED).  While the FP32 recursion runs
 * it also carries, per current, a bound on its components computed as if
 * every product were taken in modulus (the classical running error bound, up
 * to constant factors): 1 for an external polarization, and for a current of
 * a gluon range or subset |1/P^2| (E sum_splits S_1 S_2 + ...), E the sum of
 * |p^0| over the gluons, the remaining terms being the four-gluon vertex
 * (colour-ordered, Section 2.3 eq. cobg) or the tensor couplings
 * (colour-dressed, eq. color_dressed_currents) term by term.  An event whose
 *   est = sum_sigma S_sigma^2 / sum_sigma |A_sigma|^2   (colour-ordered, and
 *         leading colour over its (n-1)! orderings),
 *   est = S^2 / |A|^2                                    (colour-dressed), or
 *   est = (sum_sigma S_sigma)^2 / |A|^2                  (colour-sampled
 *         colour-ordered: A the sum of the closing orderings' amplitudes)
 * exceeds tau(mode, n) -- its amplitudes cancel strongly, so FP32 rounding of
 * the inputs and of the recursion is amplified -- is listed on the device and
 * evaluated again in FP64 by a second kernel on the same stream (no host
 * synchronisation), which overwrites its me2 (BG_MODE_COMC: the listed
 * event's orderings are evaluated again and summed again).  Helicity configurations whose
 * tree amplitude vanishes identically (fewer than two gluons of either
 * helicity) are never listed.  The default tau are chosen so that the
 * per-event relative error of me2 against FP64 stays below 1e-5 for 99% of
 * the sampled-helicity (and sampled-flow) events of the RAMBO workloads.
 * mode: BG_MODE_COBG or BG_MODE_LC (n in [4, 7]), BG_MODE_CDBG or
 * BG_MODE_COMC (n in [4, 9]), the bg_me2 modes the check applies to.  tau = 0 lists every
 * non-vanishing event (then me2 equals the FP64 path bit for bit); tau =
 * +inf lists none (as BG_FLAG_FP32_UNCHECKED).  Host only; BG_EINVAL for another mode or n, or
 * tau < 0 or NaN. */
int bg_fp32_check_set(bg_context* ctx, int mode, int n, float tau);
int bg_fp32_check_get(bg_context* ctx, int mode, int n, float* tau);

/* Gradient of the COBG colour-summed |M|^2 with respect to every momentum
 * component, contracted with an upstream gradient:
 *   grad_mom[i][mu][e] = grad_me2[e] * d me2[e] / d mom[i][mu][e]
 * (grad_me2 NULL means 1).  The differentiated function is the one bg_me2
 * computes, with the generic Minkowski P^2 and the polarization formulas above
 * applied off the mass shell.  Also writes me2 if req->me2 is non-NULL.
 * Requires mode COBG and hel non-NULL; n in [4, 7]. */
int bg_me2_grad(bg_context* ctx, const bg_request* req, const double* grad_me2,
                double* grad_mom, void* stream);

/* Several requests (mixed multiplicities, uneven event counts) in one
 * persistent kernel launch per pass, or (config split_kinds, the default) one
 * per segment kind, each with the LDS and register budget of its own kind:
 * the colour-ordered launch on `stream` and the colour-dressed one
 * concurrently on a side stream that the context owns, forked from and
 * joined back into `stream` through events; either way a fixed set of
 * launches that a graph recording `stream` captures.  Mode BG_MODE_AUTO picks COBG for n <= 7 and CDBG
 * for n >= 8 per segment; explicit modes are honoured (COBG needs n <= 7).
 * Every segment must have the same precision, hel non-NULL, me2 non-NULL when
 * its n_events > 0, and col for CDBG; at most BG_BATCH_MAX_SEGS segments.
 * Colour-ordered FP64 segments with n <= 6 give bg_me2's results on each
 * segment alone bit for bit (the same device routines evaluate every event;
 * only the scheduling differs).  Other segments agree within the two paths'
 * error bars: bg_me2 runs FP64 n = 7 in two stages (1/P^2 from prefix sums,
 * another colour-sum order), the FP32 kernels may contract products into multiply-adds
 * differently, a colour-dressed event is split over 256 lanes here and over
 * 64, 128 or 256 in bg_me2, and an FP32 event close to the check threshold of
 * bg_fp32_check_set may be re-evaluated in FP64 by one path only.
 * BG_PREC_FP32_MIXED batches apply that check per segment (threshold of the
 * segment's mode and n; BG_FLAG_FP32_UNCHECKED in a segment's flags turns it
 * off for that segment): an FP32 pass lists the events, a one-block kernel
 * turns the per-segment counts into a tile table on the device, and an FP64
 * pass of the same persistent kernel re-evaluates them (per kind when split);
 * every launch can be recorded into a graph.
 * The events are cut into tiles (config below), the tiles are ordered by
 * decreasing estimated cost and the blocks of the persistent grid take them
 * from an atomic queue.
 * The tile table depends only on the segments' (n, mode, n_events), the
 * precision and the config; it is built on the first call with that shape
 * (synchronous host-to-device upload) and cached in the context (at most
 * BG_BATCH_MAX_PLANS shapes; older ones are evicted after a device
 * synchronisation).  A call whose shape is cached allocates nothing, copies
 * nothing and only enqueues kernels on `stream`, so it may be recorded
 * into a HIP graph; such a graph remains valid while its shape stays cached
 * and the context lives.  Recording a call whose shape is not cached returns
 * BG_EINVAL.  Calls on one context must not overlap in time (they share the
 * context's scratch memory). */
#define BG_BATCH_MAX_SEGS 32
#define BG_BATCH_MAX_PLANS 64
int bg_me2_batch(bg_context* ctx, const bg_request* segs, int n_segs, void* stream);

/* Tile and grid shape of the batch kernel, per precision. */
typedef struct bg_batch_config {
    int blocks_per_cu;      /* persistent 256-lane blocks per compute unit; 0 = as many
                               as registers and LDS allow */
    int cobg_tile_events;   /* events per colour-ordered tile, multiple of 128, <= 8192 */
    int cdbg_tile_events;   /* events per colour-dressed tile, multiple of 32, <= 8192 (a tile
                               of ~5 % valid flows is evaluated event by event, so smaller
                               tiles shorten the queue's tail) */
    int waves_per_simd;     /* register budget of the kernel: 1 = all registers the
                               largest branch wants (one block per CU), 2 = at most 256
                               per lane (two blocks per CU, some spilling at n = 7) */
    int split_kinds;        /* 0 = one persistent launch over every tile; 1 = one over
                               the colour-ordered tiles (with waves_per_simd), then one
                               over the colour-dressed tiles, each sized by the LDS and
                               registers of its own kind (the dressed kernel always at
                               budget 2), so that a dressed segment does not run at the
                               occupancy the colour-ordered branches need */
} bg_batch_config;

/* Current batch config of `precision` (defaults: 0, 128, 256, 2, 1) into *out (host). */
int bg_batch_config_get(bg_context* ctx, int precision, bg_batch_config* out);
/* Set it; BG_EINVAL for values outside the ranges above. */
int bg_batch_config_set(bg_context* ctx, int precision, const bg_batch_config* cfg);

/* Autotuner: times bg_me2_batch on the given segments (their outputs are
 * written) for candidate configs -- split {1, 0} x register budget {2, 1} x
 * blocks per CU {max, 1}, then
 * colour-ordered tile {128, 256, 512, 1024}, then colour-dressed tile
 * {32, 64, 128, 256, 512}, each stage keeping the best -- with HIP events on
 * `stream`, and installs the fastest config for the segments' precision.
 * Synchronous; writes the chosen config and its time in milliseconds to
 * *best and *best_ms when non-NULL.  Must not be called during graph capture. */
int bg_me2_batch_tune(bg_context* ctx, const bg_request* segs, int n_segs,
                      bg_batch_config* best, double* best_ms, void* stream);

/* On-device phase-space points (Section 3: RAMBO, massless, all momenta
 * outgoing with the beams (sqrt_s/2)(1,0,0,+-1) negated as gluons 1 and 2;
 * Section 5: p_T > pt_min for each outgoing gluon and Delta R > dr_min for
 * each pair, pseudo-rapidity of massless momenta), with sampled helicities and
 * colour-flow pairs.  Randomness: keyed SplitMix64 (Steele, Lea, Flood 2014);
 * attempt t takes u_j = ((z >> 11) + 0.5) 2^-53 with
 * z = mix64(mix64(seed + G (t + 1)) + G (j + 1)), G = 0x9E3779B97F4A7C15,
 * j = 0 .. 4(n-2)-1 for RAMBO (cos theta = 2u-1, phi = 2 pi u,
 * E = -log(u u) per outgoing gluon, then the RAMBO boost and scaling), then
 * n draws for helicities (u < 1/2 -> +1, else -1), then 2n for the colour
 * pairs (i_k, j_k) = min(floor(3u), 2).  The same stream and laws as the
 * seeded host generator of the tests, so the two produce the same events.
 * Attempts first_attempt .. first_attempt + n_attempts - 1 are tried; the
 * accepted ones, in attempt order, are written at ranks 0 .. max_events - 1
 * of mom [n][4][max_events], hel [n][max_events] (flag BG_GEN_HEL),
 * col [2][n][max_events] (flag BG_GEN_COL) and attempt [max_events] (int64,
 * the attempt index of each event; may be NULL).  *n_generated (DEVICE
 * int64) receives min(accepted, max_events); slots beyond it are untouched.
 * Without BG_GEN_CUTS every attempt is accepted.  Asynchronous; uses a
 * context workspace of about n_attempts / 8 bytes (allocated on first use
 * of a size).  1 <= n_attempts <= 2^31, max_events >= 1. */
#define BG_GEN_CUTS 1
#define BG_GEN_HEL  2
#define BG_GEN_COL  4
typedef struct bg_gen_params {
    int n;                   /* gluons, BG_N_MIN..BG_N_MAX */
    int flags;               /* BG_GEN_* */
    double sqrt_s;           /* GeV, > 0 */
    double pt_min;           /* GeV */
    double dr_min;
    uint64_t seed;
    uint64_t first_attempt;
} bg_gen_params;
int bg_generate(bg_context* ctx, const bg_gen_params* params, int64_t n_attempts,
                int64_t max_events, double* mom, int8_t* hel, int8_t* col, int64_t* attempt,
                int64_t* n_generated, void* stream);

/* Continuous colour and polarization sampling with the colour-dressed
 * recursion, all arithmetic real (Section 2.1 eqs. polarization_kleiss,
 * polarization_simple, color_angles, gluon_color_polarization; Section 2.3
 * eq. color_dressed_currents).  Per event and gluon k:
 *   phi : double [n][E], the polarization angle; gluon k's polarization is
 *         e_k = e^{i phi} X^+ + e^{-i phi} X^- = sqrt2 (cos phi e1 + sin phi e2)
 *         with the helicity currents X^h and e1, e2 of `hel` above, so the
 *         average over phi of |A|^2 is the helicity sum;
 *   eta : double [2][n][3][E], eta[0][k] = eta(z_k), eta[1][k] = eta(zbar_k),
 *         the two colour vectors of eq. gluon_color_polarization (unit vectors
 *         for the sampling; any real vectors are accepted, the amplitude is
 *         linear in each).  Gluon k's colour matrix is eta(zbar_k) eta(z_k)^T
 *         (a colour-flow pair (i, j) is eta(z) = e_i, eta(zbar) = e_j).
 * me2[e] = A^2 of the (real) amplitude.  With phi uniform in [0, 2 pi) and the
 * eta vectors uniform on the unit sphere, 9^n E[me2] is the colour- and
 * helicity-summed |M|^2 (each sphere integral carries N_c).  n in [4, 9];
 * both precisions (FP32: currents in FP32, invariants 1/P^2 and the final
 * contraction in FP64).  The first FP64 call at n = 9 allocates a per-block
 * state buffer in the context (its state exceeds the LDS), synchronising the
 * device; later calls allocate nothing.  One event per
 * workgroup; every split of every subset costs a 3x3 colour-matrix product,
 * so this is compute-bound and far costlier per event than CDBG, but no
 * sampled event has a zero weight. */
int bg_me2_continuous(bg_context* ctx, int n, int precision, int64_t n_events, const double* mom,
                      const double* phi, const double* eta, double* me2, void* stream);

/* The continuous variables of bg_me2_continuous, drawn on the device from
 * the same keyed SplitMix64 stream as bg_generate: event e uses counter
 * first_event + e and, for gluon k, draws 5k .. 5k+4: phi = 2 pi u, then
 * (cos theta = 2u - 1, azimuth = 2 pi u) of eta(z_k) and of eta(zbar_k)
 * (uniform on the sphere, Section 2.1 eq. color_angles).  Writes phi [n][E]
 * and eta [2][n][3][E] (device pointers, caller-owned).  Stream-ordered,
 * allocates nothing. */
int bg_generate_continuous(bg_context* ctx, int n, uint64_t seed, uint64_t first_event,
                           int64_t n_events, double* phi, double* eta, void* stream);

/* Self-test of the matrix-core operand layout used by bg_color_contract:
 * runs one v_mfma_f64_16x16x4f64 with lane l supplying A[l%16][l/16] =
 * (l%16 + 1) + 100 (l/16) and B[l/16][l%16] = (l%16 + 1) 8^(l/16), and copies
 * the 64 lanes x 4 accumulator registers (out[4 l + r]) to HOST memory `out`
 * (256 doubles).  The caller decodes which (row, column) of D each element is.
 * Synchronous. */
int bg_mfma_layout_probe(bg_context* ctx, double* out);

#ifdef __cplusplus
}
#endif

#endif /* BG_H_ */
