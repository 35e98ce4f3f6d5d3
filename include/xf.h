/*
 * xf.h -- C ABI of the MI355X (gfx950) Born-rule probability library for
 * circuits made of passive (particle-number-conserving) matchgates and
 * controlled-phase gates, after "ExtraFerm: An Extended Matchgate Simulator"
 * (arXiv 2511.12416).
 *
 * What is computed (column convention, Sec. II-B Eq. 2-3 read together with the
 * composition of Sec. IV-B Eq. 14):
 *   A rotation layer U maps a_c^dag to sum_r U[r][c] a_r^dag.  The circuit is
 *   rotation 0, then the CPhase gates of layer 0, rotation 1, ..., rotation
 *   n_rot-1.  Replacing every CPhase(theta_j) by d_{x_j}(theta_j) (Sec. III-B,
 *   Eq. 7) gives the trajectory mode matrix
 *       V(x) = R_{L} D_{L-1}(x) R_{L-1} ... D_0(x) R_0,   L = n_rot - 1,
 *   with D_l(x) diagonal: mode q gets prod over the layer's gates j touching q
 *   of e^{i theta_j/2} (x_j = 0) or -e^{i theta_j/2} (x_j = 1).  For an output
 *   bitstring b with occupied modes R (ascending) and input occupation C:
 *       Exact (Sec. III-B Eq. 8-9, exponent of cos read as 1 - x_j):
 *           A_b = sum_x w(x) det V(x)[R, C],
 *           w(x) = prod_j cos(theta_j/4)^{1-x_j} (i sin(theta_j/4))^{x_j}
 *       Raw Estimate (Sec. III-A, trajectories drawn from Eq. 10-11):
 *           A_b = sqrt(xi*)/t * sum_{s<t} phase(x_s) det V(x_s)[R, C],
 *           phase(x) = prod_{j: x_j = 1} (i if theta_j >= 0 else -i)
 *       p_b = |A_b|^2.
 *   The global phase e^{-i theta_j/4} of every gate is dropped from A_b.
 *   Trajectories differing only where the same modes flip (same pattern N of
 *   Sec. IV-B Eq. 16-19) share one determinant, which is evaluated once.
 *
 * Trajectory sampler (both this library and any checker implement it from this
 * definition; it draws from the product distribution of Eq. 10-11):
 *   p_j = s_j / (s_j + c_j), s_j = sin(|theta_j|/4), c_j = cos(|theta_j|/4).
 *   Table T[a][j] (0 <= a <= j < k) = min(floor(2^32 * (1 - S)), 2^32 - 1) with
 *   S = prod_{i=a..j} (1 - p_i) accumulated left to right in IEEE FP64 without
 *   fused multiply-add.  Sample s of the bitstring with batch index i starts at
 *   a = 0 and draws u_0, u_1, ... from Philox4x32-10 (Salmon et al., SC'11)
 *   with key (lo32(seed), hi32(seed)): u_0 is word (s mod 4) of the block with
 *   counter (s div 4, 2^32 - 1, lo32(i), hi32(i)) (so one block gives the
 *   first draws of four consecutive samples), and u_d for d >= 1 is word
 *   ((d-1) mod 4) of the block with counter (s, (d-1) div 4, lo32(i),
 *   hi32(i)).  While a < k: draw the next u; the next gate with x_j = 1 is
 *   the smallest j >= a with u < T[a][j]; if there is none the sample ends,
 *   otherwise set x_j = 1 and continue at a = j + 1.
 *
 * Conventions for every call:
 *   - Complex numbers are interleaved (re, im) doubles; matrices row-major.
 *   - Pointers named d_* are device memory on the plan's device, h_* and
 *     unprefixed pointers are host memory.  The caller owns every buffer.
 *   - Asynchronous calls are ordered on the given hip_stream (a hipStream_t,
 *     NULL = default stream) and return before the kernels finish.
 *   - On any error the call returns a non-zero xf_status, writes nothing to
 *     its outputs, and xf_last_error() describes the problem.
 *   - A plan may be used from one host thread at a time; distinct plans are
 *     independent.  Calls on one plan share its device scratch (counters,
 *     workspace): issue them on one stream, or synchronise between calls on
 *     different streams.
 */
#ifndef XF_H
#define XF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XF_OK = 0,
    XF_EINVAL = 1,        /* invalid argument (null pointer, bad size, NaN, non-unitary layer, ...) */
    XF_EUNSUPPORTED = 2,  /* valid but outside what this library implements (sizes below)          */
    XF_ENOMEM = 3,        /* device or host allocation failed                                       */
    XF_EDEVICE = 4        /* a HIP runtime call failed                                              */
} xf_status;

typedef enum { XF_EXACT = 0, XF_RAW_ESTIMATE = 1 } xf_mode;

/* XF_FP64: every step in FP64.
 * XF_MIXED: the composition of Sec. IV-B Eq. 16-19 runs in FP32 where it is a
 * product: under the general determinant-lemma evaluation (see
 * xf_plan_set_evaluation) the products forming H from a well-conditioned
 * base run on the FP32 matrix cores (xf_plan_set_mixed_condition); where a
 * trajectory's submatrix is factorised directly, its low-rank correction is
 * formed in FP32.  The base inverse or elimination, the pivot products and
 * the cross-term accumulation stay FP64. */
typedef enum { XF_FP64 = 0, XF_MIXED = 1 } xf_precision;

/* 128-bit occupation / bitstring: bit p of (w[0] | w[1] << 64) <=> mode p occupied
 * (Jordan-Wigner: qubit p in |1> <=> fermion in mode p, Sec. II-B; bit-packed
 * 128-bit states as in Sec. IV-A). */
typedef struct { uint64_t w[2]; } xf_bits128;

/* A circuit in the layered form of Sec. IV-B (Eq. 14): passive matchgate
 * layers, each given by its n x n mode matrix (Sec. II-B Eq. 2-3; a layer
 * of matchgates G(A, B) multiplies out to one such unitary), with the
 * controlled-phase gates of Sec. III-B (Eq. 7) between consecutive layers. */
typedef struct {
    int32_t n;              /* modes = qubits, 1 <= n <= 128                                   */
    int32_t n_rot;          /* rotation layers in time order, 1 <= n_rot <= 65 (more than 3
                               needs k <= 63)                                                   */
    const double *rot;      /* host [n_rot][n][n][2]: unitary mode matrices (column convention) */
    int32_t k;              /* CPhase gates (k = 0 requires nothing else)                      */
    const int32_t *pairs;   /* host [k][2]: the two modes of gate j, distinct, in [0, n)        */
    const int32_t *layer;   /* host [k]: gate j acts after rotation layer[j], 0 <= layer[j] < n_rot-1 */
    const double *theta;    /* host [k]: angles, finite, |theta| < 2*pi                        */
} xf_circuit;

typedef struct xf_plan xf_plan;

/* One gate of a circuit given gate by gate (Sec. II-B): a nearest-neighbour
 * particle-number-conserving matchgate G(A, B) (Eq. 1 with A diagonal, so
 * that |00> and |11> keep their weight, det A = det B, unitary) on qubits
 * (q0, q1 = q0 + 1), or a controlled-phase gate diag(1, 1, 1, e^{i theta}) on
 * two distinct qubits (Sec. III-B). */
typedef enum { XF_GATE_MATCHGATE = 0, XF_GATE_CPHASE = 1 } xf_gate_kind;
typedef struct {
    int32_t kind;       /* xf_gate_kind */
    int32_t q0, q1;     /* the qubits (= modes) the gate acts on */
    double theta;       /* CPhase angle, finite, |theta| < 2 pi (ignored for a matchgate) */
    double g[16][2];    /* matchgate: the 4 x 4 unitary, row-major, basis |x_q0 x_q1> = 00, 01, 10, 11
                           (ignored for a CPhase gate) */
} xf_gate;

/* Matchgate ingestion: the layered circuit (xf_circuit) of a gate list in
 * time order.  Consecutive matchgates multiply into one rotation layer (their
 * mode matrices, Sec. II-B Eq. 2: the single-particle block of G scaled by
 * the vacuum phase G[00][00], which is a global phase and dropped; later
 * gates multiply on the left); consecutive CPhase gates form one CPhase layer
 * between two rotation layers.  The first and last layers may be the
 * identity.  With rot == NULL only *n_rot and *k are written (the sizes to
 * allocate); otherwise rot host [max_rot][n][n][2], pairs [max_k][2],
 * layer [max_k], theta [max_k] receive the circuit (XF_EINVAL if it needs
 * more than max_rot layers or max_k gates).  2 <= n <= 128.  Errors:
 * XF_EINVAL (a gate that is not of the forms above, within 1e-12 on the zero
 * entries and 1e-10 on unitarity and det A = det B). */
xf_status xf_circuit_from_gates(int32_t n, int32_t n_gates, const xf_gate *gates, int32_t max_rot, int32_t max_k,
                                double *rot, int32_t *pairs, int32_t *layer, double *theta, int32_t *n_rot,
                                int32_t *k);

/* Creates a plan on HIP device `device` for circuit `c` and input occupation
 * `input` (eta = popcount <= 64, all bits below n; the input Slater
 * determinant of Sec. II-B).  Precomputes what every probability call
 * shares: the layer products and low-rank factors of Sec. IV-B Eq. 14-19,
 * the extent of Sec. III-A Eq. 5 and the trajectory-sampling table of
 * Eq. 10-11 (see the sampler definition above).  Copies what it needs
 * from the host arrays; they may be freed afterwards.  Validates unitarity of
 * every layer (max |U^H U - I| <= 1e-10).  The trajectory-sampling table is
 * frozen at the angles given here (see xf_plan_refreeze).
 * Errors: XF_EINVAL, XF_EUNSUPPORTED (n > 128, eta > 64, n_rot > 65, or
 * n_rot > 3 with k > 63), XF_ENOMEM, XF_EDEVICE. */
xf_status xf_plan_create(const xf_circuit *c, xf_bits128 input, xf_precision precision,
                         int device, xf_plan **plan);

/* Replaces rotation entries and angles (same shapes as at creation; either
 * pointer may be NULL to keep the current values), recomputing the factors
 * of Sec. IV-B Eq. 14-19 and the extent of Sec. III-A Eq. 5.  The sampling table stays
 * frozen, so Raw Estimate draws the same trajectories: this is the estimator
 * whose derivative xf_log_prob_backward returns.  Synchronous. */
xf_status xf_plan_set_params(xf_plan *plan, const double *rot, const double *theta);

/* Rebuilds the sampling table (Sec. III-A Eq. 10-11) from the current
 * angles.  Synchronous. */
xf_status xf_plan_refreeze(xf_plan *plan);

/* Frees the plan and its device memory (synchronises the plan's device).
 * NULL is accepted and ignored. */
xf_status xf_plan_destroy(xf_plan *plan);

/* Extent of the current angles, Sec. III-A Eq. 5:
 * xi* = prod_j (cos(|theta_j|/4) + sin(|theta_j|/4))^2. */
xf_status xf_extent(const xf_plan *plan, double *xi);

/* Trajectory count of Sec. III-A Eq. 6 (natural logarithm):
 * t = ceil(2 (sqrt(xi) + sqrt(p_max))^2 / (sqrt(p_max + eps) - sqrt(p_max))^2
 *          * log(2 e^2 / delta)).
 * Requires eps > 0, 0 < delta < 1, 0 <= p_max <= 1, xi >= 1; XF_EUNSUPPORTED
 * if t exceeds 2^62. */
xf_status xf_trajectory_bound(double eps, double delta, double p_max, double xi, int64_t *t);

/* Born-rule probabilities of B output bitstrings (Sec. III-A/B).
 *   d_bits  device [B] xf_bits128 (batch index i of d_bits[i] keys the sampler)
 *   mode    XF_EXACT (all 2^k trajectories; k <= 24) or XF_RAW_ESTIMATE
 *           (1 <= t < 2^31 samples per bitstring, k <= 128, and either the
 *           modes touched by the gates of each CPhase layer, summed over
 *           layers, number at most 63, or k <= 63: a trajectory's key must fit
 *           in 63 bits; XF_EUNSUPPORTED otherwise)
 *   seed    sampler key (ignored in exact mode)
 *   d_prob  device [B] doubles: p_b
 *   d_amp   device [B][2] doubles: A_b, or NULL
 *   d_logp  device [B] doubles: log p_b in FP64 (-inf where p_b = 0), or NULL
 * A bitstring whose weight differs from eta, or with bits at or above n, gets
 * p = 0 and A = 0 (passive circuits conserve the weight, Sec. II-B).  B = 0 is
 * a no-op.  Uses plan-owned device scratch (under the determinant lemma, a
 * workspace holding each bitstring's distinct patterns, see
 * xf_plan_set_workspace_limit, grown on demand, the call then synchronising
 * hip_stream first); results are bitwise reproducible for fixed inputs. */
xf_status xf_probabilities(xf_plan *plan, const xf_bits128 *d_bits, int64_t B, xf_mode mode,
                           int64_t t, uint64_t seed, double *d_prob, double *d_amp,
                           double *d_logp, void *hip_stream);

/* No-allocation variant of xf_probabilities, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, results (bitwise) and errors as
 * xf_probabilities, except:
 *   - the determinant-lemma workspace is a fixed device array of 256 MiB per
 *     device, held until the process ends; bitstrings are processed in chunks
 *     of floor((2^28 - 256) / (16 c + 4 + h)), c = min(t + t/511 + 2, 8192)
 *     entries and h the general lemma's per-bitstring setup bytes (16 per
 *     complex entry of H plus a 48-byte record; 0 for the eta <= 16
 *     one-layer kernels); exact mode under the general lemma holds
 *     4 B + h (+ the segments' 64-byte partial sums) per bitstring of the
 *     whole batch and returns XF_EUNSUPPORTED if they do not fit;
 *   - no device memory, pinned host memory or event is allocated and no
 *     kernel time is recorded (xf_plan_last_work reports zero times); the
 *     first call on a device looks up the array's device address;
 *   - exact mode needs the term list that an earlier xf_probabilities call on
 *     the plan built for the current parameters (XF_EUNSUPPORTED otherwise).
 * All calls on one device share its array and leave their contents in it (no
 * part of it needs to start at zero): calls that overlap in time on one
 * device, from different streams, plans or host threads, race and give wrong
 * results; serialise them. */
xf_status xf_probabilities_noalloc(xf_plan *plan, const xf_bits128 *d_bits, int64_t B, xf_mode mode,
                                   int64_t t, uint64_t seed, double *d_prob, double *d_amp,
                                   double *d_logp, void *hip_stream);

/* Estimate (Sec. III-A): Raw Estimate probabilities to additive error eps
 * with failure probability at most delta per bitstring, without a bound
 * p_max on the probability.  The paper names the algorithm (start from loose
 * error and probability bounds, then call Raw Estimate repeatedly, after
 * Pashayan et al.) without giving its schedule; this library's is:
 *   p_max_b = 1 for every bitstring; for i = 1, 2, ...:
 *     eps_i = max(eps, 2^-i), delta_i = delta 2^-i;
 *     t_b = Eq. 6 at (eps_i, delta_i, p_max_b, xi*) (xf_trajectory_bound),
 *       rounded up to at most four significant bits (the smallest m 2^e >= t_b
 *       with m < 16);
 *     the bitstrings are ordered by t_b (ties by batch index) and each run of
 *       equal t_b is one Raw Estimate call (xf_probabilities) with t_b
 *       samples and seed (seed + i - 1) mod 2^64, a bitstring's samples keyed
 *       by its position in the run;
 *     if eps_i = eps these estimates are the result; otherwise
 *       p_max_b = min(p_max_b, 1, p_hat_b + eps_i).
 *   Each later bound holds when the earlier estimates were within their
 *   eps_i, and sum_i delta_i < delta.
 *   d_bits  device [B] xf_bits128;  d_prob  device [B] doubles (p_hat_b)
 *   h_t     host [B] int64: the last iteration's t_b, or NULL
 *   h_iterations  host int32: the number of iterations, or NULL
 * Requires 0 < eps < 1, 0 < delta < 1 (XF_EINVAL); XF_EUNSUPPORTED if some
 * t_b reaches 2^31 or Raw Estimate is unsupported for the plan.  Allocates
 * device memory for the grouped batch and synchronises hip_stream. */
xf_status xf_estimate(xf_plan *plan, const xf_bits128 *d_bits, int64_t B, double eps, double delta,
                      uint64_t seed, double *d_prob, int64_t *h_t, int32_t *h_iterations, void *hip_stream);

/* Weak simulation (Sec. II-A): S output samples of a circuit given gate by
 * gate, by the gate-by-gate algorithm (Bravyi, Gosset and Liu, 2022), which
 * needs only probabilities of chosen bitstrings.  Every chain starts at the
 * input; a CPhase gate (diagonal) leaves the distribution unchanged; at a
 * matchgate gi on (q, q + 1), a chain whose pair holds one particle (the
 * other assignments are fixed by particle-number conservation) moves to the
 * candidate c10 (mode q occupied) or c01 (mode q + 1 occupied), with
 * probabilities p10, p01 of the circuit of gates 0..gi (xf_probabilities in
 * `mode` with t samples and seed (seed + gi) mod 2^64, the candidates of the
 * chains that move ordered by chain, c10 before c01): c10 if
 * u (p10 + p01) < p10 in FP64, u = w 2^-32 with w word 0 of Philox4x32-10 at
 * counter (lo32(s), gi, 2^32 - 2, hi32(s)) and key (lo32(seed), hi32(seed)),
 * s the chain; a chain with p10 + p01 = 0 stays.  With exact probabilities the
 * samples follow the output distribution exactly; with Raw Estimate,
 * approximately.  Same gate rules as xf_circuit_from_gates; input as for
 * xf_plan_create; h_samples host [S].  Creates a plan on `device` per run of
 * matchgates between CPhase gates, allocates device memory for 2S
 * candidates, and synchronises hip_stream.  Errors: those of
 * xf_circuit_from_gates, xf_plan_create and xf_probabilities. */
xf_status xf_sample_gates(int32_t n, int32_t n_gates, const xf_gate *gates, xf_bits128 input, int64_t S,
                          xf_mode mode, int64_t t, uint64_t seed, xf_precision precision, int device,
                          xf_bits128 *h_samples, void *hip_stream);

/* Gradient of L = sum_b g_b log p_b, g = d_grad_logp (device [B] doubles),
 * with respect to every rotation entry (h_grad_rot, host [n_rot][n][n][2],
 * as dL/dRe + i dL/dIm) and every angle (h_grad_theta, host [k]).  Same
 * bitstrings, mode, t and seed as the forward call it differentiates; Raw
 * Estimate samples are held fixed (frozen table), the weights depend on the
 * angles through sqrt(xi*).  Uses Jacobi's formula d det M = det M tr(M^-1 dM)
 * and recomputes every trajectory's submatrix instead of storing it.
 * Bitstrings with p_b = 0 contribute nothing.  Synchronises hip_stream. */
xf_status xf_log_prob_backward(xf_plan *plan, const xf_bits128 *d_bits, int64_t B, xf_mode mode,
                               int64_t t, uint64_t seed, const double *d_grad_logp,
                               double *h_grad_rot, double *h_grad_theta, void *hip_stream);

/* How the determinant of each distinct flip pattern N of a bitstring is
 * evaluated (Raw Estimate and exact mode; Sec. IV-B Eq. 16-19).
 *   XF_EVAL_LU: LU factorisation with partial pivoting of the eta x eta
 *     submatrix M_N = M_0 - 2 A[R, N] Phi[N, :] (the two-layer form for two
 *     CPhase layers, the full product for three).
 *   XF_EVAL_AUTO (default): the matrix determinant lemma
 *     det M_N = det M_B det(I_r - 2 diag(sigma) H[D, D]),
 *     H = V M_B^-1 U formed once per bitstring from a base M_B (the empty
 *     pattern, or for one CPhase layer the flips of one gate when the empty
 *     pattern's base is singular or ill-conditioned; D = N xor base pattern,
 *     sigma = -1 where the base flips and N does not), so that each pattern
 *     costs an r x r determinant (r = |D|; one lane for r <= 4, lane groups
 *     of 8 to 32 above).  Applies to one or two CPhase layers with
 *     n_rot = L + 1.  When every rotation layer is block-diagonal over a
 *     partition of the modes into at most two blocks (spin-restricted layers
 *     U (+) U), V(x) is block-diagonal for every trajectory and the
 *     determinant is the product of the blocks' (one base per block, each of
 *     at most 32 rows and 64 active modes).  A bitstring whose bases are all
 *     singular or have 1-norm condition number above 1e4, with a pattern
 *     beyond the largest lane group, or whose patterns overflow its workspace
 *     region, is evaluated with the LU of every M_N instead.  The gradient
 *     (xf_log_prob_backward) uses the lemma for one CPhase layer and
 *     eta <= 16 under Raw Estimate, the LU elsewhere.
 * Exact mode under XF_EVAL_AUTO: the patterns' determinants det S are
 * principal minors of one matrix per bitstring (I - 2H for one CPhase layer,
 * I + 2T - 2H with T = R'_1 between the layers' positions for two, I + 2TT -
 * 2K for more), so terms whose flipped
 * positions share a prefix share its elimination.  The plan arranges the
 * term list as a prefix tree over those positions (at most 32 in all; anchors
 * every four positions, each a Schur complement of its parent's), and waves
 * walk it, each bitstring's walk split into parts (runs of the depth-first
 * order, about 16K waves per call, at most one per 256 terms) whose exact
 * partial sums are added: each term then costs a determinant of at most
 * 4 x 4 (all principal minors by the recursion of Griffin and Tsatsomeros,
 * Linear Algebra Appl. 419 (2006)).  Bitstrings with a shifted base, an
 * exactly singular pivot block, or entries grown beyond 10^4 times G's
 * largest take the per-pattern evaluation instead.
 *   XF_EVAL_PATTERNS: XF_EVAL_AUTO without the prefix tree (every pattern's
 *     r x r determinant on its own). */
typedef enum { XF_EVAL_AUTO = 0, XF_EVAL_LU = 1, XF_EVAL_PATTERNS = 2 } xf_evaluation;
xf_status xf_plan_set_evaluation(xf_plan *plan, xf_evaluation evaluation);

/* XF_MIXED under the general determinant-lemma evaluation (see
 * xf_plan_set_evaluation): the products forming H from a bitstring's base
 * (X = M_B^-1 U, H = V X, the composition of Sec. IV-B Eq. 16-19 moved onto
 * the base) run on the FP32 matrix cores for bases with 1-norm condition
 * number at most kappa_max, and in FP64 otherwise; the base inverse, the
 * per-pattern determinants and the accumulation stay FP64.  The FP32 error of
 * H grows with ||M_B^-1||, so kappa_max trades speed for accuracy (default
 * 100; 0 gives FP64 results).  kappa_max >= 0, else XF_EINVAL. */
xf_status xf_plan_set_mixed_condition(xf_plan *plan, double kappa_max);

/* Exact mode along the prefix tree (see xf_plan_set_evaluation): the largest
 * growth accepted, as max |entry| of the Schur complements over max |G| and
 * as the largest |multiplier| of the 4 x 4 block eliminations (default 1e4;
 * growth > 0, else XF_EINVAL).  A bitstring beyond it takes the per-pattern
 * evaluation.  Takes effect at the next xf_probabilities call. */
xf_status xf_plan_set_tree_growth(xf_plan *plan, double growth);

/* Device memory the determinant-lemma path may use for its workspace
 * (default 16 GiB; bytes > 0).  Each bitstring's region holds
 * min(t + t/511 + 2, 8192) distinct patterns, 16 bytes each, plus 4 bytes; a
 * bitstring with more distinct patterns is evaluated by the LU path.  The
 * batch is processed in chunks of as many bitstrings as fit, at least one.
 * Results do not depend on the chunking.  Takes effect at the next
 * xf_probabilities call; a workspace already allocated is kept while large
 * enough. */
xf_status xf_plan_set_workspace_limit(xf_plan *plan, uint64_t bytes);

/* Backward without resampling (default off).  When on, an
 * xf_log_prob_backward call in Raw Estimate mode whose d_bits, B, t and seed
 * equal those of the plan's last xf_probabilities call takes that call's
 * distinct flip patterns and counts (the determinant table of Sec. IV-B,
 * drawn per Sec. III-B Eq. 10-12) from the plan's workspace instead of
 * drawing them again; the gradient is the same.  This applies only when both
 * calls use the one-layer determinant-lemma kernels (eta <= 16) and the
 * forward call processed the batch in one chunk (see
 * xf_plan_set_workspace_limit); otherwise the backward draws the samples
 * itself.  Any other xf_probabilities or xf_estimate call on the plan, and
 * any parameter or setting change, ends the reuse until the next forward
 * call.  The caller guarantees that the bitstrings at d_bits are unchanged
 * between the two calls and that the backward is ordered after the forward
 * (the same stream, or an event).  on is 0 or 1, else XF_EINVAL. */
xf_status xf_plan_set_reuse_samples(xf_plan *plan, int32_t on);

/* Work done by the last xf_probabilities call on this plan (synchronises the
 * device): *count = distinct (bitstring, flip-pattern) determinants
 * evaluated; *rank_sum (nullable) = the sum over them of the number of
 * flipped modes, i.e. of the ranks of the low-rank corrections composed. */
xf_status xf_plan_last_term_count(xf_plan *plan, int64_t *count, int64_t *rank_sum);

/* Same counters plus the arithmetic executed for them and the kernel times
 * of the call (synchronises the device).  flops counts real FP64-equivalent
 * operations of the determinant evaluations actually performed:
 * (4/3)(m-1)m(2m-1) + 3m(m-1) per m x m LU plus 8 m^2 per rank of each
 * composed correction, or, for a pattern taken by the determinant lemma, the
 * same LU count at size r plus 6, plus the lemma's per-bitstring setup
 * (Gauss-Jordan inverse of M_0 and the products forming H, 8 per complex
 * multiply-add).  The sampling is not counted.  lemma = 1 if the call used
 * the determinant lemma; it then runs a sampling kernel and an evaluation
 * kernel per chunk of bitstrings, timed separately (sample_ms, eval_ms, from
 * HIP events on the call's stream); other calls run one kernel, reported in
 * eval_ms. */
typedef struct {
    int64_t determinants;
    int64_t rank_sum;
    double flops;
    double sample_ms;
    double eval_ms;
    int32_t lemma;
    int32_t backward_lemma;   /* the last xf_log_prob_backward call used the determinant lemma */
    int32_t general;          /* the call used the general determinant-lemma kernel (see below) */
    int32_t backward_reused;  /* the last xf_log_prob_backward call took the forward call's sampled
                                 patterns (see xf_plan_set_reuse_samples) */
    int64_t fp32_bases;       /* bases (per block) whose lemma products ran in FP32 (XF_MIXED) */
    int64_t philox_blocks;    /* Raw Estimate under the lemma: Philox4x32-10 blocks the sampling
                                 definition draws (one per four samples' first draws, one per four
                                 further draws of a sample); 100 32-bit integer operations each */
    int64_t tree_bitstrings;  /* exact mode: bitstrings evaluated along the prefix tree (see
                                 xf_plan_set_evaluation) */
} xf_work;
xf_status xf_plan_last_work(xf_plan *plan, xf_work *work);

/* Host FP64 helpers for rotations parametrised by anti-Hermitian generators
 * (U = exp(K), the unitary mode matrix of Sec. II-B Eq. 2-3 written through
 * its generator; used by the differentiation interface), n <= 128:
 *   xf_expm_antihermitian: U = exp(K), K and U host [n][n][2].
 *   xf_expm_adjoint: G_K = L(K^H, G_U), the adjoint of the Frechet derivative
 *     of exp at K applied to G_U; with G_U = dL/dRe U + i dL/dIm U it returns
 *     dL/dRe K + i dL/dIm K. */
xf_status xf_expm_antihermitian(int32_t n, const double *K, double *U);
xf_status xf_expm_adjoint(int32_t n, const double *K, const double *G_U, double *G_K);

/* Spin-restricted rotation layers (the same orbital rotation on both spin
 * sectors, modes 0..d-1 and d..2d-1; the LUCJ orbital rotations of Sec. IV-B), host
 * FP64, 1 <= d <= 64:
 *   xf_spin_rotations: rot[l] = exp(K_l) (+) exp(K_l), K host
 *     [n_layers][d][d][2] anti-Hermitian, rot host [n_layers][2d][2d][2]
 *     (every entry written).
 *   xf_spin_rotations_adjoint: G_K[l] = L(K_l^H, G_rot[l][:d, :d] +
 *     G_rot[l][d:, d:]) (the two blocks' gradients add), G_rot in the layout
 *     of xf_log_prob_backward's h_grad_rot, G_K [n_layers][d][d][2].
 * Errors: XF_EINVAL (sizes, NULL, NaN/Inf, K not anti-Hermitian). */
xf_status xf_spin_rotations(int32_t n_layers, int32_t d, const double *K, double *rot);
xf_status xf_spin_rotations_adjoint(int32_t n_layers, int32_t d, const double *K, const double *G_rot,
                                    double *G_K);

/* Gradient with respect to the d^2 real parameters of an anti-Hermitian
 * generator K -- (Re K_ij) for i < j in row-major order, then (Im K_ij) for
 * i < j, then Im K_ii -- from G_K = dL/dRe K + i dL/dIm K of the full
 * matrix (K_ji = -conj(K_ij)).  G_K host [d][d][2], g host [d^2],
 * 1 <= d <= 128.  Errors: XF_EINVAL. */
xf_status xf_antihermitian_reals_grad(int32_t d, const double *G_K, double *g);

/* Message for the last error on the calling thread ("" if none). */
const char *xf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XF_H */
