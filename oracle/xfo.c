/*
 * xfo.c -- plain FP64 CPU oracle for Born-rule probabilities of circuits made
 * of passive (particle-number-conserving) matchgates and controlled-phase
 * gates, following "ExtraFerm: An Extended Matchgate Simulator"
 * (arXiv 2511.12416).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library and is deliberately slow and plain: every trajectory's
 * mode matrix is built as an explicit matrix product, every determinant by a
 * textbook partial-pivot LU, and every sum in the order the definition gives.
 *
 * Conventions
 *   rot     [n_rot][n][n] complex, row-major, rotation layer 0 acts first.
 *           Column convention (Sec. II-B, Eq. 2-3 read with the composition of
 *           Eq. 14): a layer U maps a_c^dag to sum_r U[r][c] a_r^dag, so the
 *           amplitude <b|M|a> is det(V[R, C]), R = occupied modes of b, C of a.
 *   gates   gate j acts on modes (pairs[2j], pairs[2j+1]) after rotation layer
 *           layer[j] and before layer[j]+1.
 *   bits    [B][2] uint64 (low word, high word); bit p <=> mode p occupied.
 *
 * Readings of the paper (all also listed in the design notes):
 *   - Eq. 9 prints the exponent of cos as (x_j - 1); the decomposition of Eq. 7
 *     fixes it as (1 - x_j).
 *   - d_0 and d_1 of Eq. 7 are, up to the global phase e^{-i theta/2}, passive
 *     gates multiplying modes q1 and q2 by e^{i theta/2} (d_0) or by
 *     -e^{i theta/2} (d_1).  All global phases (e^{-i theta/4} per gate) are
 *     dropped: they do not change |A|^2.
 *   - Raw Estimate (Sec. III-A, Eq. 10-11) samples x from P(x) = prod_j p(x_j)
 *     and averages sqrt(xi*) * phase(x) * <b|V(x)|a>, with
 *     phase(x) = prod_{j: x_j = 1} i*sign(theta_j); p_hat = |A_hat|^2.
 *   - Trajectory sampling uses the inverse-transform sampler of
 *     "next d_1 gate" positions described at xfo_sampler_table(), driven by
 *     Philox4x32-10; it draws from the same product distribution as Eq. 12.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box with a      */
/* Weyl-sequence key schedule.                                                */
/* ------------------------------------------------------------------------ */
void xfo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The d-th uniform 32-bit draw u_d of sample s of bitstring index bidx,
 * Philox4x32-10 with key (seed_lo, seed_hi): u_0 is word (s mod 4) of the
 * block with counter (s div 4, 2^32 - 1, bidx_lo, bidx_hi); u_d for d >= 1
 * is word ((d-1) mod 4) of the block with counter (s, (d-1) div 4, bidx_lo,
 * bidx_hi). */
static uint32_t draw_u32(uint64_t seed, uint64_t bidx, uint32_t s, uint32_t d)
{
    uint32_t ctr[4] = { d == 0 ? s >> 2 : s, d == 0 ? 0xFFFFFFFFu : (d - 1) >> 2,
                        (uint32_t)bidx, (uint32_t)(bidx >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    xfo_philox4x32_10(ctr, key, out);
    return out[d == 0 ? (s & 3) : ((d - 1) & 3)];
}

/* ------------------------------------------------------------------------ */
/* Sampling distribution, Sec. III-B Eq. 10-11                               */
/* ------------------------------------------------------------------------ */

/* p(x_j = 1) = sin(|theta|/4) / (sin(|theta|/4) + cos(|theta|/4)). */
static double p_one(double theta)
{
    double s = sin(fabs(theta) / 4.0);
    double c = cos(fabs(theta) / 4.0);
    return s / (s + c);
}

/*
 * Inverse-transform table for the position of the next x_j = 1.
 *
 * Under P(x) = prod_j p_j^{x_j} (1-p_j)^{1-x_j} the gates are independent, so
 * starting at gate a the probability that the first x_j = 1 lies at or before
 * gate j is F(a, j) = 1 - prod_{i=a..j} (1 - p_i).  One uniform draw u then
 * gives the next selected gate as the smallest j >= a with u < F(a, j) (none:
 * the trajectory has no further x_j = 1); sampling resumes at j + 1.  In
 * 32-bit integers: T[a*k + j] = min(floor(2^32 * F(a, j)), 2^32 - 1), with the
 * product accumulated left to right in FP64, and the test is u < T.
 */
void xfo_sampler_table(int k, const double *theta, uint32_t *T)
{
    for (int a = 0; a < k; ++a) {
        double surv = 1.0;
        for (int j = 0; j < k; ++j) {
            if (j < a) { T[a * k + j] = 0; continue; }
            surv = surv * (1.0 - p_one(theta[j]));
            double f = 1.0 - surv;
            double v = floor(f * 4294967296.0);
            T[a * k + j] = (v >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)v;
        }
    }
}

/* Draws trajectory x (bit j <=> x_j = 1) for sample s of bitstring index bidx. */
static void sample_trajectory(int k, const uint32_t *T, uint64_t seed, uint64_t bidx,
                              uint32_t s, uint64_t x[2])
{
    x[0] = x[1] = 0;
    int a = 0;
    uint32_t d = 0;
    while (a < k) {
        uint32_t u = draw_u32(seed, bidx, s, d);
        d++;
        int j = a;
        while (j < k && !(u < T[a * k + j])) j++;
        if (j == k) break;
        x[j >> 6] |= (uint64_t)1 << (j & 63);
        a = j + 1;
    }
}

void xfo_sample_trajectories(int k, const double *theta, uint64_t seed, uint64_t bidx,
                             int64_t t, uint64_t *x_out /* [t][2] */)
{
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(k > 0 ? k * k : 1));
    xfo_sampler_table(k, theta, T);
    for (int64_t s = 0; s < t; ++s)
        sample_trajectory(k, T, seed, bidx, (uint32_t)s, x_out + 2 * s);
    free(T);
}

/* ------------------------------------------------------------------------ */
/* Dense complex helpers                                                     */
/* ------------------------------------------------------------------------ */

static int bit_of(const uint64_t b[2], int p) { return (int)((b[p >> 6] >> (p & 63)) & 1u); }

static int occupied(const uint64_t b[2], int n, int *idx)
{
    int m = 0;
    for (int p = 0; p < n; ++p)
        if (bit_of(b, p)) idx[m++] = p;
    return m;
}

/* LU with partial pivoting of the m x m row-major matrix a (overwritten):
 * the pivot of column c is the row (among rows c..m-1) with the largest
 * re^2 + im^2, the lowest row index on ties.  perm[r] records the original
 * row now in position r.  Returns det(a); a zero pivot gives det = 0 and
 * *singular = 1. */
static cplx lu_factor(cplx *a, int m, int *perm, int *singular)
{
    cplx det = 1.0;
    *singular = 0;
    for (int r = 0; r < m; ++r) perm[r] = r;
    for (int c = 0; c < m; ++c) {
        int p = c;
        double best = creal(a[c * m + c]) * creal(a[c * m + c]) + cimag(a[c * m + c]) * cimag(a[c * m + c]);
        for (int r = c + 1; r < m; ++r) {
            double v = creal(a[r * m + c]) * creal(a[r * m + c]) + cimag(a[r * m + c]) * cimag(a[r * m + c]);
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) { *singular = 1; return 0.0; }
        if (p != c) {
            for (int j = 0; j < m; ++j) {
                cplx tmp = a[c * m + j]; a[c * m + j] = a[p * m + j]; a[p * m + j] = tmp;
            }
            int tp = perm[c]; perm[c] = perm[p]; perm[p] = tp;
            det = -det;
        }
        cplx piv = a[c * m + c];
        det *= piv;
        for (int r = c + 1; r < m; ++r) {
            cplx l = a[r * m + c] / piv;
            a[r * m + c] = l;
            for (int j = c + 1; j < m; ++j) a[r * m + j] -= l * a[c * m + j];
        }
    }
    return det;
}

void xfo_det(int m, const double *a_in /* [m][m][2] */, double *det_out /* [2] */)
{
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)(m > 0 ? m * m : 1));
    int *perm = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m * m; ++i) a[i] = a_in[2 * i] + I * a_in[2 * i + 1];
    int sing;
    cplx d = (m == 0) ? 1.0 : lu_factor(a, m, perm, &sing);
    det_out[0] = creal(d); det_out[1] = cimag(d);
    free(a); free(perm);
}

/* Inverse from the LU factors: solves (P a) X = P I column by column. */
static void lu_inverse(const cplx *lu, const int *perm, int m, cplx *inv)
{
    cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    for (int e = 0; e < m; ++e) {
        for (int r = 0; r < m; ++r) col[r] = (perm[r] == e) ? 1.0 : 0.0;
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < r; ++c) col[r] -= lu[r * m + c] * col[c];
        for (int r = m - 1; r >= 0; --r) {
            for (int c = r + 1; c < m; ++c) col[r] -= lu[r * m + c] * col[c];
            col[r] /= lu[r * m + r];
        }
        for (int r = 0; r < m; ++r) inv[r * m + e] = col[r];
    }
    free(col);
}

/* C (p x r) = A (p x q) * B (q x r), all row-major. */
static void matmul(const cplx *A, const cplx *B, cplx *C, int p, int q, int r)
{
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < r; ++j) {
            cplx acc = 0.0;
            for (int l = 0; l < q; ++l) acc += A[i * q + l] * B[l * r + j];
            C[i * r + j] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Circuit                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, n_rot, k;
    cplx *rot;          /* [n_rot][n][n] */
    const int *pairs;
    const int *layer;
    const double *theta;
} circuit;

static void circuit_load(circuit *c, int n, int n_rot, const double *rot, int k,
                         const int *pairs, const int *layer, const double *theta)
{
    c->n = n; c->n_rot = n_rot; c->k = k;
    c->pairs = pairs; c->layer = layer; c->theta = theta;
    size_t nn = (size_t)n_rot * n * n;
    c->rot = (cplx *)malloc(sizeof(cplx) * nn);
    for (size_t i = 0; i < nn; ++i) c->rot[i] = rot[2 * i] + I * rot[2 * i + 1];
}

/* Diagonal of the CPhase layer between rotation layers l and l+1 for
 * trajectory x: mode q gets prod over the layer's gates j touching q of
 * e^{i theta_j/2} (x_j = 0, d_0) or -e^{i theta_j/2} (x_j = 1, d_1). */
static void layer_diag(const circuit *c, int l, const uint64_t x[2], cplx *d)
{
    for (int q = 0; q < c->n; ++q) d[q] = 1.0;
    for (int j = 0; j < c->k; ++j) {
        if (c->layer[j] != l) continue;
        cplx f = cexp(I * c->theta[j] / 2.0);
        if (bit_of(x, j)) f = -f;
        d[c->pairs[2 * j]] *= f;
        d[c->pairs[2 * j + 1]] *= f;
    }
}

/* Columns C of V(x) = R_L D_{L-1}(x) R_{L-1} ... D_0(x) R_0 (Eq. 14 extended to
 * several CPhase layers), evaluated right to left: Y = R_0[:, C], then for each
 * later layer Y <- R_l (D_{l-1} Y).  Output n x m row-major. */
static void mode_matrix_cols(const circuit *c, const uint64_t x[2], const int *C, int m, cplx *Y)
{
    int n = c->n;
    cplx *d = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n * m);
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < m; ++a) Y[r * m + a] = c->rot[r * n + C[a]];
    for (int l = 1; l < c->n_rot; ++l) {
        layer_diag(c, l - 1, x, d);
        for (int r = 0; r < n; ++r)
            for (int a = 0; a < m; ++a) tmp[r * m + a] = d[r] * Y[r * m + a];
        matmul(c->rot + (size_t)l * n * n, tmp, Y, n, n, m);
    }
    free(d); free(tmp);
}

/* Exact weight, Eq. 8-9 (with the exponent read as 1 - x_j):
 * w(x) = prod_j cos(theta_j/4)^{1-x_j} (i sin(theta_j/4))^{x_j}. */
static cplx exact_weight(const circuit *c, const uint64_t x[2])
{
    cplx w = 1.0;
    for (int j = 0; j < c->k; ++j)
        w *= bit_of(x, j) ? I * sin(c->theta[j] / 4.0) : cos(c->theta[j] / 4.0);
    return w;
}

/* Extent, Eq. 5: xi* = prod_j (cos(|theta_j|/4) + sin(|theta_j|/4))^2. */
double xfo_extent(int k, const double *theta)
{
    double xi = 1.0;
    for (int j = 0; j < k; ++j) {
        double f = cos(fabs(theta[j]) / 4.0) + sin(fabs(theta[j]) / 4.0);
        xi *= f * f;
    }
    return xi;
}

/* Raw Estimate importance weight of one sample: w(x)/P(x) = sqrt(xi*) phase(x)
 * with phase(x) = prod_{x_j=1} i sign(theta_j). */
static cplx sample_phase(const circuit *c, const uint64_t x[2])
{
    cplx ph = 1.0;
    for (int j = 0; j < c->k; ++j)
        if (bit_of(x, j)) ph *= (c->theta[j] < 0.0) ? -I : I;
    return ph;
}

static int cmp_x(const void *pa, const void *pb)
{
    const uint64_t *a = (const uint64_t *)pa, *b = (const uint64_t *)pb;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    return 0;
}

/* One term of a bitstring's sum: trajectory x and its complex weight. */
typedef struct { uint64_t x[2]; cplx w; } term;

/* The term list of bitstring b: all 2^k trajectories with w(x) (exact), or
 * the distinct sampled trajectories with (sqrt(xi*)/t) * count * phase(x). */
static int build_terms(const circuit *c, int mode, int64_t t, uint64_t seed, uint64_t bidx,
                       const uint32_t *T, double sqrt_xi, term **out)
{
    if (mode == 0) {
        int64_t nx = (int64_t)1 << c->k;
        term *ts = (term *)malloc(sizeof(term) * (size_t)nx);
        for (int64_t xi = 0; xi < nx; ++xi) {
            ts[xi].x[0] = (uint64_t)xi; ts[xi].x[1] = 0;
            ts[xi].w = exact_weight(c, ts[xi].x);
        }
        *out = ts;
        return (int)nx;
    }
    uint64_t *xs = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)t);
    for (int64_t s = 0; s < t; ++s) sample_trajectory(c->k, T, seed, bidx, (uint32_t)s, xs + 2 * s);
    qsort(xs, (size_t)t, 2 * sizeof(uint64_t), cmp_x);
    term *ts = (term *)malloc(sizeof(term) * (size_t)t);
    int nt = 0;
    for (int64_t s = 0; s < t;) {
        int64_t e = s;
        while (e < t && xs[2 * e] == xs[2 * s] && xs[2 * e + 1] == xs[2 * s + 1]) e++;
        ts[nt].x[0] = xs[2 * s]; ts[nt].x[1] = xs[2 * s + 1];
        ts[nt].w = (sqrt_xi / (double)t) * (double)(e - s) * sample_phase(c, ts[nt].x);
        nt++;
        s = e;
    }
    free(xs);
    *out = ts;
    return nt;
}

/*
 * Probabilities.  mode 0 = Exact (Eq. 8), mode 1 = Raw Estimate.
 * theta_sample (nullable) gives the angles the sampling table is built from;
 * the weights sqrt(xi*) phase(x) and the circuit itself always use theta.
 * Holding theta_sample fixed while theta moves freezes the samples, which is
 * what a derivative of the estimator with respect to theta differentiates.
 * batch_index (nullable) gives the index that keys bitstring b's samples
 * (default b), so a subset of a larger batch can be recomputed.
 * prob[B], amp[B][2] (nullable), abssum[B] (nullable): the sum of the terms'
 * magnitudes, sum_i |w_i det M_i|, whose ratio to |A_b| measures how much the
 * terms cancel.  Returns 0, or -1 on unsupported sizes.
 */
int xfo_probabilities(int n, int n_rot, const double *rot, int k, const int *pairs,
                      const int *layer, const double *theta, const double *theta_sample,
                      const uint64_t *input_bits, int64_t B, const uint64_t *bits,
                      const uint64_t *batch_index, int mode, int64_t t, uint64_t seed,
                      double *prob, double *amp, double *abssum)
{
    if (n < 1 || n > 128 || n_rot < 1 || k < 0 || (mode == 0 && k > 24) || (mode == 1 && (k > 128 || t < 1)))
        return -1;
    circuit c;
    circuit_load(&c, n, n_rot, rot, k, pairs, layer, theta);
    int C[128];
    int m = occupied(input_bits, n, C);
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(k > 0 ? k * k : 1));
    xfo_sampler_table(k, theta_sample ? theta_sample : theta, T);
    double sqrt_xi = sqrt(xfo_extent(k, theta));

    /* Exact mode: V(x)[:, C] is the same for every bitstring; build it once. */
    int64_t nx = (mode == 0) ? ((int64_t)1 << k) : 0;
    cplx *Ycache = NULL;
    if (mode == 0) {
        Ycache = (cplx *)malloc(sizeof(cplx) * (size_t)nx * n * (m > 0 ? m : 1));
        #pragma omp parallel for schedule(dynamic)
        for (int64_t xi = 0; xi < nx; ++xi) {
            uint64_t x[2] = { (uint64_t)xi, 0 };
            mode_matrix_cols(&c, x, C, m, Ycache + (size_t)xi * n * m);
        }
    }

    #pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < B; ++b) {
        int R[128];
        int mb = occupied(bits + 2 * b, n, R);
        cplx A = 0.0;
        double S = 0.0;
        if (mb == m) {
            term *ts;
            int nt = build_terms(&c, mode, t, seed, batch_index ? batch_index[b] : (uint64_t)b, T, sqrt_xi, &ts);
            cplx *Y = (cplx *)malloc(sizeof(cplx) * (size_t)n * (m > 0 ? m : 1));
            cplx *M = (cplx *)malloc(sizeof(cplx) * (size_t)(m > 0 ? m * m : 1));
            int *perm = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
            for (int i = 0; i < nt; ++i) {
                const cplx *Yx;
                if (mode == 0) Yx = Ycache + (size_t)ts[i].x[0] * n * m;
                else { mode_matrix_cols(&c, ts[i].x, C, m, Y); Yx = Y; }
                for (int r = 0; r < m; ++r)
                    for (int a = 0; a < m; ++a) M[r * m + a] = Yx[R[r] * m + a];
                int sing;
                cplx det = (m == 0) ? 1.0 : lu_factor(M, m, perm, &sing);
                A += ts[i].w * det;
                S += cabs(ts[i].w * det);
            }
            free(Y); free(M); free(perm); free(ts);
        }
        prob[b] = creal(A) * creal(A) + cimag(A) * cimag(A);
        if (amp) { amp[2 * b] = creal(A); amp[2 * b + 1] = cimag(A); }
        if (abssum) abssum[b] = S;
    }
    free(Ycache);
    free(T);
    free(c.rot);
    return 0;
}

/*
 * Gradient of L = sum_b g[b] * log p_b with respect to every rotation entry
 * and every angle, by the chain rule written out plainly:
 *   d log p_b = 2 Re(dA_b / A_b),  A_b = sum_x w_x det M_x,
 *   d det M = det M * tr(M^{-1} dM)   (Jacobi's formula),
 *   M_x = [P_l R_l Q_l][R, C] for every rotation layer l, where P_l is the
 *   product to the left of R_l and Q_l the product to its right.
 * In Raw Estimate mode the samples are held fixed; the weights depend on the
 * angles only through sqrt(xi*) (the phases are piecewise constant).
 * grad_rot [n_rot][n][n][2] receives dL/dRe + i dL/dIm; grad_theta [k].
 * Bitstrings whose amplitude is exactly zero contribute nothing.
 */
int xfo_log_prob_grad(int n, int n_rot, const double *rot, int k, const int *pairs,
                      const int *layer, const double *theta, const double *theta_sample,
                      const uint64_t *input_bits, int64_t B, const uint64_t *bits,
                      const uint64_t *batch_index, int mode, int64_t t, uint64_t seed,
                      const double *g, double *grad_rot, double *grad_theta)
{
    if (n < 1 || n > 128 || n_rot < 1 || k < 0 || (mode == 0 && k > 24) || (mode == 1 && (k > 128 || t < 1)))
        return -1;
    circuit c;
    circuit_load(&c, n, n_rot, rot, k, pairs, layer, theta);
    int C[128];
    int m = occupied(input_bits, n, C);
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(k > 0 ? k * k : 1));
    xfo_sampler_table(k, theta_sample ? theta_sample : theta, T);
    double sqrt_xi = sqrt(xfo_extent(k, theta));
    size_t nrot_el = (size_t)n_rot * n * n;

    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    /* per-thread partial sums, added in thread order at the end */
    cplx *Gpart = (cplx *)calloc(nrot_el * (size_t)nthreads, sizeof(cplx));
    double *Tpart = (double *)calloc((size_t)(k > 0 ? k : 1) * (size_t)nthreads, sizeof(double));

    #pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *Gl = Gpart + nrot_el * (size_t)tid;
        double *Tl = Tpart + (size_t)(k > 0 ? k : 1) * (size_t)tid;
        cplx *Zl = (cplx *)malloc(sizeof(cplx) * (size_t)n_rot * m * n);  /* M^{-1} (P_{l+1} R_{l+1})[R, :] */
        /* scratch */
        cplx *Qc = (cplx *)malloc(sizeof(cplx) * (size_t)n_rot * n * m);   /* Q_l[:, C]  (n x m) */
        cplx *PR = (cplx *)malloc(sizeof(cplx) * (size_t)n_rot * m * n);   /* P_l[R, :]  (m x n) */
        cplx *Dg = (cplx *)malloc(sizeof(cplx) * (size_t)n_rot * n);       /* D_l diagonals */
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
        cplx *tmp2 = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
        cplx *M = (cplx *)malloc(sizeof(cplx) * (size_t)(m > 0 ? m * m : 1));
        cplx *Mi = (cplx *)malloc(sizeof(cplx) * (size_t)(m > 0 ? m * m : 1));
        cplx *dA_th = (cplx *)malloc(sizeof(cplx) * (size_t)(k > 0 ? k : 1));
        cplx *dA_rot = (cplx *)malloc(sizeof(cplx) * nrot_el);
        int *perm = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));

        #pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < B; ++b) {
            int R[128];
            int mb = occupied(bits + 2 * b, n, R);
            if (mb != m || g[b] == 0.0) continue;
            term *ts;
            int nt = build_terms(&c, mode, t, seed, batch_index ? batch_index[b] : (uint64_t)b, T, sqrt_xi, &ts);
            cplx A = 0.0;
            memset(dA_rot, 0, sizeof(cplx) * nrot_el);
            for (int j = 0; j < k; ++j) dA_th[j] = 0.0;
            for (int i = 0; i < nt; ++i) {
                const uint64_t *x = ts[i].x;
                /* D_l(x) for each CPhase layer l = 0..n_rot-2 */
                for (int l = 0; l + 1 < n_rot; ++l) layer_diag(&c, l, x, Dg + (size_t)l * n);
                /* Q_l[:, C] = (D_{l-1} R_{l-1} ... D_0 R_0)[:, C]; Q_0[:, C] = I[:, C] */
                for (int r = 0; r < n; ++r)
                    for (int a = 0; a < m; ++a) Qc[r * m + a] = (r == C[a]) ? 1.0 : 0.0;
                for (int l = 1; l < n_rot; ++l) {
                    const cplx *Rp = c.rot + (size_t)(l - 1) * n * n;
                    matmul(Rp, Qc + (size_t)(l - 1) * n * m, tmp, n, n, m);
                    for (int r = 0; r < n; ++r)
                        for (int a = 0; a < m; ++a)
                            Qc[(size_t)l * n * m + r * m + a] = Dg[(size_t)(l - 1) * n + r] * tmp[r * m + a];
                }
                /* P_l[R, :] = (R_L D_{L-1} ... R_{l+1} D_l)[R, :]; P_L[R, :] = I[R, :] */
                int L = n_rot - 1;
                for (int a = 0; a < m; ++a)
                    for (int q = 0; q < n; ++q) PR[(size_t)L * m * n + a * n + q] = (q == R[a]) ? 1.0 : 0.0;
                for (int l = L - 1; l >= 0; --l) {
                    const cplx *Rn = c.rot + (size_t)(l + 1) * n * n;
                    matmul(PR + (size_t)(l + 1) * m * n, Rn, tmp, m, n, n);
                    for (int a = 0; a < m; ++a)
                        for (int q = 0; q < n; ++q)
                            PR[(size_t)l * m * n + a * n + q] = tmp[a * n + q] * Dg[(size_t)l * n + q];
                }
                /* M = P_0[R, :] R_0 Q_0[:, C] */
                matmul(PR, c.rot, tmp, m, n, n);
                matmul(tmp, Qc, M, m, n, m);
                int sing;
                cplx det = (m == 0) ? 1.0 : lu_factor(M, m, perm, &sing);
                /* An exactly singular M has det = 0: it adds nothing to A, and its
                 * adjugate term in dA is dropped (measure-zero for generic inputs). */
                if (m > 0 && sing) continue;
                A += ts[i].w * det;
                if (m > 0) lu_inverse(M, perm, m, Mi);
                cplx beta = ts[i].w * det;
                /* rotation entries: dA/d(R_l)_{pq} += beta * (Q_l[:, C] M^{-1} P_l[R, :])_{qp} */
                for (int l = 0; l < n_rot; ++l) {
                    matmul(Qc + (size_t)l * n * m, Mi, tmp, n, m, m);
                    matmul(tmp, PR + (size_t)l * m * n, tmp2, n, m, n);
                    for (int p = 0; p < n; ++p)
                        for (int q = 0; q < n; ++q)
                            dA_rot[(size_t)l * n * n + p * n + q] += beta * tmp2[q * n + p];
                }
                /* angles through D_l: dD_l/dtheta_j = (i/2)(E_q1 + E_q2) D_l, so
                 * d log det M = (i/2) sum_q [Q_{l+1}[:, C] M^{-1} (P_{l+1} R_{l+1})[R, :]]_{qq} */
                for (int l = 0; l + 1 < n_rot; ++l) {
                    matmul(PR + (size_t)(l + 1) * m * n, c.rot + (size_t)(l + 1) * n * n, tmp, m, n, n);
                    matmul(Mi, tmp, Zl + (size_t)l * m * n, m, m, n);
                }
                for (int j = 0; j < k; ++j) {
                    int l = layer[j];
                    const cplx *Q1 = Qc + (size_t)(l + 1) * n * m;
                    const cplx *Z = Zl + (size_t)l * m * n;
                    cplx tr = 0.0;
                    for (int side = 0; side < 2; ++side) {
                        int q = pairs[2 * j + side];
                        for (int a = 0; a < m; ++a) tr += Q1[q * m + a] * Z[a * n + q];
                    }
                    dA_th[j] += beta * (I / 2.0) * tr;
                    /* weight dependence */
                    cplx dw;
                    if (mode == 0) {
                        cplx rest = 1.0;
                        for (int jj = 0; jj < k; ++jj) {
                            if (jj == j) continue;
                            rest *= bit_of(x, jj) ? I * sin(theta[jj] / 4.0) : cos(theta[jj] / 4.0);
                        }
                        dw = rest * (bit_of(x, j) ? I * cos(theta[j] / 4.0) / 4.0 : -sin(theta[j] / 4.0) / 4.0);
                    } else {
                        double sg = (theta[j] > 0.0) ? 1.0 : (theta[j] < 0.0 ? -1.0 : 0.0);
                        double s = sin(fabs(theta[j]) / 4.0), cc = cos(fabs(theta[j]) / 4.0);
                        double dlog = sg * (cc - s) / (4.0 * (s + cc));
                        dw = ts[i].w * dlog;
                    }
                    dA_th[j] += dw * det;
                }
            }
            free(ts);
            if (A == 0.0) continue;
            cplx f = g[b] / A;
            for (size_t e = 0; e < nrot_el; ++e) Gl[e] += f * dA_rot[e];
            for (int j = 0; j < k; ++j) Tl[j] += 2.0 * creal(f * dA_th[j]);
        }
        free(Zl); free(Qc); free(PR); free(Dg); free(tmp); free(tmp2);
        free(M); free(Mi); free(dA_th); free(dA_rot); free(perm);
    }
    cplx *Gacc = (cplx *)calloc(nrot_el, sizeof(cplx));
    double *Tacc = (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
    for (int th = 0; th < nthreads; ++th) {
        for (size_t e = 0; e < nrot_el; ++e) Gacc[e] += Gpart[nrot_el * (size_t)th + e];
        for (int j = 0; j < k; ++j) Tacc[j] += Tpart[(size_t)(k > 0 ? k : 1) * (size_t)th + j];
    }
    free(Gpart); free(Tpart);
    /* dL = 2 Re sum G dZ  =>  dL/dRe + i dL/dIm = 2 conj(G) */
    for (size_t e = 0; e < nrot_el; ++e) {
        grad_rot[2 * e] = 2.0 * creal(Gacc[e]);
        grad_rot[2 * e + 1] = -2.0 * cimag(Gacc[e]);
    }
    for (int j = 0; j < k; ++j) grad_theta[j] = Tacc[j];
    free(Gacc); free(Tacc); free(T); free(c.rot);
    return 0;
}
