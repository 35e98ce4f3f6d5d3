// General determinant-lemma evaluation: exact mode and Raw Estimate, one or
// two CPhase layers, bases of up to 32 rows, optionally split into two
// independent blocks of modes.
//
// For one CPhase layer the trajectory submatrix is M_N = M_0 - 2 U[:, N] V[N, :]
// with M_0 = P[R, :], U = A1[R, act], V = Phi0[act, :] (Sec. IV-B Eq. 16-19);
// for two layers (the same form applied twice) U = [T[R, act0] | R'_2[R, act1]],
// V = [Phi0[act0, :]; Q[act1, :] - 2 R'_1[act1, N0] Phi0[N0, :]], whose last
// term depends on the layer-0 pattern N0.  The matrix determinant lemma gives
//   det M_N = det M_0 det S_N,  S_N = I - 2 (V M_0^-1 U)[N, N],
// and with H = [Phi0[act0, :]; Q[act1, :]] M_0^-1 U formed once per bitstring,
// row i of S_N (flipped mode n_i, position p_i in act) is
//   delta_ij - 2 H[p_i, p_j]                                  (n_i in N0)
//   delta_ij - 2 (H[p_i, p_j] - 2 sum_{l in N0} R'_1[n_i, n_l] H[p_l, p_j])  (n_i in N1).
//
// Block factorisation: when every rotation layer is block-diagonal over a
// partition of the modes (for instance spin-restricted layers U (+) U),
// V(x) is block-diagonal for every trajectory (the CPhase layers are
// diagonal), so det V(x)[R, C] is the product of the blocks' determinants
// (zero unless R and C have the same number of modes in every block), and
// each block has its own base, H and S_N.
//
// Per bitstring: the blocks' bases M_0 are inverted by Gauss-Jordan with
// partial pivoting (one wave, a block per half-wave: k_gen_setup_wave; the
// workgroup form gen_setup_block for the shifted bases of k_gen_setup),
// checked for conditioning (kappa_1 <= 1e4, else a shifted base, else the
// LU kernels), and X = M_0^-1 U, H = V X are formed on the matrix cores
// (v_mfma_f64_16x16x4f64; with MIXED, v_mfma_f32_16x16x4f32 on FP32-rounded
// operands).  Then every distinct pattern takes an r x r determinant per
// block: one lane for r <= 4, lane groups of 8, 16 or 32 above; the weighted
// determinants are summed exactly.
#pragma once
#include "xf_device.h"

namespace xf {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kGenMaxM = 32;      // rows of a block's base
constexpr int kGenMaxKb = 64;     // active modes of a block (both layers)
constexpr int kGenMaxRank = 32;   // flipped modes of a block in one pattern
constexpr int kGenMaxSteps = kGenMaxM / 4;   // 4-wide K slices of a product over a base
// Setup scratch (the augmented base and X) overlays the entry slots, pivot
// scratch and reduction scratch of the RawSmem layout: 40960 bytes.
constexpr size_t kGenSetupBytes = (size_t)kHashSlots * 16 + 2 * (size_t)kThreads * 16;
// The pattern evaluation takes a bitstring's entries in chunks of SLOTS
// (lane groups of 32: 2048, else 1024, so that two workgroups fit a CU);
// bytes of its entry slots (keys, counts, list) and pivot and reduction
// scratch.
template <int SLOTS>
constexpr size_t gen_base_bytes() {
    return ((size_t)SLOTS * (8 + 8 + 2) + 2 * (size_t)kThreads * 16 + 15) & ~(size_t)15;
}
constexpr uint16_t kNoPos = 0xFFFF;

// Plan tables the general kernels keep in LDS (after the RawSmem layout):
// every block's H (kb x hld, hld odd so that a lane group's rows fall in
// different banks), the lane groups' LU pivot rows, R'_1[act1, act0] of every
// block (two CPhase layers), the key-bit table, and the blocks' active modes
// and input columns.
struct GenLds {
    double2 *H, *gpiv, *R1a;
    uint16_t *kbt;
    uint8_t *act, *col;
};

__host__ __device__ __forceinline__ size_t gen_tables_bytes(const GenPlan &g) {
    return align16((size_t)g.hsize * 16) + (size_t)kThreads * 16 + align16((size_t)g.r1size * 16) + 256 + 128 + 64;
}

template <int SLOTS>
__device__ __forceinline__ GenLds carve_gen(unsigned char *smem, const GenPlan &g) {
    GenLds t;
    unsigned char *q = smem + gen_base_bytes<SLOTS>();
    t.H = (double2 *)q;
    q += align16((size_t)g.hsize * 16);
    t.gpiv = (double2 *)q;
    q += (size_t)kThreads * 16;
    t.R1a = (double2 *)q;
    q += align16((size_t)g.r1size * 16);
    t.kbt = (uint16_t *)q;
    t.act = q + 256;
    t.col = q + 256 + 128;
    return t;
}

// Copies the plan tables into LDS (once per workgroup).
__device__ __forceinline__ void load_gen_tables(const DevPlan &p, const GenPlan &g, const GenLds &t) {
    const int tid = threadIdx.x;
    for (int e = tid; e < 128; e += kThreads) t.kbt[e] = g.kbt[e];
    for (int e = tid; e < 2 * kGenMaxKb; e += kThreads) t.act[e] = g.act[e];
    for (int e = tid; e < 2 * kGenMaxM; e += kThreads) t.col[e] = g.col[e];
    if (g.multi) {
        for (int blk = 0; blk < g.nblk; ++blk) {
            const int kb = g.kb[blk];
            for (int e = tid; e < kb * kb; e += kThreads)
                t.R1a[g.r1off[blk] + e] = g.TT[((size_t)blk * 64 + e / kb) * 64 + e % kb];
        }
    } else if (p.L == 2) {
        for (int blk = 0; blk < g.nblk; ++blk) {
            const int kb0 = g.kb0[blk], kb1 = g.kb[blk] - kb0;
            const uint8_t *act = g.act + blk * kGenMaxKb;
            for (int e = tid; e < kb1 * kb0; e += kThreads) {
                const int p1 = e / kb0, p0 = e % kb0;
                t.R1a[g.r1off[blk] + e] = p.R1[(size_t)act[kb0 + p1] * p.n + act[p0]];
            }
        }
    }
    __syncthreads();
}

// C (M x N) = A (M x K) B (K x N), complex, on the matrix cores, K <= 32.
// a_at(i, k) and b_at(k, j) return operands, c_put(i, j, v) stores a result.
// Each wave of the workgroup computes whole 16 x 16 tiles of C: lane l
// supplies A[16 tm + l % 16][k0 + l / 16] and B[k0 + l / 16][16 tn + l % 16]
// for every 4-wide slice k0 of K (all loaded before the first product, so
// their latencies overlap), and the four real products re.re, -im.im, re.im,
// im.re accumulate into the real and imaginary tiles.  Lane l then holds, in
// element r, C[16 tm + i][16 tn + l % 16] with i = l / 16 + 4 r for the FP64
// instruction and i = 4 (l / 16) + r for the FP32 one (the two order their
// output rows differently).  Out-of-range operands are zero.
template <bool F32, class FA, class FB, class FC>
__device__ __forceinline__ void cgemm_mfma(int M, int N, int K, FA a_at, FB b_at, FC c_put) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kThreads / 64;
    const int tm_n = (M + 15) / 16, tn_n = (N + 15) / 16;
    const int li = lane & 15, lk = lane >> 4;
    const int ns = (K + 3) / 4;
    for (int t = wave; t < tm_n * tn_n; t += NW) {
        const int tm = t / tn_n, tn = t % tn_n;
        const int row = tm * 16 + li, col = tn * 16 + li;
        double2 av[kGenMaxSteps], bv[kGenMaxSteps];
#pragma unroll
        for (int st = 0; st < kGenMaxSteps; ++st) {
            const int k = 4 * st + lk;
            av[st] = (st < ns && row < M && k < K) ? a_at(row, k) : make_double2(0.0, 0.0);
            bv[st] = (st < ns && k < K && col < N) ? b_at(k, col) : make_double2(0.0, 0.0);
        }
        if constexpr (!F32) {
            d4v cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < kGenMaxSteps; ++st) {
                if (st < ns) {
                    const double2 a = av[st], b = bv[st];
                    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
                    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = tm * 16 + lk + 4 * r;
                if (orow < M && col < N) c_put(orow, col, make_double2(cr[r], ci[r]));
            }
        } else {
            f4v cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < kGenMaxSteps; ++st) {
                if (st < ns) {
                    const float ax = (float)av[st].x, ay = (float)av[st].y;
                    const float bx = (float)bv[st].x, by = (float)bv[st].y;
                    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, bx, cr, 0, 0, 0);
                    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ay, by, cr, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, by, ci, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(ay, bx, ci, 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = tm * 16 + 4 * lk + r;
                if (orow < M && col < N) c_put(orow, col, make_double2((double)cr[r], (double)ci[r]));
            }
        }
    }
}

// Value of v in lane `src` (wave-uniform) for every lane.
__device__ __forceinline__ double read_lane_d(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double2 read_lane_c(double2 v, int src) {
    return make_double2(read_lane_d(v.x, src), read_lane_d(v.y, src));
}

// Per-bitstring shared state of the general kernels.
struct GenShared {
    int ok;                        // row counts / base status
    int piv[kGenMaxM];             // pivot row of each column (Gauss-Jordan)
    double2 uinv[kGenMaxM];        // 1 / pivot
    double2 det;                   // product of the blocks' det M_0
    double norm;                   // ||M_0||_1 of the current block
    double kappa;                  // kappa_1(M_0) of the current block
    int nrow[2];                   // rows of R in each block
    uint8_t rows[2][kGenMaxM];     // those rows (modes), ascending
    uint64_t shift[2];             // positions of each block's base pattern N* (see gen_setup_block)
};

__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

// Rows of the loaded bitstring in each block (thread 0); sh.ok = 0 if a
// block's count differs from the input's (the amplitude is then zero).
__device__ __forceinline__ void gen_rows(const DevPlan &p, const GenPlan &g, const uint8_t *Rb, GenShared &sh) {
    if (threadIdx.x == 0) {
        sh.nrow[0] = sh.nrow[1] = 0;
        sh.ok = 1;
        for (int r = 0; r < p.m; ++r) {
            const int q = Rb[r];
            const int blk = (int)((g.bmask[1][q >> 6] >> (q & 63)) & 1);
            if (sh.nrow[blk] < kGenMaxM) sh.rows[blk][sh.nrow[blk]] = (uint8_t)q;
            ++sh.nrow[blk];
        }
        for (int blk = 0; blk < g.nblk; ++blk)
            if (sh.nrow[blk] != g.mb[blk]) sh.ok = 0;
        sh.det = make_double2(1.0, 0.0);
        sh.shift[0] = sh.shift[1] = 0;
    }
}

// Setup of block blk for the loaded bitstring: the base M_B = M_{N*} (N* the
// base pattern, empty at first) is inverted by Gauss-Jordan (augmented rows
// [M_B | I] in the setup scratch W, row stride 2m; rows stay in place, row
// piv[c] ends as u_c e_c | u_c M_B^-1[c, :]) and checked for conditioning;
// then X = M_B^-1 U and H = V X.  A singular or ill-conditioned M_0 is
// replaced by M_{N*} with N* the flips of one gate (of layer 0 for two
// CPhase layers; the first few gates touching the block are tried in turn):
// with Delta = N xor N* and sigma = -1 on N* \ N, +1 on N \ N*,
//   M_N = M_{N*} - 2 U[:, Delta] diag(sigma) V_N[Delta, :],
//   det M_N = det M_{N*} det(I - 2 diag(sigma) V_N[Delta, :] M_{N*}^-1 U[:, Delta]),
// where for two layers the layer-1 rows of V_N carry the pattern's own
// layer-0 flips N0 (N* has none in layer 1, so those rows keep sigma = +1).
// Returns false if no base was acceptable (kappa_1 > kLemmaMaxCond or
// singular).  Whole workgroup.
constexpr int kGenBaseTries = 4;

template <bool MIXED, bool MULTI>
__device__ __forceinline__ bool gen_setup_block(const DevPlan &p, const GenPlan &g, const GenLds &T, int blk,
                                                unsigned char *scratch, GenShared &sh, Work &wk) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int m = g.mb[blk], kb = g.kb[blk], kb0 = g.kb0[blk], hld = g.hld[blk], n = p.n, G = p.G;
    const uint8_t *rows = sh.rows[blk];
    const uint8_t *col = T.col + blk * kGenMaxM;
    const uint8_t *act = T.act + blk * kGenMaxKb;
    double2 *H = T.H + g.hoff[blk];
    double2 *W = (double2 *)scratch;
    const int ld = 2 * m;
    double2 *X = (double2 *)(scratch + align16((size_t)m * ld * 16));
    if (m == 0) {
        for (int e = tid; e < kb * hld; e += kThreads) H[e] = make_double2(0.0, 0.0);
        __syncthreads();
        return true;
    }
    int gate = -1;   // base pattern: the flips of this gate in the block (-1: none)
    for (int attempt = 0;; ++attempt) {
    uint64_t bmask = 0;   // positions of N* in this block
    if (gate >= 0) {
        for (int e = 0; e < 2; ++e) {
            const uint16_t v = g.gpos[2 * gate + e];
            if (v != kNoPos && (v >> 8) == blk) bmask ^= 1ull << (v & 0xFF);
        }
    }
    for (int e = tid; e < m * ld; e += kThreads) {
        const int i = e / ld, j = e % ld;
        double2 v;
        if (j < m) {
            v = p.P[(size_t)rows[i] * G + col[j]];
            for (uint64_t mm = bmask; mm; mm &= mm - 1) {
                const int c = act[__ffsll((long long)mm) - 1];
                const double2 a1 = p.A1[(size_t)rows[i] * n + c];
                v = c_fma(v, make_double2(-2.0 * a1.x, -2.0 * a1.y), p.Phi0[(size_t)c * G + col[j]]);
            }
        } else {
            v = make_double2(j - m == i ? 1.0 : 0.0, 0.0);
        }
        W[e] = v;
    }
    __syncthreads();
    if (tid < 64) {
        double cs = 0.0;
        if (lane < m)
            for (int i = 0; i < m; ++i) cs += sqrt(cabs2(W[i * ld + lane]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
        if (lane == 0) sh.norm = cs;
    }
    // Elimination: every wave finds the pivot of column c itself (the same
    // reduction over the same values gives the same row in all waves), so one
    // barrier per column suffices; lane j - c - 1 of every wave updates column
    // j > c in the wave's rows (wave, wave + 4, ...), the multipliers coming
    // from the lanes that read column c.
    __syncthreads();   // the norm has been read
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = kThreads / 64;
    uint64_t used = 0;          // rows already used as pivots
    unsigned inversions = 0;
    double2 det = make_double2(1.0, 0.0);
    bool singular = false;
    for (int c = 0; c < m; ++c) {
        const double2 a = lane < m ? W[lane * ld + c] : make_double2(0.0, 0.0);
        const bool act_row = lane < m && !((used >> lane) & 1);
        double best = act_row ? cabs2(a) : -1.0;
        int idx = lane;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double vo = __shfl_xor(best, off, 64);
            const int io = __shfl_xor(idx, off, 64);
            if (vo > best || (vo == best && io < idx)) {
                best = vo;
                idx = io;
            }
        }
        idx = __builtin_amdgcn_readfirstlane(idx);
        best = read_lane_d(best, 0);
        if (!(best > 0.0)) {
            singular = true;   // exactly singular base (the same decision in every wave)
            break;
        }
        inversions += __popcll(~used & ((1ull << idx) - 1) & ((1ull << m) - 1));
        used |= 1ull << idx;
        const double2 u = read_lane_c(a, idx);
        det = c_mul(det, u);
        const double inv = 1.0 / best;
        const double2 ui = make_double2(u.x * inv, -u.y * inv);
        if (tid == 0) {
            sh.piv[c] = idx;
            sh.uinv[c] = ui;
        }
        const double2 l = (lane < m && lane != idx)
                              ? make_double2(-(a.x * ui.x - a.y * ui.y), -(a.x * ui.y + a.y * ui.x))
                              : make_double2(0.0, 0.0);
        const int j = c + 1 + lane;
        const bool jin = j < ld;
        const double2 pv = jin ? W[idx * ld + j] : make_double2(0.0, 0.0);
        double2 v[kGenMaxM / NW];
#pragma unroll
        for (int q = 0; q < kGenMaxM / NW; ++q) {
            const int i = wave + NW * q;
            v[q] = (jin && i < m) ? W[i * ld + j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < kGenMaxM / NW; ++q) {
            const int i = wave + NW * q;
            if (i < m) {
                const double2 li = read_lane_c(l, i);
                if (jin && i != idx) W[i * ld + j] = c_fma(v[q], li, pv);
            }
        }
        __syncthreads();
    }
    // det M_B (wave 0) and the conditioning: ||M_B^-1||_1 from rows piv[c] / u_c
    if (!singular && tid < 64) {
        double cs = 0.0;
        if (lane < m)
            for (int c = 0; c < m; ++c) cs += sqrt(cabs2(c_mul(W[sh.piv[c] * ld + m + lane], sh.uinv[c])));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
        if (lane == 0) {
            const bool good = cs * sh.norm <= kLemmaMaxCond;
            sh.ok = good ? 1 : 2;
            sh.kappa = cs * sh.norm;
            if (good) {
                if (inversions & 1) det = make_double2(-det.x, -det.y);
                sh.det = c_mul(sh.det, det);
                sh.shift[blk] = bmask;
            }
            // Gauss-Jordan (m steps of m - 1 row updates over 2m - c - 1
            // columns), conditioning, X and H
            unsigned long long f = 0;
            for (int c = 0; c < m; ++c) f += 11ull * (m - 1) + 8ull * (m - 1) * (2 * m - c - 1);
            if (good) f += 8ull * m * m * kb + 8ull * kb * m * kb;
            wk.flops += f;
        }
    }
    __syncthreads();
    if (!singular && sh.ok == 1) break;
    // next base: the next gate whose flips touch this block (of layer 0 for
    // two CPhase layers; more layers keep the empty pattern)
    if (MULTI || attempt + 1 >= kGenBaseTries) return false;
    auto touches = [&](uint16_t v) { return v != kNoPos && (v >> 8) == blk && (p.L == 1 || (v & 0xFF) < kb0); };
    do {
        ++gate;
    } while (gate < p.k && gate < 64 && !(touches(g.gpos[2 * gate]) || touches(g.gpos[2 * gate + 1])));
    if (gate >= p.k || gate >= 64) return false;
    __syncthreads();
    }
    // X = M_0^-1 U (m x kb), then H = V X (kb x kb), V = [Phi0[act0, cols]; Q[act1, cols]]
    const double2 *A1 = p.A1, *A2 = p.A2, *Phi0 = p.Phi0, *Q = p.Q;
    auto minv = [&](int i, int k) { return c_mul(W[sh.piv[i] * ld + m + k], sh.uinv[i]); };
    auto uop = [&](int k, int q) { return (q < kb0 ? A1 : A2)[(size_t)rows[k] * n + act[q]]; };
    auto xput = [&](int i, int q, double2 v) { X[i * kb + q] = v; };
    auto vop = [&](int q, int k) { return (q < kb0 ? Phi0 : Q)[(size_t)act[q] * G + col[k]]; };
    auto xop = [&](int k, int q) { return X[k * kb + q]; };
    auto hput = [&](int q, int q2, double2 v) { H[q * hld + q2] = v; };
    // mixed precision: FP32 matrix cores for bases with kappa_1 <= p.mixed_cond
    // (the FP32 error of H grows with ||M_B^-1||), FP64 for the others
    if constexpr (MULTI) {
        // U = GA[R, positions], V = HC[positions, cols]
        const double2 *GA = g.GA + (size_t)blk * n * 64, *HC = g.HC + (size_t)blk * 64 * G;
        auto uopm = [&](int k, int q) { return GA[(size_t)rows[k] * 64 + q]; };
        auto vopm = [&](int q, int k) { return HC[(size_t)q * G + col[k]]; };
        if (MIXED && sh.kappa <= p.mixed_cond) {
            cgemm_mfma<true>(m, kb, m, minv, uopm, xput);
            __syncthreads();
            cgemm_mfma<true>(kb, kb, m, vopm, xop, hput);
            if (tid == 0) ++wk.fp32;
        } else {
            cgemm_mfma<false>(m, kb, m, minv, uopm, xput);
            __syncthreads();
            cgemm_mfma<false>(kb, kb, m, vopm, xop, hput);
        }
    } else if (MIXED && sh.kappa <= p.mixed_cond) {
        cgemm_mfma<true>(m, kb, m, minv, uop, xput);
        __syncthreads();
        cgemm_mfma<true>(kb, kb, m, vop, xop, hput);
        if (tid == 0) ++wk.fp32;
    } else {
        cgemm_mfma<false>(m, kb, m, minv, uop, xput);
        __syncthreads();
        cgemm_mfma<false>(kb, kb, m, vop, xop, hput);
    }
    __syncthreads();
    return true;
}

// Flipped positions of a pattern in each block's H (bit p of pm[blk] <=>
// position p flipped), from the key bits through the LDS key-bit table: a
// compressed key bit names one (block, position); a trajectory bit (gate)
// names two, which cancel where gates share a mode.
__device__ __forceinline__ void gen_masks(const uint16_t *kbt, uint64_t key, uint64_t (&pm)[2]) {
    pm[0] = pm[1] = 0;
    while (key) {
        const int j = __ffsll((long long)key) - 1;
        key &= key - 1;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint16_t v = kbt[2 * j + e];
            if (v != kNoPos) pm[v >> 8] ^= 1ull << (v & 0xFF);
        }
    }
}

// The first NP set bits of mask, ascending.
template <int NP>
__device__ __forceinline__ void mask_positions(uint64_t mask, int (&pos)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        pos[i] = mask ? __ffsll((long long)mask) - 1 : 0;
        mask &= mask - 1;
    }
}

// Entry (i, j) of S in a block (i, j < r; positions pos of the flips
// relative to the base pattern N*, r0 of them in layer 0):
// delta_ij - 2 sigma_i H[p_i, p_j], with, for two CPhase layers, the
// layer-1 rows corrected by the pattern's own layer-0 flips N0, which are
// the relative positions with sigma = +1 plus `both` (flipped by the pattern
// and by the base; the base flips layer-0 modes only).
template <int NP>
__device__ __forceinline__ double2 gen_s_entry(bool two_layers, const double2 *H, int hld, const double2 *R1a,
                                               int kb0, int i, int pi, int j, int r0, const int (&pos)[NP],
                                               uint64_t neg, uint64_t both) {
    double2 h = H[pi * hld + pos[j]];
    if ((neg >> pi) & 1) h = make_double2(-h.x, -h.y);
    if (two_layers && i >= r0) {
        double2 corr = make_double2(0.0, 0.0);
        const double2 *r1 = R1a + (pi - kb0) * kb0;
#pragma unroll
        for (int l = 0; l < NP; ++l)
            if (l < r0 && !((neg >> pos[l]) & 1)) corr = c_fma(corr, r1[pos[l]], H[pos[l] * hld + pos[j]]);
        for (uint64_t mm = both; mm; mm &= mm - 1) {
            const int q = __ffsll((long long)mm) - 1;
            corr = c_fma(corr, r1[q], H[q * hld + pos[j]]);
        }
        h.x -= 2.0 * corr.x;
        h.y -= 2.0 * corr.y;
    }
    return make_double2((i == j ? 1.0 : 0.0) - 2.0 * h.x, -2.0 * h.y);
}

// Entry (i, j) of S in a block of a circuit with more than two CPhase
// layers: with K = HC M_0^-1 GA (the block's H) and TT the layer-to-layer
// transfer blocks, det M_N = det M_0 det(I + 2 TT[N, N] - 2 K[N, N]) (the
// product of the layers' I - 2 E_l expands into chains whose sum is
// GA (I + 2 TT)^-1 HC, and I + 2 TT is unit triangular in layer order).
template <int NP>
__device__ __forceinline__ double2 gen_s_entry_multi(const double2 *H, int hld, const double2 *TT, int kb, int i,
                                                     int pi, int j, const int (&pos)[NP]) {
    const double2 h = H[pi * hld + pos[j]];
    const double2 tt = TT[pi * kb + pos[j]];
    return make_double2((i == j ? 1.0 : 0.0) - 2.0 * h.x + 2.0 * tt.x, -2.0 * h.y + 2.0 * tt.y);
}

// Row `lane` of S (identity row beyond r) for a lane group: the same
// entries as gen_s_entry / gen_s_entry_multi, with the two-layer correction
// added position by position (a loop over the correcting positions around an
// unrolled loop over the row, so that the row stays in registers).
template <int GS, bool MULTI>
__device__ __forceinline__ void gen_s_row(bool two_layers, const double2 *H, int hld, const double2 *R1a, int kb0,
                                          int kb, int lane, int pi, int r, int r0, const int (&pos)[GS],
                                          uint64_t pmb, uint64_t neg, uint64_t both, double2 (&a)[GS]) {
    const bool row = lane < r;
    const double sg = ((neg >> pi) & 1) ? -2.0 : 2.0;
#pragma unroll
    for (int j = 0; j < GS; ++j) {
        double2 v = make_double2(j == lane ? 1.0 : 0.0, 0.0);
        if (row && j < r) {
            const double2 h = H[pi * hld + pos[j]];
            v.x -= sg * h.x;
            v.y -= sg * h.y;
            if constexpr (MULTI) {
                const double2 tt = R1a[pi * kb + pos[j]];
                v.x += 2.0 * tt.x;
                v.y += 2.0 * tt.y;
            }
        }
        a[j] = v;
    }
    if (!MULTI && two_layers && row && lane >= r0) {
        const uint64_t l0 = kb0 >= 64 ? ~0ull : ((1ull << kb0) - 1);
        const double2 *r1 = R1a + (pi - kb0) * kb0;
        for (uint64_t mm = (pmb & l0 & ~neg) | both; mm; mm &= mm - 1) {
            const int q = __ffsll((long long)mm) - 1;
            const double2 w = r1[q];
            const double2 w4 = make_double2(4.0 * w.x, 4.0 * w.y);
#pragma unroll
            for (int j = 0; j < GS; ++j)
                if (j < r) a[j] = c_fma(a[j], w4, H[q * hld + pos[j]]);
        }
    }
}

// det of a 4 x 4 (top-left r x r of a, identity elsewhere) by LU with
// partial pivoting (largest |a|^2, lowest row on ties), row swaps through
// static-index selects; 0 for an exactly singular matrix.
__device__ __forceinline__ double2 small_det4(double2 (&a)[4][4], int r) {
    bool neg = false;
    double2 det = make_double2(1.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c < r) {
            int piv = c;
            double best = cabs2(a[c][c]);
#pragma unroll
            for (int i = c + 1; i < 4; ++i) {
                const double v = cabs2(a[i][c]);
                if (i < r && v > best) {
                    best = v;
                    piv = i;
                }
            }
            if (!(best > 0.0)) return make_double2(0.0, 0.0);
            neg ^= piv != c;
#pragma unroll
            for (int i = c + 1; i < 4; ++i) {
                if (piv == i) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double2 t = a[c][j];
                        a[c][j] = a[i][j];
                        a[i][j] = t;
                    }
                }
            }
            det = c_mul(det, a[c][c]);
            const double inv = 1.0 / best;
            const double2 ui = make_double2(-a[c][c].x * inv, a[c][c].y * inv);
#pragma unroll
            for (int i = c + 1; i < 4; ++i) {
                if (i < r) {
                    const double2 l = c_mul(a[i][c], ui);
#pragma unroll
                    for (int j = c + 1; j < 4; ++j) a[i][j] = c_fma(a[i][j], l, a[c][j]);
                }
            }
        }
    }
    return neg ? make_double2(-det.x, -det.y) : det;
}

// Product over blocks of det S for a pattern whose blocks flip at most 4
// positions each (one lane); pm already relative to the blocks' base
// patterns (shift): sigma = -1 on shift & pm (flipped by the base only);
// code: its lane code (the positions).
// Compact form of a pattern that one lane evaluates (at most 4 flipped
// positions per block), kept in its key slot after classification: bit 63
// set (keys use bits 0..62), block b from bit 27 b: its rank (3 bits), then
// its positions ascending (6 bits each, 0 past the rank).
__device__ __forceinline__ uint64_t lane_code(const uint64_t (&pm)[2]) {
    uint64_t c = 1ull << 63;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        uint64_t mm = pm[b];
        c |= (uint64_t)__popcll(mm) << (27 * b);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (mm) c |= (uint64_t)(__ffsll((long long)mm) - 1) << (27 * b + 3 + 6 * i);
            mm &= mm - 1;
        }
    }
    return c;
}

// The masks of a lane code.
__device__ __forceinline__ void lane_masks(uint64_t c, uint64_t (&pm)[2]) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int r = (int)((c >> (27 * b)) & 7);
        uint64_t m = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i < r) m |= 1ull << ((c >> (27 * b + 3 + 6 * i)) & 63);
        pm[b] = m;
    }
}

template <bool MULTI>
__device__ __forceinline__ double2 gen_det_lane(const DevPlan &p, const GenPlan &g, const GenLds &T, uint64_t code,
                                                const uint64_t (&pm)[2], const uint64_t (&shift)[2]) {
    double2 det = make_double2(1.0, 0.0);
    for (int blk = 0; blk < g.nblk; ++blk) {
        const int r = __popcll(pm[blk]);
        if (r == 0) continue;
        const uint64_t neg = shift[blk] & pm[blk], both = shift[blk] & ~pm[blk];
        const int kb0 = g.kb0[blk];
        const int r0 = __popcll(pm[blk] & (kb0 >= 64 ? ~0ull : ((1ull << kb0) - 1)));
        int pos[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) pos[i] = (int)((code >> (27 * blk + 3 + 6 * i)) & 63);
        const double2 *H = T.H + g.hoff[blk];
        const double2 *R1a = T.R1a + g.r1off[blk];
        double2 a[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a[i][j] = (i < r && j < r)
                              ? (MULTI ? gen_s_entry_multi<4>(H, g.hld[blk], R1a, g.kb[blk], i, pos[i], j, pos)
                                         : gen_s_entry<4>(p.L == 2, H, g.hld[blk], R1a, kb0, i, pos[i], j, r0, pos,
                                                          neg, both))
                              : make_double2(i == j ? 1.0 : 0.0, 0.0);
        det = c_mul(det, small_det4(a, r));
    }
    return det;
}

// Same by a group of GS lanes (row `lane` of S per lane; blocks flip at most
// GS positions each); every lane of the group returns the product.
template <int GS, bool MULTI>
__device__ __forceinline__ double2 gen_det_group(const DevPlan &p, const GenPlan &g, const GenLds &T,
                                                 const uint64_t (&pm)[2], const uint64_t (&shift)[2], int lane,
                                                 double2 *piv) {
    double2 det = make_double2(1.0, 0.0);
    for (int blk = 0; blk < g.nblk; ++blk) {
        const int r = __popcll(pm[blk]);
        if (r == 0) continue;
        const uint64_t neg = shift[blk] & pm[blk], both = shift[blk] & ~pm[blk];
        const int kb0 = g.kb0[blk];
        const int r0 = __popcll(pm[blk] & (kb0 >= 64 ? ~0ull : ((1ull << kb0) - 1)));
        int pos[GS];
        mask_positions<GS>(pm[blk], pos);
        // this lane's row position (the lane-th flipped position), without a
        // dynamically indexed register array
        uint64_t rest = pm[blk];
        for (int q = 0; q < lane && rest; ++q) rest &= rest - 1;
        const int pi = rest ? __ffsll((long long)rest) - 1 : 0;
        const double2 *H = T.H + g.hoff[blk];
        const double2 *R1a = T.R1a + g.r1off[blk];
        double2 a[GS];
        gen_s_row<GS, MULTI>(p.L == 2, H, g.hld[blk], R1a, kb0, g.kb[blk], lane, pi, r, r0, pos, pm[blk], neg, both,
                             a);
        det = c_mul(det, lu_det<GS>(a, r, lane, piv));
    }
    return det;
}

// A pattern's flipped positions relative to the blocks' base patterns
// (the symmetric difference with the base pattern).
__device__ __forceinline__ void gen_relative(const uint16_t *kbt, uint64_t key, const uint64_t (&shift)[2],
                                             uint64_t (&pm)[2]) {
    gen_masks(kbt, key, pm);
#pragma unroll
    for (int b = 0; b < 2; ++b) pm[b] ^= shift[b];
}

// Algorithmic FLOPs of one pattern: per block the r x r elimination, the
// two-layer correction of the layer-1 rows (8 r0 per entry), the product of
// the determinants, and the weight multiply.
__device__ __forceinline__ unsigned long long gen_pattern_flops(const GenPlan &g, bool two_layers,
                                                                const uint64_t (&pm)[2]) {
    unsigned long long f = 8;
    for (int blk = 0; blk < g.nblk; ++blk) {
        const int r = __popcll(pm[blk]);
        if (r == 0) continue;
        const int kb0 = g.kb0[blk];
        const int r0 = __popcll(pm[blk] & (kb0 >= 64 ? ~0ull : ((1ull << kb0) - 1)));
        f += lu_flops(r) + 6 + (g.multi ? 4ull * r * r : (two_layers ? 8ull * (r - r0) * r0 * r : 0ull));
    }
    return f;
}

__device__ __forceinline__ int gen_max_rank(const uint64_t (&pm)[2]) {
    return max(__popcll(pm[0]), __popcll(pm[1]));
}

__device__ __forceinline__ int rank_bin(int r) { return r <= 4 ? 0 : (r <= 8 ? 1 : (r <= 16 ? 2 : (r <= 32 ? 3 : 4))); }

// Evaluates the nl entries in the slots (keys in s.hkey; weights in s.hcnt
// as Gaussian-integer counts, or, with w != nullptr, w[e] for entry e) and
// adds weight * det M_0 * prod det S_N to the bitstring's exact sum.  Entries
// are classified by their largest block rank (counting sort into s.piv) so
// that lanes and lane groups of a pass take like patterns.  Returns false if a
// block flips more than kGenMaxRank positions, or, without BIG (no lane groups
// of 32), more than 16.
template <bool MULTI, bool BIG>
__device__ __forceinline__ bool gen_sum_entries(const DevPlan &p, const GenPlan &g, const GenLds &T, const RawSmem &s,
                                                int nl, const double2 *w, double2 detB, const uint64_t (&shift)[2],
                                                Work &wk, uint64_t *sacc) {
    const int tid = threadIdx.x;
    int *cnt = (int *)s.red;   // [0..4] bins (lane, 8, 16, 32, too large), [8..11] cursors
    uint16_t *order = (uint16_t *)s.piv;
    if (tid < 16) cnt[tid] = 0;
    __syncthreads();
    // each entry's bin is kept in s.list (free until the accumulation), and
    // the key of an entry for one lane is replaced by its lane code
    for (int e = tid; e < nl; e += kThreads) {
        uint64_t pm[2];
        gen_relative(T.kbt, s.hkey[e], shift, pm);
        const int bin = rank_bin(gen_max_rank(pm));
        s.list[e] = (uint16_t)bin;
        if (bin == 0) s.hkey[e] = lane_code(pm);
        atomicAdd(&cnt[bin], 1);
    }
    __syncthreads();
    if (cnt[4] > 0 || (!BIG && cnt[3] > 0)) return false;
    const int n0 = cnt[0], n1 = cnt[1], n2 = cnt[2], n3 = cnt[3];
    __syncthreads();
    if (tid == 0) {
        cnt[8] = 0;
        cnt[9] = n0;
        cnt[10] = n0 + n1;
        cnt[11] = n0 + n1 + n2;
    }
    __syncthreads();
    for (int e = tid; e < nl; e += kThreads) order[atomicAdd(&cnt[8 + s.list[e]], 1)] = (uint16_t)e;
    __syncthreads();
    // value of entry e: weight * detB * prod det S, into its slot (each entry
    // is read and written by the same lane or lane group)
    auto store = [&](int e, double2 dS) {
        const double2 d = c_mul(detB, dS);
        double2 v;
        if (w) {
            v = c_mul(w[e], d);
        } else {
            const int2 c = s.hcnt[e];
            v = make_double2((double)c.x * d.x - (double)c.y * d.y, (double)c.x * d.y + (double)c.y * d.x);
        }
        s.hkey[e] = (uint64_t)__double_as_longlong(v.x);
        *(double *)&s.hcnt[e] = v.y;
    };
    unsigned long long rank = 0, flops = 0;
    for (int i = tid; i < n0; i += kThreads) {
        const int e = order[i];
        const uint64_t code = s.hkey[e];
        uint64_t pm[2];
        lane_masks(code, pm);
        rank += __popcll(pm[0]) + __popcll(pm[1]);
        flops += gen_pattern_flops(g, p.L == 2, pm);
        store(e, gen_det_lane<MULTI>(p, g, T, code, pm, shift));
    }
    {
        const int l8 = tid & 7, g8 = tid >> 3;
        for (int i = n0 + g8; i < n0 + n1; i += kThreads / 8) {
            const int e = order[i];
            uint64_t pm[2];
            gen_relative(T.kbt, s.hkey[e], shift, pm);
            const double2 dS = gen_det_group<8, MULTI>(p, g, T, pm, shift, l8, T.gpiv + g8 * 8);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (l8 == 0) {
                rank += __popcll(pm[0]) + __popcll(pm[1]);
                flops += gen_pattern_flops(g, p.L == 2, pm);
                store(e, dS);
            }
        }
    }
    {
        const int l16 = tid & 15, g16 = tid >> 4;
        for (int i = n0 + n1 + g16; i < n0 + n1 + n2; i += kThreads / 16) {
            const int e = order[i];
            uint64_t pm[2];
            gen_relative(T.kbt, s.hkey[e], shift, pm);
            const double2 dS = gen_det_group<16, MULTI>(p, g, T, pm, shift, l16, T.gpiv + g16 * 16);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (l16 == 0) {
                rank += __popcll(pm[0]) + __popcll(pm[1]);
                flops += gen_pattern_flops(g, p.L == 2, pm);
                store(e, dS);
            }
        }
    }
    if constexpr (BIG) {
        const int l32 = tid & 31, g32 = tid >> 5;
        for (int i = n0 + n1 + n2 + g32; i < n0 + n1 + n2 + n3; i += kThreads / 32) {
            const int e = order[i];
            uint64_t pm[2];
            gen_relative(T.kbt, s.hkey[e], shift, pm);
            const double2 dS = gen_det_group<32, MULTI>(p, g, T, pm, shift, l32, T.gpiv + g32 * 32);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (l32 == 0) {
                rank += __popcll(pm[0]) + __popcll(pm[1]);
                flops += gen_pattern_flops(g, p.L == 2, pm);
                store(e, dS);
            }
        }
    }
    __syncthreads();
    wk.rank += rank;
    wk.flops += flops;
    if (tid == 0) wk.terms += (unsigned)nl;
    // every slot e < nl holds a value: accumulate_slots reads s.list
    for (int e = tid; e < nl; e += kThreads) s.list[e] = (uint16_t)e;
    __syncthreads();
    accumulate_slots(s, nl, sacc);
    return true;
}

__device__ __forceinline__ void write_zero(int64_t b, double *prob, double *amp, double *logp) {
    prob[b] = 0.0;
    if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
    if (logp) logp[b] = -INFINITY;
}

__device__ __forceinline__ void write_result(int64_t b, double2 total, double sc, double *prob, double *amp,
                                             double *logp) {
    const double ax = total.x * sc, ay = total.y * sc;
    const double pb = ax * ax + ay * ay;
    prob[b] = pb;
    if (amp) { amp[2 * b] = ax; amp[2 * b + 1] = ay; }
    if (logp) logp[b] = log(pb);
}

// The evaluation runs in separate kernels per chunk of bitstrings, so that
// the setup (base inverses and the products forming H, long dependent chains
// of small steps) runs at the occupancy its small footprint allows, and the
// pattern evaluation at its own:
//   k_gen_setup_wave: per bitstring (one wave) the blocks' bases M_B, their
//     inverses, X and H; H goes to the bitstring's slot of a workspace
//     (hsize complex entries, the blocks at hoff with row stride hld), det
//     M_B, the base patterns and (Raw Estimate) the outcome to a GenRec.
//   k_gen_setup (retry): the workgroup setup with shifted bases (gen_setup_block)
//     for the bitstrings the first rejected.
//   k_gen_eval: per bitstring, H back into LDS and every distinct pattern's
//     r x r determinant, summed exactly.
// Flags in ecount[i] (Raw Estimate: the sampler's entry count, with the
// setup's outcome in the record until the pattern pass merges it; exact
// mode: written by the setup): kEntryInvalid once p = 0 is written,
// kEntryDeferred for the bitstrings left to k_gen_lu (singular or
// ill-conditioned bases, a pattern beyond kGenMaxRank in a block, or, from
// the sampler, patterns that overflowed the workspace region).
// A bitstring with a pattern of 17..32 flipped positions in a block, left by
// the evaluation without lane groups of 32 to the one with them.
constexpr uint32_t kEntryWide = 0xFFFFFFFCu;

// LDS bytes of k_gen_setup: the setup scratch and the blocks' input columns
// and active modes.
constexpr size_t kGenSetupLds = kGenSetupBytes + 128 + 64;

// Dynamic LDS of k_gen_eval, and the limit of the general kernels' dynamic
// LDS (the static per-bitstring state takes the rest of the 160 KiB).
__host__ __device__ __forceinline__ size_t gen_lds_bytes(const GenPlan &g, bool big) {
    return (big ? gen_base_bytes<2048>() : gen_base_bytes<1024>()) + gen_tables_bytes(g);
}

// The entry slots of the pattern evaluation (the RawSmem fields it uses).
template <int SLOTS>
__device__ __forceinline__ RawSmem carve_eval(unsigned char *smem) {
    RawSmem s{};
    s.hkey = (uint64_t *)smem;
    s.hcnt = (int2 *)(s.hkey + SLOTS);
    s.piv = (double2 *)(s.hcnt + SLOTS);
    s.red = s.piv + kThreads;
    s.list = (uint16_t *)(s.red + kThreads);
    return s;
}
constexpr size_t kGenMaxLds = 150 * 1024;

// A bitstring whose base the one-wave setup did not accept (singular or
// kappa_1 above the bound): the workgroup setup (k_gen_setup, retry mode)
// takes it and tries the shifted bases.  Raw Estimate keeps its entry count
// in its record meanwhile.
constexpr uint32_t kEntryRetry = 0xFFFFFFFBu;
// Exact mode: a bitstring that the prefix-tree kernel (lemma_tree.h) has
// evaluated; the pattern pass skips it.
constexpr uint32_t kEntryTree = 0xFFFFFFFAu;

// Position of the n-th (from 0) set bit of x, which has more than n set bits.
__device__ __forceinline__ int nth_bit64(uint64_t x, int n) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll(x & ((1ull << w) - 1));
        if (n >= c) {
            n -= c;
            x >>= w;
            pos += w;
        }
    }
    return pos;
}

// Maximum over the 32 lanes of a half wave.
__device__ __forceinline__ double half_max(double v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Dynamic LDS of k_gen_setup_wave: each block's base, m_b x m_b complex
// (at least kGenMaxM entries: during the elimination, while the rows are in
// registers, the region's first kGenMaxM entries hold the pivot row).
__host__ __device__ __forceinline__ int gen_setup_wave_region(int mb) {
    return mb * mb > kGenMaxM ? mb * mb : kGenMaxM;
}
__host__ __device__ __forceinline__ size_t gen_setup_wave_lds(const GenPlan &g) {
    size_t e = (size_t)gen_setup_wave_region(g.mb[0]);
    if (g.nblk > 1) e += (size_t)gen_setup_wave_region(g.mb[1]);
    return align16(e * 16);
}

// H = V M_B^-1 U of one block on the matrix cores, one wave: for each
// 16-column tile tn of U, the tiles of X = M_B^-1 U (rows 16 tm ..) are formed
// and, still in the output registers, serve as the B operand of H += V X: the
// FP64 instruction leaves X[16 tm + l / 16 + 4 r][16 tn + l % 16] in element r
// of lane l, which is the B operand of a 4-wide K slice whose lane group
// l / 16 takes row 16 tm + l / 16 + 4 r (FP32: row 16 tm + 4 (l / 16) + r);
// the A operand (V) takes the same K index.  minv(i, k), uop(k, q), vop(q, k)
// return operands, hput(q, q2, v) stores H.
template <bool F32, class FM, class FU, class FV, class FH>
__device__ __forceinline__ void gen_wave_products(int m, int kb, FM minv, FU uop, FV vop, FH hput) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int tiles = (kb + 15) / 16, tm_n = (m + 15) / 16, ns = (m + 3) / 4;
    constexpr int TQ = kGenMaxKb / 16, TM = kGenMaxM / 16;
    typedef typename std::conditional<F32, f4v, d4v>::type acc_t;
    for (int tn = 0; tn < tiles; ++tn) {
        const int col = 16 * tn + li;
        acc_t hr[TQ], hi[TQ];
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq) {
            hr[tq] = acc_t{0, 0, 0, 0};
            hi[tq] = acc_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            if (tm >= tm_n) break;
            const int row = 16 * tm + li;
            acc_t xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
            // the K slices in two groups, each group's operands loaded before its products
            constexpr int SG = kGenMaxSteps / 2;
#pragma unroll
            for (int st0 = 0; st0 < kGenMaxSteps; st0 += SG) {
            if (st0 >= ns) break;
            double2 av[SG], bv[SG];
#pragma unroll
            for (int e = 0; e < SG; ++e) {
                const int st = st0 + e, k = 4 * st + lk;
                av[e] = (st < ns && row < m && k < m) ? minv(row, k) : make_double2(0.0, 0.0);
                bv[e] = (st < ns && k < m && col < kb) ? uop(k, col) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int e = 0; e < SG; ++e) {
                const int st = st0 + e;
                if (st < ns) {
                    if constexpr (F32) {
                        const float ax = (float)av[e].x, ay = (float)av[e].y;
                        const float bx = (float)bv[e].x, by = (float)bv[e].y;
                        xr = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, bx, xr, 0, 0, 0);
                        xr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ay, by, xr, 0, 0, 0);
                        xi = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, by, xi, 0, 0, 0);
                        xi = __builtin_amdgcn_mfma_f32_16x16x4f32(ay, bx, xi, 0, 0, 0);
                    } else {
                        const double2 a = av[e], b = bv[e];
                        xr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, xr, 0, 0, 0);
                        xr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, xr, 0, 0, 0);
                        xi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, xi, 0, 0, 0);
                        xi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, xi, 0, 0, 0);
                    }
                }
            }
            }
#pragma unroll
            for (int tq = 0; tq < TQ; ++tq) {
                if (tq >= tiles) break;
                const int q = 16 * tq + li;
                double2 va[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = F32 ? 16 * tm + 4 * lk + r : 16 * tm + lk + 4 * r;
                    va[r] = (q < kb && k < m) ? vop(q, k) : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // FP64: slice r holds rows 16 tm + 4 r .. 16 tm + 4 r + 3 (none left past m)
                    if (!F32 && 16 * tm + 4 * r >= m) break;
                    if constexpr (F32) {
                        const float ax = (float)va[r].x, ay = (float)va[r].y;
                        hr[tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, xr[r], hr[tq], 0, 0, 0);
                        hr[tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ay, xi[r], hr[tq], 0, 0, 0);
                        hi[tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, xi[r], hi[tq], 0, 0, 0);
                        hi[tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(ay, xr[r], hi[tq], 0, 0, 0);
                    } else {
                        hr[tq] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[r].x, xr[r], hr[tq], 0, 0, 0);
                        hr[tq] = __builtin_amdgcn_mfma_f64_16x16x4f64(-va[r].y, xi[r], hr[tq], 0, 0, 0);
                        hi[tq] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[r].x, xi[r], hi[tq], 0, 0, 0);
                        hi[tq] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[r].y, xr[r], hi[tq], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq) {
            if (tq >= tiles) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 16 * tq + (F32 ? 4 * lk + r : lk + 4 * r);
                if (q < kb && col < kb) hput(q, col, make_double2((double)hr[tq][r], (double)hi[tq][r]));
            }
        }
    }
}

// Setup of the general lemma with one wave per bitstring and no barrier
// between waves: the blocks' bases are inverted at the same time, block b in
// lanes 32 b .. 32 b + 31, by in-place Gauss-Jordan exchange steps in LDS.
// Lane j of a half holds column j of its base; at step c, with pivot row p
// (largest |a_ic|^2 among unused rows, lowest row on ties) and u = a_pc,
//   a_ij += l_i a_pj (j != c),  a_ic = l_i,  l_i = -a_ic / u  (i != p),
//   a_pj = a_pj / u (j != c),   a_pc = 1 / u.
// Rows stay in place; after m steps entry (piv[c], pos[r]) holds M_B^-1[c, r],
// piv[c] the pivot row of step c and pos[r] the step at which row r was the
// pivot.  det M_B is the product of the pivots with the sign of that
// permutation, and the largest column sum of |a| is ||M_B^-1||_1.  A base
// that is singular or has kappa_1 above the bound is left to the workgroup
// setup (kEntryRetry), which tries shifted bases; every other bitstring gets
// H and its record here, as from k_gen_setup.
template <bool EXACT, bool MIXED, bool MULTI>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_gen_setup_wave(DevPlan p, GenPlan g, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb,
                 uint32_t *__restrict__ ecount, double2 *__restrict__ hbuf, GenRec *__restrict__ rec,
                 double *__restrict__ prob, double *__restrict__ amp, double *__restrict__ logp,
                 unsigned long long *nterm) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint8_t sRow[2][kGenMaxM], sPiv[2][kGenMaxM], sPos[2][kGenMaxM];
    __shared__ uint8_t sCol[2][kGenMaxM], sAct[2][kGenMaxKb];
    const int lane = threadIdx.x, hb = lane >> 5, hl = lane & 31;
    for (int e = lane; e < 2 * kGenMaxKb; e += 64) (&sAct[0][0])[e] = g.act[e];
    for (int e = lane; e < 2 * kGenMaxM; e += 64) (&sCol[0][0])[e] = g.col[e];
    const int m0 = g.mb[0], m1 = g.nblk > 1 ? g.mb[1] : 0;
    const int mh = hb ? m1 : m0, mmax = m0 > m1 ? m0 : m1;
    const uint32_t rowmask = mh >= 32 ? 0xFFFFFFFFu : (1u << mh) - 1;
    double2 *base = (double2 *)smem;
    double2 *Ah = base + (hb ? gen_setup_wave_region(m0) : 0);
    // the pivot row of the current step (this half's block), over the base
    // while the rows are in registers
    double2 *prow = Ah;
    const int n = p.n, G = p.G;
    Work wk;
    __syncthreads();
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = b0 + i;
        bool ok = true;
        // weight, range and the rows of each block (as load_bitstring, gen_rows)
        const uint64_t w0 = bits[2 * b], w1 = bits[2 * b + 1];
        ok = ok && (__popcll(w0) + __popcll(w1)) == p.m;
        if (p.n < 128) {
            const uint64_t hi0 = p.n >= 64 ? 0ull : (~0ull << p.n);
            const uint64_t hi1 = p.n <= 64 ? ~0ull : (~0ull << (p.n - 64));
            ok = ok && !(w0 & hi0) && !(w1 & hi1);
        }
        const uint64_t x0 = hb ? (w0 & g.bmask[1][0]) : (w0 & ~g.bmask[1][0]);
        const uint64_t x1 = hb ? (w1 & g.bmask[1][1]) : (w1 & ~g.bmask[1][1]);
        const int c0 = __popcll(x0);
        // every half (a missing second block has no rows) must hold its block's count
        ok = ok && c0 + __popcll(x1) == mh;
        if (__ballot(!ok) != 0) {
            if (lane == 0) {
                write_zero(b, prob, amp, logp);
                if constexpr (EXACT) ecount[i] = kEntryInvalid;
                else rec[i].status = kRecZero;
            }
            continue;
        }
        if (hl < mh) sRow[hb][hl] = (uint8_t)(hl < c0 ? nth_bit64(x0, hl) : 64 + nth_bit64(x1, hl - c0));
        __syncthreads();
        // the base, column hl of this half's block, and ||M_B||_1
        double csum = 0.0;
        if (hl < mh) {
            // eight loads in flight before their stores
            const double2 *Pc = p.P + sCol[hb][hl];
            int r = 0;
            for (; r + 8 <= mh; r += 8) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = Pc[(size_t)sRow[hb][r + u] * G];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    Ah[(r + u) * mh + hl] = v[u];
                    csum += sqrt(cabs2(v[u]));
                }
            }
            for (; r < mh; ++r) {
                const double2 v = Pc[(size_t)sRow[hb][r] * G];
                Ah[r * mh + hl] = v;
                csum += sqrt(cabs2(v));
            }
        }
        const double norm = half_max(csum);
        __syncthreads();
        // Gauss-Jordan with each lane's row in registers: a[] holds row hl in
        // a physical column order that rotates left by 4 after every 4 steps,
        // so that the pivot column of step 4 q + t is always a[t] (static
        // register indices); the pivot row goes through LDS (prow).
        static_assert(kGenMaxM == 32, "the column rotation works modulo 32 in steps of 4");
        double2 a[kGenMaxM];
#pragma unroll
        for (int j = 0; j < kGenMaxM; ++j) a[j] = (hl < mh && j < mh) ? Ah[hl * mh + j] : make_double2(0.0, 0.0);
        uint32_t used = 0;
        unsigned inversions = 0;
        double2 det = make_double2(1.0, 0.0);
        bool singular = false;
        const int nchunk = (mmax + 3) / 4;
        for (int q = 0; q < nchunk; ++q) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * q + t;   // logical column (physical t)
                if (c >= mmax) break;
                const bool live = c < mh && !singular;
                const double2 ac = a[t];
                double best = (live && hl < mh && !((used >> hl) & 1)) ? cabs2(ac) : -1.0;
                int idx = hl;
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) {
                    const double vo = __shfl_xor(best, off, 64);
                    const int io = __shfl_xor(idx, off, 64);
                    if (vo > best || (vo == best && io < idx)) {
                        best = vo;
                        idx = io;
                    }
                }
                if (live && !(best > 0.0)) singular = true;
                const bool go = live && best > 0.0;
                const bool piv = go && hl == idx;
                if (piv) {
#pragma unroll
                    for (int j = 0; j < kGenMaxM; ++j) prow[j] = a[j];
                }
                __syncthreads();
                if (go) {
                    const double2 u = prow[t];
                    const double inv = 1.0 / best;
                    const double2 ui = make_double2(u.x * inv, -u.y * inv);
                    inversions += __popc(~used & ((1u << idx) - 1) & rowmask);
                    used |= 1u << idx;
                    det = c_mul(det, u);
                    if (hl == 0) {
                        sPiv[hb][c] = (uint8_t)idx;
                        sPos[hb][idx] = (uint8_t)c;
                    }
                    // exchange step: a_ij += l_i a_pj with l_i = -a_ic / u; the
                    // pivot row takes l = 1 / u - 1 (a_pj / u); column c then
                    // holds l_i, and 1 / u in the pivot row
                    const double2 l = piv ? make_double2(ui.x - 1.0, ui.y)
                                          : make_double2(-(ac.x * ui.x - ac.y * ui.y), -(ac.x * ui.y + ac.y * ui.x));
                    // in groups of 8 columns, so that the pivot-row reads of
                    // one group are in registers at a time
#pragma unroll
                    for (int j0 = 0; j0 < kGenMaxM; j0 += 8) {
#pragma unroll
                        for (int j = j0; j < j0 + 8; ++j) a[j] = c_fma(a[j], l, prow[j]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    a[t] = piv ? ui : l;
                }
                __syncthreads();
            }
            // rotate: physical column j takes j + 4
            const double2 r0 = a[0], r1 = a[1], r2 = a[2], r3 = a[3];
#pragma unroll
            for (int j = 0; j < kGenMaxM - 4; ++j) a[j] = a[j + 4];
            a[kGenMaxM - 4] = r0;
            a[kGenMaxM - 3] = r1;
            a[kGenMaxM - 2] = r2;
            a[kGenMaxM - 1] = r3;
        }
        // back to LDS in logical column order: physical j is logical (j + 4 nchunk) mod 32
        {
            const int off = (4 * nchunk) & (kGenMaxM - 1);
#pragma unroll
            for (int j = 0; j < kGenMaxM; ++j) {
                const int lc = (j + off) & (kGenMaxM - 1);
                if (hl < mh && lc < mh) Ah[hl * mh + lc] = a[j];
            }
        }
        __syncthreads();
        // kappa_1 from the column sums of |M_B^-1| (a permutation of its columns)
        double cs = 0.0;
        if (!singular && hl < mh)
            for (int r = 0; r < mh; ++r) cs += sqrt(cabs2(Ah[r * mh + hl]));
        const double kappa = half_max(cs) * norm;
        const bool good = !singular && kappa <= kLemmaMaxCond;
        if (__ballot(!good) != 0) {
            if (lane == 0) {
                if constexpr (EXACT) ecount[i] = kEntryRetry;
                else rec[i].status = kRecRetry;
                if (nterm) atomicAdd(nterm + 5, 1ull);
            }
            __syncthreads();
            continue;
        }
        if (inversions & 1) det = make_double2(-det.x, -det.y);
        const double2 d1 = read_lane_c(det, 32);
        det = c_mul(read_lane_c(det, 0), d1);
        const double kap[2] = {read_lane_d(kappa, 0), read_lane_d(kappa, 32)};
        // X and H of each block on the matrix cores, written to the bitstring's slot
        double2 *Hb = hbuf + (size_t)i * g.hsize;
        for (int blk = 0; blk < g.nblk; ++blk) {
            const int m = g.mb[blk], kb = g.kb[blk], kb0 = g.kb0[blk], hld = g.hld[blk];
            const double2 *Ab = base + (blk ? gen_setup_wave_region(m0) : 0);
            const uint8_t *piv = sPiv[blk], *pos = sPos[blk], *rows = sRow[blk], *col = sCol[blk], *act = sAct[blk];
            double2 *H = Hb + g.hoff[blk];
            auto minv = [&](int r, int k) { return Ab[piv[r] * m + pos[k]]; };
            auto hput = [&](int q, int q2, double2 v) { H[q * hld + q2] = v; };
            const bool f32 = MIXED && kap[blk] <= p.mixed_cond;
            if constexpr (MULTI) {
                const double2 *GA = g.GA + (size_t)blk * n * 64, *HC = g.HC + (size_t)blk * 64 * G;
                auto uop = [&](int k, int q) { return GA[(size_t)rows[k] * 64 + q]; };
                auto vop = [&](int q, int k) { return HC[(size_t)q * G + col[k]]; };
                if (f32) gen_wave_products<true>(m, kb, minv, uop, vop, hput);
                else gen_wave_products<false>(m, kb, minv, uop, vop, hput);
            } else {
                const double2 *A1 = p.A1, *A2 = p.A2, *Phi0 = p.Phi0, *Q = p.Q;
                auto uop = [&](int k, int q) { return (q < kb0 ? A1 : A2)[(size_t)rows[k] * n + act[q]]; };
                auto vop = [&](int q, int k) { return (q < kb0 ? Phi0 : Q)[(size_t)act[q] * G + col[k]]; };
                if (f32) gen_wave_products<true>(m, kb, minv, uop, vop, hput);
                else gen_wave_products<false>(m, kb, minv, uop, vop, hput);
            }
            if (lane == 0) {
                // m exchange steps of (m - 1) x m complex multiply-adds, the
                // multipliers, the pivot row and the pivot search; the
                // conditioning; X and H
                wk.flops += (unsigned long long)m * (8ull * (m - 1) * m + 6ull * (m - 1) + 6ull * m + 4ull * m) +
                            4ull * m * m + 8ull * m * m * kb + 8ull * kb * m * kb;
                if (f32) ++wk.fp32;
            }
        }
        if (lane == 0) {
            GenRec r;
            r.det = det;
            r.shift[0] = r.shift[1] = 0;
            r.count = 0;
            r.status = kRecOk;
            r.pad[0] = r.pad[1] = 0;
            rec[i] = r;
            if constexpr (EXACT) ecount[i] = 0;
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

template <bool EXACT, bool MIXED, bool MULTI>
__global__ void __launch_bounds__(kThreads, 2)
k_gen_setup(DevPlan p, GenPlan g, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb,
            uint32_t *__restrict__ ecount, double2 *__restrict__ hbuf, GenRec *__restrict__ rec,
            double *__restrict__ prob, double *__restrict__ amp, double *__restrict__ logp,
            unsigned long long *nterm, int retry) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok;
    __shared__ GenShared sh;
    __shared__ uint8_t s_Rb[128];
    const int tid = threadIdx.x;
    if (retry && nterm && *(volatile unsigned long long *)(nterm + 5) == 0) return;   // none left
    GenLds T;
    T.act = smem + kGenSetupBytes;
    T.col = T.act + 128;
    T.kbt = nullptr;
    T.R1a = T.gpiv = nullptr;
    for (int e = tid; e < 2 * kGenMaxKb; e += kThreads) T.act[e] = g.act[e];
    for (int e = tid; e < 2 * kGenMaxM; e += kThreads) T.col[e] = g.col[e];
    __syncthreads();
    Work wk;
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = b0 + i;
        bool zero = false;
        if (retry) {
            // only the bitstrings the one-wave setup left
            if (EXACT ? ecount[i] != kEntryRetry : rec[i].status != kRecRetry) continue;
        }
        if (!zero) zero = !load_bitstring(p, bits, b, s_Rb, &s_ok);
        if (!zero) {
            gen_rows(p, g, s_Rb, sh);
            __syncthreads();
            zero = sh.ok == 0;
            __syncthreads();
        }
        if (zero) {
            if (tid == 0) {
                write_zero(b, prob, amp, logp);
                if constexpr (EXACT) ecount[i] = kEntryInvalid;
                else rec[i].status = kRecZero;
            }
            __syncthreads();
            continue;
        }
        T.H = hbuf + (size_t)i * g.hsize;
        bool ok = true;
        for (int blk = 0; blk < g.nblk && ok; ++blk)
            ok = gen_setup_block<MIXED, MULTI>(p, g, T, blk, smem, sh, wk);
        if (tid == 0) {
            if (ok) {
                GenRec r;
                r.det = sh.det;
                r.shift[0] = sh.shift[0];
                r.shift[1] = sh.shift[1];
                r.count = 0;
                r.status = kRecOk;
                r.pad[0] = r.pad[1] = 0;
                rec[i] = r;
                if constexpr (EXACT) ecount[i] = 0;
            } else {
                if constexpr (EXACT) ecount[i] = kEntryDeferred;
                else rec[i].status = kRecDeferred;
            }
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

// BIG: lane groups of 32 for patterns of 17..32 flipped positions in a block;
// without, such bitstrings get kEntryWide (and keep their entries) for a
// second pass with.  WIDE_ONLY: that second pass, over the kEntryWide ones.
template <bool EXACT, bool MULTI, bool BIG, bool WIDE_ONLY>
__global__ void __launch_bounds__(kThreads, 1)
k_gen_eval(DevPlan p, GenPlan g, int64_t b0, int64_t nb, const uint64_t *__restrict__ ekey,
           const int2 *__restrict__ ecnt, uint32_t *__restrict__ ecount, uint64_t cap,
           const uint64_t *__restrict__ xkeys, const double2 *__restrict__ xw, int64_t nkeys,
           const double2 *__restrict__ hbuf, GenRec *__restrict__ rec, double *__restrict__ prob,
           double *__restrict__ amp, double *__restrict__ logp, unsigned long long *nterm, int nseg,
           uint64_t *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t s_acc[kAccWords];
    constexpr int SLOTS = BIG ? 2048 : 1024;
    if (WIDE_ONLY && nterm && *(volatile unsigned long long *)(nterm + 6) == 0) return;   // none left
    const RawSmem s = carve_eval<SLOTS>(smem);
    const GenLds T = carve_gen<SLOTS>(smem, g);
    const int tid = threadIdx.x;
    Work wk;
    load_gen_tables(p, g, T);
    // exact mode may split each bitstring's term list into nseg segments
    // (multiples of 256 terms; work items i * nseg + j), whose exact partial
    // sums k_gen_reduce_segments adds; otherwise one item per bitstring
    const int64_t seglen = EXACT ? (((nkeys + nseg - 1) / nseg + 255) / 256) * 256 : 0;
    for (int64_t item = blockIdx.x; item < nb * (int64_t)nseg; item += gridDim.x) {
        const int64_t i = item / nseg, j = item % nseg;
        const int64_t b = b0 + i;
        const uint32_t flag = ecount[i];
        if (WIDE_ONLY ? flag != kEntryWide
                      : (flag == kEntryDeferred || flag == kEntryInvalid || flag == kEntryWide || flag == kEntryTree))
            continue;
        if (!EXACT && !WIDE_ONLY) {
            // the setup's outcome: p = 0 already written, or no acceptable base (to k_gen_lu)
            const uint32_t st = rec[i].status;
            if (st == kRecZero) continue;
            if (st == kRecDeferred) {
                if (tid == 0) ecount[i] = kEntryDeferred;
                continue;
            }
        }
        const double2 detB = rec[i].det;
        const uint64_t shift[2] = {rec[i].shift[0], rec[i].shift[1]};
        const double2 *Hg = hbuf + (size_t)i * g.hsize;
        {
            // eight loads in flight before their stores
            int e = tid;
            for (; e + 7 * kThreads < g.hsize; e += 8 * kThreads) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = Hg[e + u * kThreads];
#pragma unroll
                for (int u = 0; u < 8; ++u) T.H[e + u * kThreads] = v[u];
            }
            for (; e < g.hsize; e += kThreads) T.H[e] = Hg[e];
        }
        acc_clear(s_acc);
        __syncthreads();
        const int64_t lo = EXACT ? j * seglen : 0;
        const int64_t nent = EXACT ? min(nkeys, lo + seglen) : (int64_t)(WIDE_ONLY ? rec[i].count : flag);
        bool ok = true;
        for (int64_t c0 = lo; ok && c0 < nent; c0 += SLOTS) {
            const int nc = (int)min((int64_t)SLOTS, nent - c0);
            int e = tid;
            if constexpr (!EXACT) {
                // four entries in flight before their stores
                const uint64_t *kin = ekey + (size_t)i * cap + c0;
                const int2 *cin = ecnt + (size_t)i * cap + c0;
                for (; e + 3 * kThreads < nc; e += 4 * kThreads) {
                    uint64_t kv[4];
                    int2 cv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        kv[u] = kin[e + u * kThreads];
                        cv[u] = cin[e + u * kThreads];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        s.hkey[e + u * kThreads] = kv[u];
                        s.hcnt[e + u * kThreads] = cv[u];
                    }
                }
            }
            for (; e < nc; e += kThreads) {
                if constexpr (EXACT) {
                    s.hkey[e] = xkeys[c0 + e];
                } else {
                    s.hkey[e] = ekey[(size_t)i * cap + c0 + e];
                    s.hcnt[e] = ecnt[(size_t)i * cap + c0 + e];
                }
            }
            __syncthreads();
            ok = gen_sum_entries<MULTI, BIG>(p, g, T, s, nc, EXACT ? xw + c0 : nullptr, detB, shift, wk, s_acc);
        }
        if (!ok) {
            if (tid == 0) {
                if (!BIG && !EXACT) rec[i].count = flag;   // for the pass with lane groups of 32
                ecount[i] = BIG ? kEntryDeferred : kEntryWide;
                if (!BIG && nterm) atomicAdd(nterm + 6, 1ull);
            }
            __syncthreads();
            continue;
        }
        if (nseg > 1) {
            if (tid < kAccWords) part[(size_t)item * 8 + tid] = s_acc[tid];
        } else {
            const double2 total = acc_value(s_acc);
            if (tid == 0) write_result(b, total, EXACT ? 1.0 : p.scale, prob, amp, logp);
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

// The sum of a bitstring's segment partials (in segment order; the words are
// exact integers, so the order does not change the result) for the
// bitstrings whose flag is `want` (0: evaluated by k_gen_eval; kEntryDeferred:
// by k_gen_lu).  One thread per bitstring.
__global__ void k_gen_reduce_segments(int64_t nb, int nseg, const uint32_t *__restrict__ flags, uint32_t want,
                                      const uint64_t *__restrict__ part, double *__restrict__ prob,
                                      double *__restrict__ amp, double *__restrict__ logp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || flags[i] != want) return;
    Fix192 R, I;
    uint64_t bad = 0;
    for (int j = 0; j < nseg; ++j) {
        const uint64_t *q = part + ((size_t)i * nseg + j) * 8;
        fix_add(R, q[0], q[1], (int64_t)q[2]);
        fix_add(I, q[3], q[4], (int64_t)q[5]);
        bad |= q[6];
    }
    uint64_t acc[kAccWords] = {R.w0, R.w1, (uint64_t)R.w2, I.w0, I.w1, (uint64_t)I.w2, bad};
    write_result(i, acc_value(acc), 1.0, prob, amp, logp);
}

// ---------------------------------------------------------------------------
// Fallback for the bitstrings the general evaluation left (flag
// kEntryDeferred): every pattern's submatrix M_N is factorised directly,
// block by block, by lane groups of 32 (one row of the block per lane),
// composing the rows from the low-rank form of Sec. IV-B Eq. 19 (two-layer
// form for two CPhase layers) restricted to the block.  Raw Estimate samples
// the bitstring again with its LDS hash.
// ---------------------------------------------------------------------------

// Row i (mode Ri) of block blk of M_N over the block's columns, from global
// memory; lanes >= m give identity rows.
__device__ __forceinline__ void gen_lu_row(const DevPlan &p, const GenPlan &g, const GenShared &sh, const Flips &f,
                                           int blk, int lane, double2 (&a)[32]) {
    const int m = g.mb[blk], n = p.n, G = p.G;
    const uint8_t *col = g.col + blk * kGenMaxM;
#pragma unroll
    for (int j = 0; j < 32; ++j) a[j] = make_double2(j == lane ? 1.0 : 0.0, 0.0);
    if (lane >= m) return;
    const int Ri = sh.rows[blk][lane];
    const size_t rn = (size_t)Ri * n;
#pragma unroll
    for (int j = 0; j < 32; ++j)
        if (j < m) a[j] = p.P[(size_t)Ri * G + col[j]];
    const uint64_t n0[2] = {f.n0[0] & g.bmask[blk][0], f.n0[1] & g.bmask[blk][1]};
    const uint64_t n1[2] = {f.n1[0] & g.bmask[blk][0], f.n1[1] & g.bmask[blk][1]};
    for (int w0 = 0; w0 < 2; ++w0)
        for (uint64_t mm = n0[w0]; mm; mm &= mm - 1) {
            const int c = 64 * w0 + __ffsll((long long)mm) - 1;
            double2 al = p.A1[rn + c];
            if (p.L == 2) {
                for (int w1 = 0; w1 < 2; ++w1)
                    for (uint64_t qq = n1[w1]; qq; qq &= qq - 1) {
                        const int q = 64 * w1 + __ffsll((long long)qq) - 1;
                        const double2 t = p.A2[rn + q], r = p.R1[(size_t)q * n + c];
                        al = c_fma(al, make_double2(-2.0 * t.x, -2.0 * t.y), r);
                    }
            }
            const double2 s2 = make_double2(-2.0 * al.x, -2.0 * al.y);
            const double2 *phi = p.Phi0 + (size_t)c * G;
#pragma unroll
            for (int j = 0; j < 32; ++j)
                if (j < m) a[j] = c_fma(a[j], s2, phi[col[j]]);
        }
    if (p.L == 2) {
        for (int w1 = 0; w1 < 2; ++w1)
            for (uint64_t qq = n1[w1]; qq; qq &= qq - 1) {
                const int q = 64 * w1 + __ffsll((long long)qq) - 1;
                const double2 t = p.A2[rn + q];
                const double2 s2 = make_double2(-2.0 * t.x, -2.0 * t.y);
                const double2 *qrow = p.Q + (size_t)q * G;
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    if (j < m) a[j] = c_fma(a[j], s2, qrow[col[j]]);
            }
    }
}

// Slot values (weight * det M_N) of the nl entries whose slots are list[e]
// (keys in s.hkey, counts in s.hcnt, or exact weights w[e] with list[e] = e),
// then their exact sum.
__device__ __forceinline__ void gen_lu_entries(const DevPlan &p, const GenPlan &g, const GenShared &sh,
                                               const RawSmem &s, int nl, const double2 *w, Work &wk,
                                               uint64_t *sacc) {
    const int tid = threadIdx.x, lane = tid & 31, grp = tid >> 5;
    for (int e = grp; e < nl; e += kThreads / 32) {
        const uint16_t slot = s.list[e];
        const Flips f = decode_key(p, s.hkey[slot]);
        double2 det = make_double2(1.0, 0.0);
        for (int blk = 0; blk < g.nblk; ++blk) {
            double2 a[32];
            gen_lu_row(p, g, sh, f, blk, lane, a);
            det = c_mul(det, lu_det<32>(a, g.mb[blk], lane, s.piv + grp * 32));
        }
        if (lane == 0) {
            double2 v;
            if (w) {
                v = c_mul(w[e], det);
            } else {
                const int2 c = s.hcnt[slot];
                v = make_double2((double)c.x * det.x - (double)c.y * det.y, (double)c.x * det.y + (double)c.y * det.x);
            }
            s.hkey[slot] = (uint64_t)__double_as_longlong(v.x);
            *(double *)&s.hcnt[slot] = v.y;
            wk.terms += 1;
            for (int blk = 0; blk < g.nblk; ++blk) wk.flops += lu_flops(g.mb[blk]);
        }
    }
    __syncthreads();
    accumulate_slots(s, nl, sacc);
}

// Bytes of LDS the fallback adds for circuits with more than two CPhase
// layers: Y (64 x 32) and one submatrix (32 x 32).
constexpr size_t kGenMultiLuBytes = (size_t)(64 * 32 + 32 * 32) * 16;

// The same for circuits with more than two CPhase layers: the whole
// workgroup composes one pattern's submatrix at a time from
//   M_N = M_0 - 2 GA[R, N] Y,  (I + 2 TT[N, N]) Y = HC[N, cols]
// (Y by forward substitution in layer order, I + 2 TT being unit lower
// triangular), then a lane group of 32 factorises it.
__device__ __forceinline__ void gen_lu_entries_multi(const DevPlan &p, const GenPlan &g, const GenShared &sh,
                                                     const RawSmem &s, int nl, const double2 *w, Work &wk,
                                                     uint64_t *sacc, double2 *Y, double2 *M) {
    const int tid = threadIdx.x, n = p.n, G = p.G;
    __shared__ double2 s_det;
    for (int e = 0; e < nl; ++e) {
        const uint16_t slot = s.list[e];
        uint64_t pm[2];
        gen_masks(g.kbt, s.hkey[slot], pm);
        if (tid == 0) s_det = make_double2(1.0, 0.0);
        for (int blk = 0; blk < g.nblk; ++blk) {
            const int m = g.mb[blk], r = __popcll(pm[blk]);
            const double2 *GA = g.GA + (size_t)blk * n * 64, *HC = g.HC + (size_t)blk * 64 * G;
            const double2 *TT = g.TT + (size_t)blk * 64 * 64;
            const uint8_t *col = g.col + blk * kGenMaxM;
            // Y: lane c of wave 0 solves column c
            if (tid < m) {
                int f = 0;
                for (uint64_t mm = pm[blk]; mm; mm &= mm - 1, ++f) {
                    const int q = __ffsll((long long)mm) - 1;
                    double2 y = HC[(size_t)q * G + col[tid]];
                    int f2 = 0;
                    for (uint64_t m2 = pm[blk] & ((1ull << q) - 1); m2; m2 &= m2 - 1, ++f2) {
                        const int q2 = __ffsll((long long)m2) - 1;
                        const double2 tt = TT[(size_t)q * 64 + q2];
                        y = c_fma(y, make_double2(-2.0 * tt.x, -2.0 * tt.y), Y[f2 * 32 + tid]);
                    }
                    Y[f * 32 + tid] = y;
                }
            }
            __syncthreads();
            for (int ij = tid; ij < m * m; ij += kThreads) {
                const int i = ij / m, c = ij % m;
                const int Ri = sh.rows[blk][i];
                double2 v = p.P[(size_t)Ri * G + col[c]];
                int f = 0;
                for (uint64_t mm = pm[blk]; mm; mm &= mm - 1, ++f) {
                    const int q = __ffsll((long long)mm) - 1;
                    const double2 ga = GA[(size_t)Ri * 64 + q];
                    v = c_fma(v, make_double2(-2.0 * ga.x, -2.0 * ga.y), Y[f * 32 + c]);
                }
                M[i * 32 + c] = v;
            }
            __syncthreads();
            if (tid < 32) {
                double2 a[32];
#pragma unroll
                for (int j = 0; j < 32; ++j)
                    a[j] = (tid < m && j < m) ? M[tid * 32 + j] : make_double2(j == tid ? 1.0 : 0.0, 0.0);
                const double2 d = lu_det<32>(a, m, tid, s.piv);
                if (tid == 0) {
                    s_det = c_mul(s_det, d);
                    wk.flops += lu_flops(m) + 8ull * m * m * r + 8ull * r * r * m / 2;
                }
            }
            __syncthreads();
            (void)r;
        }
        if (tid == 0) {
            const double2 det = s_det;
            double2 v;
            if (w) {
                v = c_mul(w[e], det);
            } else {
                const int2 c = s.hcnt[slot];
                v = make_double2((double)c.x * det.x - (double)c.y * det.y, (double)c.x * det.y + (double)c.y * det.x);
            }
            s.hkey[slot] = (uint64_t)__double_as_longlong(v.x);
            *(double *)&s.hcnt[slot] = v.y;
            wk.terms += 1;
        }
        __syncthreads();
    }
    accumulate_slots(s, nl, sacc);
}

template <bool EXACT>
__global__ void __launch_bounds__(kThreads, 1)
k_gen_lu(DevPlan p, GenPlan g, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb, uint32_t t, uint64_t seed,
         const uint32_t *__restrict__ flags, const uint64_t *__restrict__ xkeys, const double2 *__restrict__ xw,
         int64_t nkeys, double *__restrict__ prob, double *__restrict__ amp, double *__restrict__ logp,
         unsigned long long *nterm, int nseg, uint64_t *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_n;
    __shared__ int s_cnt[6];
    __shared__ GenShared sh;
    __shared__ uint64_t s_acc[kAccWords];
    const RawSmem s = carve_raw(smem, EXACT ? 0 : p.k, p.n, 4, false);
    double2 *Ym = (double2 *)(smem + raw_lds_bytes(EXACT ? 0 : p.k, p.n, 4, false, false));
    double2 *Mm = Ym + 64 * 32;
    const int tid = threadIdx.x;
    Work wk;
    bool loaded = false;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t slot0 = hash_slot(0);
    // exact mode: segments of the term list as in k_gen_eval (nseg = 1 under
    // Raw Estimate)
    const int64_t seglen = EXACT ? (((nkeys + nseg - 1) / nseg + 255) / 256) * 256 : 0;
    for (int64_t item = blockIdx.x; item < nb * (int64_t)nseg; item += gridDim.x) {
        const int64_t i = item / nseg, j = item % nseg;
        if (flags[i] != kEntryDeferred) continue;
        const int64_t b = b0 + i;
        if (!EXACT && !loaded) {
            load_tables(p, s);
            loaded = true;
        }
        bool zero = !load_bitstring(p, bits, b, s.Rb, &s_ok);
        if (!zero) {
            gen_rows(p, g, s.Rb, sh);
            __syncthreads();
            zero = sh.ok == 0;
            __syncthreads();
        }
        if (zero) {
            if (tid == 0) {
                if (nseg > 1) {
                    for (int w = 0; w < 8; ++w) part[(size_t)item * 8 + w] = 0;
                } else {
                    write_zero(b, prob, amp, logp);
                }
            }
            __syncthreads();
            continue;
        }
        acc_clear(s_acc);
        if constexpr (EXACT) {
            const int64_t hi = min(nkeys, j * seglen + seglen);
            for (int64_t c0 = j * seglen; c0 < hi; c0 += kHashSlots) {
                const int nc = (int)min((int64_t)kHashSlots, hi - c0);
                __syncthreads();
                for (int e = tid; e < nc; e += kThreads) {
                    s.hkey[e] = xkeys[c0 + e];
                    s.list[e] = (uint16_t)e;
                }
                __syncthreads();
                if (g.multi)
                    gen_lu_entries_multi(p, g, sh, s, nc, xw + c0, wk, s_acc, Ym, Mm);
                else
                    gen_lu_entries(p, g, sh, s, nc, xw + c0, wk, s_acc);
            }
        } else {
            Sampler st;
            unsigned long long blocks = 0;   // not reported here
            clear_table(s, s_cnt, slot0, st);
            while (true) {
                const bool done = sample_until_flush(p, s, s_cnt, slot0, b, t, k0, k1, st, blocks);
                const int nl = gather_list(s, &s_n);
                if (g.multi)
                    gen_lu_entries_multi(p, g, sh, s, nl, nullptr, wk, s_acc, Ym, Mm);
                else
                    gen_lu_entries(p, g, sh, s, nl, nullptr, wk, s_acc);
                if (done) break;
                clear_table(s, s_cnt, slot0, st);
            }
        }
        if (nseg > 1) {
            if (tid < kAccWords) part[(size_t)item * 8 + tid] = s_acc[tid];
        } else {
            const double2 total = acc_value(s_acc);
            if (tid == 0) write_result(b, total, EXACT ? 1.0 : p.scale, prob, amp, logp);
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

}  // namespace
}  // namespace xf
