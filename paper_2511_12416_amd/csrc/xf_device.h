// Device-side building blocks shared by the gfx950 kernels of the Born-rule
// probability path: complex FP64 helpers, Philox4x32-10, the per-bitstring LDS
// layout, the trajectory sampler with its pattern hash, the register LU and
// Gauss-Jordan of a lane group, the exact fixed-point accumulator and the
// per-bitstring determinant-lemma setup.  Everything here is inline; each
// kernel translation unit includes it.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "xf_internal.h"

namespace xf {
namespace {

__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ double2 c_fma(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ float2 c_fmaf(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}

// Philox4x32-10: ten rounds of two 32x32->64 multiplies (multipliers
// 0xD2511F53, 0xCD9E8D57) with the key advanced by the Weyl constants
// (0x9E3779B9, 0xBB67AE85) between rounds (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply each (v_mad_u64_u32) instead of
        // separate low and high halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        // three-input XORs as one v_bitop3_b32 each (truth table 0x96)
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Slot of a key in an LDS hash table: the key folded to 32 bits (high word
// rotated by 16), then a multiplicative (Fibonacci) hash, top bits.
__device__ __forceinline__ uint32_t hash_slot(uint64_t key) {
    static_assert(kHashSlots == 2048, "11 hash bits");
    const uint32_t hi = (uint32_t)(key >> 32);
    const uint32_t x = (uint32_t)key ^ ((hi << 16) | (hi >> 16));
    return (x * 0x9E3779B1u) >> 21;
}

// Flip masks (per CPhase layer, 128-bit mode sets) of a trajectory key.
struct Flips {
    uint64_t n0[2], n1[2];
};

__device__ __forceinline__ void flip_mode(uint64_t &lo, uint64_t &hi, int q) {
    if (q < 64) lo ^= 1ull << q;
    else hi ^= 1ull << (q - 64);
}

__device__ __forceinline__ Flips decode_key(const DevPlan &p, uint64_t key) {
    Flips f = {{0, 0}, {0, 0}};
    uint64_t mm = key;
    if (p.keykind == 0) {
        while (mm) {
            const int pos = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            const int q = p.keymode[pos];
            if (pos < p.off1) flip_mode(f.n0[0], f.n0[1], q);
            else flip_mode(f.n1[0], f.n1[1], q);
        }
    } else {
        while (mm) {
            const int j = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            const uint64_t g0 = p.gmode[2 * j], g1 = p.gmode[2 * j + 1];
            if (p.glayer[j] == 0) { f.n0[0] ^= g0; f.n0[1] ^= g1; }
            else { f.n1[0] ^= g0; f.n1[1] ^= g1; }
        }
    }
    return f;
}

template <typename F>
__device__ __forceinline__ void for_each_mode(const uint64_t (&s)[2], F f) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        uint64_t mm = s[w];
        while (mm) {
            const int q = 64 * w + __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            f(q);
        }
    }
}

// Row i (mode Ri) of the trajectory submatrix M = V(x)[R, C]: P[Ri,:] minus
// twice the low-rank correction.  FP64 accumulates straight into the row;
// MIXED forms the correction in FP32 and adds it to the FP64 base row.
template <int G, bool MIXED>
__device__ __forceinline__ void compose_row(const DevPlan &p, int Ri, const Flips &f, double2 (&a)[G]) {
    const size_t rn = (size_t)Ri * p.n;
    const double2 *prow = p.P + (size_t)Ri * G;
    if constexpr (!MIXED) {
#pragma unroll
        for (int j = 0; j < G; ++j) a[j] = prow[j];
        auto axpy = [&](double2 al, const double2 *row) {
            const double2 s2 = make_double2(-2.0 * al.x, -2.0 * al.y);
#pragma unroll
            for (int j = 0; j < G; ++j) a[j] = c_fma(a[j], s2, row[j]);
        };
        if (p.L == 1) {
            for_each_mode(f.n0, [&](int c) { axpy(p.A1[rn + c], p.Phi0 + (size_t)c * G); });
        } else if (p.L == 2) {
            for_each_mode(f.n0, [&](int c) {
                double2 al = p.A1[rn + c];
                for_each_mode(f.n1, [&](int q) {
                    const double2 t = p.A2[rn + q], r = p.R1[(size_t)q * p.n + c];
                    al = c_fma(al, make_double2(-2.0 * t.x, -2.0 * t.y), r);
                });
                axpy(al, p.Phi0 + (size_t)c * G);
            });
            for_each_mode(f.n1, [&](int q) { axpy(p.A2[rn + q], p.Q + (size_t)q * G); });
        }
    } else {
        float2 acc[G];
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] = make_float2(0.f, 0.f);
        auto axpy = [&](float2 al, const float2 *row) {
#pragma unroll
            for (int j = 0; j < G; ++j) acc[j] = c_fmaf(acc[j], al, row[j]);
        };
        if (p.L == 1) {
            for_each_mode(f.n0, [&](int c) { axpy(p.fA1[rn + c], p.fPhi0 + (size_t)c * G); });
        } else if (p.L == 2) {
            for_each_mode(f.n0, [&](int c) {
                float2 al = p.fA1[rn + c];
                for_each_mode(f.n1, [&](int q) {
                    const float2 t = p.fA2[rn + q], r = p.fR1[(size_t)q * p.n + c];
                    al = c_fmaf(al, make_float2(-2.f * t.x, -2.f * t.y), r);
                });
                axpy(al, p.fPhi0 + (size_t)c * G);
            });
            for_each_mode(f.n1, [&](int q) { axpy(p.fA2[rn + q], p.fQ + (size_t)q * G); });
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const double2 b = prow[j];
            a[j] = make_double2(b.x - 2.0 * (double)acc[j].x, b.y - 2.0 * (double)acc[j].y);
        }
    }
}

// Row of M for one CPhase layer from explicit sources (used with the LDS
// copies of a bitstring's factor rows): prow = P[Ri, :] (G entries, FP64),
// a1row = A1[Ri, :] (n entries), phi = Phi0 (n x G), in FP64 or, when MIXED,
// FP32 for the correction.
template <int G, bool MIXED, typename RT>
__device__ __forceinline__ void compose_row_l1(const double2 *prow, const RT *a1row, const RT *phi,
                                               const Flips &f, double2 (&a)[G]) {
    if constexpr (!MIXED) {
#pragma unroll
        for (int j = 0; j < G; ++j) a[j] = prow[j];
        for_each_mode(f.n0, [&](int c) {
            const double2 al = a1row[c];
            const double2 s2 = make_double2(-2.0 * al.x, -2.0 * al.y);
            const double2 *row = phi + (size_t)c * G;
#pragma unroll
            for (int j = 0; j < G; ++j) a[j] = c_fma(a[j], s2, row[j]);
        });
    } else {
        float2 acc[G];
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] = make_float2(0.f, 0.f);
        for_each_mode(f.n0, [&](int c) {
            const float2 al = a1row[c];
            const float2 *row = phi + (size_t)c * G;
#pragma unroll
            for (int j = 0; j < G; ++j) acc[j] = c_fmaf(acc[j], al, row[j]);
        });
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const double2 b = prow[j];
            a[j] = make_double2(b.x - 2.0 * (double)acc[j].x, b.y - 2.0 * (double)acc[j].y);
        }
    }
}

// Cross-lane helpers for a group of G consecutive lanes (G = 4..64, within one
// wave64).  Within a 16-lane DPP row the exchanges are DPP moves (quad
// permutes, half-row and row mirrors), across rows they are bpermutes.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Maximum of v over the group, returned to every lane of the group.
template <int G>
__device__ __forceinline__ double group_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));            // lane ^ 1 (quad_perm 1,0,3,2)
    v = fmax(v, dpp_f64<0x4E>(v));            // lane ^ 2 (quad_perm 2,3,0,1)
    if constexpr (G >= 8) v = fmax(v, dpp_f64<0x141>(v));   // row_half_mirror: quads 0 <-> 1
    if constexpr (G >= 16) v = fmax(v, dpp_f64<0x140>(v));  // row_mirror: half-rows
    if constexpr (G >= 32) v = fmax(v, __shfl_xor(v, 16));
    if constexpr (G >= 64) v = fmax(v, __shfl_xor(v, 32));
    return v;
}

// This lane's group's bits of a wave-wide ballot.
template <int G>
__device__ __forceinline__ uint64_t group_bits(bool pred) {
    const uint64_t all = __ballot(pred);
    if constexpr (G == 64) return all;
    const int base = (int)(threadIdx.x & 63) & ~(G - 1);
    return (all >> base) & ((1ull << G) - 1);
}

// Determinant of the m x m matrix whose row `lane` (< m) is held by lane
// `lane` of a group of G consecutive lanes (rows >= m are padding).  Partial
// pivoting: the pivot of column c is the active row with the largest
// re^2 + im^2 (lowest lane on ties), found by a DPP max and a ballot; rows
// stay in their lanes and the pivot row is broadcast through `piv` (G entries
// of LDS private to the group).  The permutation sign is the parity of the
// inversions between lane order and pivot order, counted from the ballot of
// still-active rows.  An exactly zero pivot column gives det = 0.  Every lane
// of the group returns the determinant.
template <int G>
__device__ __forceinline__ double2 lu_det(double2 (&a)[G], int m, int lane, double2 *piv) {
    bool active = lane < m;
    bool live = true;   // false once a zero pivot column was met (group-uniform)
    unsigned inversions = 0;
    double2 det = make_double2(1.0, 0.0);
#pragma unroll
    for (int c = 0; c < G; ++c) {
        if (c < m && live) {
            const double v = active ? fma(a[c].x, a[c].x, a[c].y * a[c].y) : -1.0;
            const double vmax = group_max<G>(v);
            const uint64_t act = group_bits<G>(active);
            const uint64_t hit = group_bits<G>(active && v == vmax);
            if (vmax > 0.0 && hit != 0) {
                const int idx = __ffsll((long long)hit) - 1;
                inversions += __popcll(act & ((1ull << idx) - 1));
                if (lane == idx) {
                    active = false;
#pragma unroll
                    for (int j = c; j < G; ++j) piv[j] = a[j];
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const double2 u = piv[c];
                det = c_mul(det, u);
                if (active) {
                    const double inv = 1.0 / fma(u.x, u.x, u.y * u.y);
                    const double2 l = c_mul(a[c], make_double2(-u.x * inv, u.y * inv));
#pragma unroll
                    for (int j = c + 1; j < G; ++j) a[j] = c_fma(a[j], l, piv[j]);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                live = false;
            }
        }
    }
    if (!live) return make_double2(0.0, 0.0);
    return (inversions & 1) ? make_double2(-det.x, -det.y) : det;
}



struct RawSmem {
    uint64_t *hkey;
    int2 *hcnt;
    double2 *piv;
    double2 *red;
    uint16_t *list;
    uint8_t *Rb;
    uint64_t *gkey;   // [k] key contribution of gate j, bit 63 = theta_j < 0
    // Sampling table, k rows of trow words (see load_tables): row a holds
    // 32 guide bytes (bucket i: the number of entries <= i << bucket_shift),
    // kpad / 4 boundaries of its 4-entry blocks, then T[a][0 .. kpad) (0
    // before a, all-ones from k on)
    uint32_t *T;
    int kpad;         // entries of a row, a multiple of 16
    int trow;         // words of a row
    // LDS copies for one-layer circuits (STAGE): P rows of the bitstring
    // (G x G FP64), its A1 rows (G x n) and Phi0 (n x G), FP64 or FP32 (MIXED)
    double2 *sP;
    void *sA1;
    void *sPhi;
};

__host__ __device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Bytes of the staged copies (0 when not staged).
__host__ __device__ __forceinline__ size_t stage_bytes(int n, int G, bool mixed) {
    const size_t el = mixed ? 8 : 16;
    return (size_t)G * G * 16 + 2 * (size_t)n * G * el;
}

__host__ __device__ __forceinline__ int table_stride(int k) { return (k + 15) & ~15; }
__host__ __device__ __forceinline__ int table_row_words(int k) { return 8 + table_stride(k) / 4 + table_stride(k); }

// Entry T[a][j] of the LDS sampling table.
__device__ __forceinline__ uint32_t table_at(const RawSmem &s, int a, int j) {
    return s.T[a * s.trow + 8 + (s.kpad >> 2) + j];
}

// Bytes of dynamic LDS the per-bitstring kernels carve (see carve_raw).
__host__ __device__ __forceinline__ size_t raw_lds_bytes(int kk, int n, int G, bool mixed, bool stage) {
    const size_t k = (size_t)kk;
    const size_t base = align16((size_t)kHashSlots * (8 + 8 + 2) + 2 * (size_t)kThreads * 16 + 64 + k * 8) +
                        k * (size_t)table_row_words(kk) * 4;
    return base + (stage ? stage_bytes(n, G, mixed) : 0);
}

__device__ __forceinline__ RawSmem carve_raw(unsigned char *smem, int k, int n, int G, bool mixed) {
    RawSmem s;
    s.hkey = (uint64_t *)smem;
    s.hcnt = (int2 *)(s.hkey + kHashSlots);
    s.piv = (double2 *)(s.hcnt + kHashSlots);
    s.red = s.piv + kThreads;
    s.list = (uint16_t *)(s.red + kThreads);
    s.Rb = (uint8_t *)(s.list + kHashSlots);
    s.gkey = (uint64_t *)(s.Rb + 64);
    s.kpad = table_stride(k);
    s.trow = table_row_words(k);
    const size_t toff = align16((size_t)kHashSlots * (8 + 8 + 2) + 2 * (size_t)kThreads * 16 + 64 + (size_t)k * 8);
    s.T = (uint32_t *)(smem + toff);
    unsigned char *st = smem + toff + (size_t)k * s.trow * 4;
    s.sP = (double2 *)st;
    s.sA1 = (void *)(st + (size_t)G * G * 16);
    s.sPhi = (void *)(st + (size_t)G * G * 16 + (size_t)n * G * (mixed ? 8 : 16));
    return s;
}

// *rank receives the number of flipped modes (the rank of the correction).
template <int G, bool MIXED>
__device__ __forceinline__ double2 term_det(const DevPlan &p, uint64_t key, const uint8_t *Rb,
                                            int lane, double2 *piv, int *rank) {
    double2 a[G];
    const Flips f = decode_key(p, key);
    *rank = __popcll(f.n0[0]) + __popcll(f.n0[1]) + __popcll(f.n1[0]) + __popcll(f.n1[1]);
    if (lane < p.m) {
        compose_row<G, MIXED>(p, Rb[lane], f, a);
    } else {
#pragma unroll
        for (int j = 0; j < G; ++j) a[j] = make_double2(j == lane ? 1.0 : 0.0, 0.0);
    }
    return lu_det<G>(a, p.m, lane, piv);
}

// Same from the LDS copies of the bitstring's factor rows (one CPhase layer).
template <int G, bool MIXED>
__device__ __forceinline__ double2 term_det_staged(const DevPlan &p, uint64_t key, const RawSmem &s,
                                                   int lane, double2 *piv, int *rank) {
    using RT = typename std::conditional<MIXED, float2, double2>::type;
    double2 a[G];
    const Flips f = decode_key(p, key);
    *rank = __popcll(f.n0[0]) + __popcll(f.n0[1]);
    if (lane < p.m) {
        compose_row_l1<G, MIXED>(s.sP + (size_t)lane * G, (const RT *)s.sA1 + (size_t)lane * p.n,
                                 (const RT *)s.sPhi, f, a);
    } else {
#pragma unroll
        for (int j = 0; j < G; ++j) a[j] = make_double2(j == lane ? 1.0 : 0.0, 0.0);
    }
    return lu_det<G>(a, p.m, lane, piv);
}

// Copies Phi0 (once per kernel) into LDS.
template <bool MIXED>
__device__ __forceinline__ void stage_phi(const DevPlan &p, const RawSmem &s) {
    const int cnt = p.n * p.G;
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        if constexpr (MIXED) ((float2 *)s.sPhi)[i] = p.fPhi0[i];
        else ((double2 *)s.sPhi)[i] = p.Phi0[i];
    }
}

// Copies bitstring b's rows of P and A1 into LDS (after load_bitstring).
template <bool MIXED>
__device__ __forceinline__ void stage_rows(const DevPlan &p, const RawSmem &s) {
    const int G = p.G, n = p.n, m = p.m;
    for (int i = threadIdx.x; i < m * G; i += kThreads) s.sP[i] = p.P[(size_t)s.Rb[i / G] * G + (i % G)];
    for (int i = threadIdx.x; i < m * n; i += kThreads) {
        const size_t src = (size_t)s.Rb[i / n] * n + (i % n);
        if constexpr (MIXED) ((float2 *)s.sA1)[i] = p.fA1[src];
        else ((double2 *)s.sA1)[i] = p.A1[src];
    }
    __syncthreads();
}

// Loads bitstring b; returns false (and writes p = 0) if its weight is not
// eta or it has bits at or above n.  Fills Rb with the occupied modes.
__device__ __forceinline__ bool load_bitstring(const DevPlan &p, const uint64_t *bits, int64_t b, uint8_t *Rb,
                               int *s_ok) {
    if (threadIdx.x == 0) {
        const uint64_t w0 = bits[2 * b], w1 = bits[2 * b + 1];
        bool ok = (__popcll(w0) + __popcll(w1)) == p.m;
        if (p.n < 128) {
            const uint64_t hi0 = p.n >= 64 ? 0ull : (~0ull << p.n);
            const uint64_t hi1 = p.n <= 64 ? ~0ull : (~0ull << (p.n - 64));
            ok = ok && !(w0 & hi0) && !(w1 & hi1);
        }
        if (ok) {
            int i = 0;
            for (uint64_t mm = w0; mm; mm &= mm - 1) Rb[i++] = (uint8_t)(__ffsll((long long)mm) - 1);
            for (uint64_t mm = w1; mm; mm &= mm - 1) Rb[i++] = (uint8_t)(64 + __ffsll((long long)mm) - 1);
        }
        *s_ok = ok;
    }
    __syncthreads();
    const bool ok = *s_ok != 0;
    // every thread has read the flag (and may leave the bitstring without
    // another barrier) before thread 0 can overwrite it for the next one
    __syncthreads();
    return ok;
}

// Fixed-order sum of out[0..cnt): each thread adds a contiguous chunk, then a
// fixed tree over the workgroup.  Result valid in thread 0.
__device__ __forceinline__ double2 ordered_sum(const double2 *out, int cnt, double2 *red) {
    const int tid = threadIdx.x;
    const int chunk = (cnt + kThreads - 1) / kThreads;
    double2 s = make_double2(0.0, 0.0);
    const int lo = tid * chunk, hi = min(cnt, lo + chunk);
    for (int e = lo; e < hi; ++e) {
        s.x += out[e].x;
        s.y += out[e].y;
    }
    red[tid] = s;
    __syncthreads();
#pragma unroll
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid].x += red[tid + w].x;
            red[tid].y += red[tid + w].y;
        }
        __syncthreads();
    }
    const double2 r = red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Order-independent summation of the entries' values.  The slots an entry
// lands in depend on the order of insertion, so the values count * det are
// added as 192-bit two's-complement fixed-point integers in units of 2^-158
// (exact, hence associative).  Every determinant is that of a submatrix of a
// unitary matrix, so |det| <= 1, and the counts of one bitstring add up to at
// most t < 2^31 in modulus: the running sum stays below 2^190 units.  Parts
// below 2^-158 are truncated toward zero.  Every pass over the same entries
// therefore gives the same double, whatever the slot, thread and table
// assignment.
// ---------------------------------------------------------------------------
struct Fix192 {
    uint64_t w0 = 0, w1 = 0;
    int64_t w2 = 0;
};

struct FixAcc {
    Fix192 re, im;
    bool bad = false;   // a NaN, an infinity or a value outside the range was added
};

__device__ __forceinline__ void fix_add(Fix192 &a, uint64_t x0, uint64_t x1, int64_t x2) {
    const uint64_t s0 = a.w0 + x0;
    const uint64_t c0 = s0 < a.w0 ? 1 : 0;
    const uint64_t s1 = a.w1 + x1;
    const uint64_t c1 = s1 < a.w1 ? 1 : 0;
    const uint64_t s1c = s1 + c0;
    const uint64_t c2 = s1c < s1 ? 1 : 0;
    a.w0 = s0;
    a.w1 = s1c;
    a.w2 += x2 + (int64_t)(c1 + c2);
}

// a += v * 2^158, truncated toward zero.
__device__ __forceinline__ void fix_add_double(Fix192 &a, bool &bad, double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    const int ex = (int)((bits >> 52) & 0x7FF);
    if (ex == 0x7FF) {
        bad = true;
        return;
    }
    if (ex == 0) return;   // |v| < 2^-1022
    const uint64_t M = (bits & ((1ull << 52) - 1)) | (1ull << 52);
    const int shift = ex - 917;   // v * 2^158 = M * 2^shift
    if (shift > 136) {            // |v| >= 2^32: outside the documented range
        bad = true;
        return;
    }
    if (shift <= -64) return;
    uint64_t x0 = 0, x1 = 0, x2 = 0;
    if (shift < 0) {
        x0 = M >> (-shift);
    } else if (shift < 64) {
        x0 = M << shift;
        x1 = shift ? (M >> (64 - shift)) : 0;
    } else if (shift < 128) {
        const int q = shift - 64;
        x1 = M << q;
        x2 = q ? (M >> (64 - q)) : 0;
    } else {
        x2 = M << (shift - 128);
    }
    if (bits >> 63) {
        x0 = ~x0 + 1;
        const uint64_t c0 = x0 == 0 ? 1 : 0;
        x1 = ~x1 + c0;
        const uint64_t c1 = (c0 && x1 == 0) ? 1 : 0;
        x2 = ~x2 + c1;
    }
    fix_add(a, x0, x1, (int64_t)x2);
}

// Rounded to double through the magnitude (no cancellation between words).
__device__ __forceinline__ double fix_to_double(Fix192 a) {
    const bool neg = a.w2 < 0;
    if (neg) {
        uint64_t x0 = ~a.w0 + 1;
        const uint64_t c0 = x0 == 0 ? 1 : 0;
        uint64_t x1 = ~a.w1 + c0;
        const uint64_t c1 = (c0 && x1 == 0) ? 1 : 0;
        a.w0 = x0;
        a.w1 = x1;
        a.w2 = (int64_t)(~(uint64_t)a.w2 + c1);
    }
    const double m = ((double)(uint64_t)a.w2 * 18446744073709551616.0 + (double)a.w1) * 18446744073709551616.0 +
                     (double)a.w0;
    const double v = ldexp(m, -158);
    return neg ? -v : v;
}

__device__ __forceinline__ void fix_wave_sum(Fix192 &a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t x0 = __shfl_xor((unsigned long long)a.w0, off, 64);
        const uint64_t x1 = __shfl_xor((unsigned long long)a.w1, off, 64);
        const int64_t x2 = __shfl_xor((long long)a.w2, off, 64);
        fix_add(a, x0, x1, x2);
    }
}

// Markers in the per-bitstring entry counts of the determinant-lemma workspace.
constexpr uint32_t kEntryInvalid = 0xFFFFFFFFu;    // bitstring of the wrong weight: p = 0
constexpr uint32_t kEntryOverflow = 0xFFFFFFFEu;   // more entries than the region holds
constexpr uint32_t kEntryDeferred = 0xFFFFFFFDu;   // left to the LU kernel (see k_eval_entries)

// Per-bitstring sum kept in LDS between tables, as 7 words: the real and
// imaginary Fix192 (w0, w1, w2 each) and a flag for bad values.
constexpr int kAccWords = 7;

__device__ __forceinline__ void acc_clear(uint64_t *sacc) {
    if (threadIdx.x < kAccWords) sacc[threadIdx.x] = 0;
}

// *sacc += the values that evaluation left in the slots of the entries e < nl
// (re in hkey, im in hcnt).  Whole workgroup; uses s.red as scratch.
__device__ __forceinline__ void accumulate_slots(const RawSmem &s, int nl, uint64_t *sacc) {
    const int tid = threadIdx.x;
    FixAcc acc;
    for (int e = tid; e < nl; e += kThreads) {
        const uint16_t slot = s.list[e];
        if (slot >= kHashSlots) continue;
        fix_add_double(acc.re, acc.bad, __longlong_as_double((long long)s.hkey[slot]));
        fix_add_double(acc.im, acc.bad, *(const double *)&s.hcnt[slot]);
    }
    fix_wave_sum(acc.re);
    fix_wave_sum(acc.im);
    const bool bad = __ballot(acc.bad) != 0;
    uint64_t *part = (uint64_t *)s.red;   // [wave][7]
    if ((tid & 63) == 0) {
        uint64_t *q = part + kAccWords * (tid >> 6);
        q[0] = acc.re.w0;
        q[1] = acc.re.w1;
        q[2] = (uint64_t)acc.re.w2;
        q[3] = acc.im.w0;
        q[4] = acc.im.w1;
        q[5] = (uint64_t)acc.im.w2;
        q[6] = bad ? 1u : 0u;
    }
    __syncthreads();
    if (tid == 0) {
        Fix192 R, I;
        R.w0 = sacc[0];
        R.w1 = sacc[1];
        R.w2 = (int64_t)sacc[2];
        I.w0 = sacc[3];
        I.w1 = sacc[4];
        I.w2 = (int64_t)sacc[5];
        uint64_t b = sacc[6];
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const uint64_t *q = part + kAccWords * w;
            fix_add(R, q[0], q[1], (int64_t)q[2]);
            fix_add(I, q[3], q[4], (int64_t)q[5]);
            b |= q[6];
        }
        sacc[0] = R.w0;
        sacc[1] = R.w1;
        sacc[2] = (uint64_t)R.w2;
        sacc[3] = I.w0;
        sacc[4] = I.w1;
        sacc[5] = (uint64_t)I.w2;
        sacc[6] = b;
    }
    __syncthreads();
}

// The accumulated sum as doubles (call after the last accumulate_slots).
__device__ __forceinline__ double2 acc_value(const uint64_t *sacc) {
    if (sacc[6]) {
        const double nan = __longlong_as_double(0x7FF8000000000000ll);
        return make_double2(nan, nan);
    }
    Fix192 R, I;
    R.w0 = sacc[0];
    R.w1 = sacc[1];
    R.w2 = (int64_t)sacc[2];
    I.w0 = sacc[3];
    I.w1 = sacc[4];
    I.w2 = (int64_t)sacc[5];
    return make_double2(fix_to_double(R), fix_to_double(I));
}

// Gathers the occupied slots of the hash (non-zero count) into s.list, in no
// particular order.  Returns the number of entries.
template <int NT = kThreads>
__device__ __forceinline__ int gather_list(const RawSmem &s, int *s_n) {
    const int tid = threadIdx.x;
    if (tid == 0) *s_n = 0;
    __syncthreads();
    for (int i = tid; i < kHashSlots; i += NT) {
        if (s.hkey[i] != kEmptyKey && (s.hcnt[i].x != 0 || s.hcnt[i].y != 0)) {
            const int at = atomicAdd(s_n, 1);
            if (at < kHashSlots) s.list[at] = (uint16_t)i;
        }
    }
    __syncthreads();
    return min(*s_n, kHashSlots);
}

// Empties the table and re-reserves the slot of the empty flip pattern.
// Samples per pass of the sampler, and the table fill past which a pass is
// not started (the table is evaluated and cleared first).
constexpr uint32_t kBatch = 1024;
constexpr int kFlushAt = (3 * kHashSlots) / 4;
static_assert(kBatch + 1 <= (uint32_t)kFlushAt, "a fresh table must take a whole batch");
static_assert(kBatch * 4 <= (uint32_t)kHashSlots * 2 && kBatch * 4 <= (uint32_t)kThreads * 16,
              "the sample queues live in the list and in the pivot scratch");

// Sampler position of one workgroup; every thread holds the same values.
struct Sampler {
    uint32_t next = 0;   // first sample of the current batch
    uint32_t j = 0;      // batch number (selects the rotating LDS counters)
    int claimed = 1;     // table slots in use after the last inserted batch
};

// Empties the hash table (slot0 keeps the empty flip pattern) and the six
// sampler counters cnt[0..5].  Whole workgroup.
template <int NT = kThreads>
__device__ __forceinline__ void clear_table(const RawSmem &s, int *cnt, uint32_t slot0, Sampler &st) {
    const int tid = threadIdx.x;
    __syncthreads();
    for (int i = tid; i < kHashSlots; i += NT) {
        s.hkey[i] = kEmptyKey;
        s.hcnt[i] = make_int2(0, 0);
    }
    if (tid < 6) cnt[tid] = 0;
    __syncthreads();
    if (tid == 0) s.hkey[slot0] = 0;
    __syncthreads();
    st.claimed = 1;
}

// Bucket shift of a table row with last entry `tail`: u < tail falls in
// bucket u >> shift, one of 32 (the row's range cut into equal parts).
__device__ __forceinline__ int bucket_shift(uint32_t tail) {
    const int sh = 27 - (int)__clz(tail);
    return sh > 0 ? sh : 0;
}

// The next selected gate from gate a for the uniform draw u (see the
// sampler definition in the public header): the number of entries <= u of
// row a of the table (the row is non-decreasing), or -1 when u >= T[a][k-1].
// The row's guide byte of u's bucket counts the entries <= the bucket's
// start, so the count is that many, rounded down to a multiple of four
// (at most kpad - 8), plus the entries <= u among the next eight, unless all
// eight are (a crowded bucket): then the boundaries of the 4-entry blocks,
// then that block's entries.  Entries past k are all-ones, above every
// u < T[a][k-1] <= 2^32 - 1.
__device__ __forceinline__ int next_gate(const RawSmem &s, int k, int a, uint32_t u) {
    const uint32_t *row = s.T + a * s.trow;
    const uint32_t *ent = row + 8 + (s.kpad >> 2);
    const uint32_t tail = ent[k - 1];
    if (!(u < tail)) return -1;
    const int g = ((const uint8_t *)row)[u >> bucket_shift(tail)];
    const int b4 = min(g & ~3, s.kpad - 8);
    const uint4 e0 = *(const uint4 *)(ent + b4), e1 = *(const uint4 *)(ent + b4 + 4);
    const int c = (e0.x <= u) + (e0.y <= u) + (e0.z <= u) + (e0.w <= u) + (e1.x <= u) + (e1.y <= u) +
                  (e1.z <= u) + (e1.w <= u);
    if (c < 8) return b4 + c;
    int cs = 0;
    for (int i = 0; i < (s.kpad >> 2); i += 4) {
        const uint4 q = *(const uint4 *)(row + 8 + i);
        cs += (q.x <= u) + (q.y <= u) + (q.z <= u) + (q.w <= u);
    }
    const uint4 e = ((const uint4 *)ent)[cs];
    return 4 * cs + (e.x <= u) + (e.y <= u) + (e.z <= u) + (e.w <= u);
}

// The rest of trajectory smp of bitstring (blo, bhi) whose first draw
// selected gate j0: draws u_1, u_2, ... (word (d - 1) mod 4 of the Philox
// block with counter (smp, (d - 1) / 4, blo, bhi)) until no further gate is
// selected.  Returns the flip-pattern key and the phase exponent e (i^e).
__device__ __forceinline__ void draw_rest(const DevPlan &p, const RawSmem &s, uint32_t smp, int j0, uint32_t blo,
                                          uint32_t bhi, uint32_t k0, uint32_t k1, uint64_t &key, uint32_t &e,
                                          unsigned long long &blocks) {
    const int k = p.k;
    uint64_t g = s.gkey[j0];
    key = g & ~(1ull << 63);
    e = 1u + 2u * (uint32_t)(g >> 63);
    int a = j0 + 1;
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t d = 0; a < k; ++d) {
        if ((d & 3) == 0) {
            r = philox10(make_uint4(smp, d >> 2, blo, bhi), k0, k1);
            ++blocks;
        }
        const uint32_t w = d & 3;
        const uint32_t u = w == 0 ? r.x : (w == 1 ? r.y : (w == 2 ? r.z : r.w));
        const int j = next_gate(s, k, a, u);
        if (j < 0) break;
        g = s.gkey[j];
        key ^= g & ~(1ull << 63);
        e += 1u + 2u * (uint32_t)(g >> 63);
        a = j + 1;
    }
}

// Draws trajectories of bitstring b (batch index b) in batches of kBatch
// samples, reducing each to its flip-pattern key in the LDS hash, until either
// all t samples are in (returns true) or the next batch could push the table
// past kFlushAt slots (returns false; that batch is drawn again after the
// table has been evaluated and cleared).  A batch runs in two phases: the
// last kBatch / 4 threads each draw the first uniforms of four consecutive
// samples (one Philox block), which decide whether a sample sets any gate at
// all (u_0 < T[0][k-1]); those samples are queued in LDS, and after the
// barrier the workgroup, from its first thread on, draws them to the end and
// inserts them, so the long draws are spread over all lanes, and with more
// than kBatch / 4 threads the first phase of the next batch runs in other
// waves than the second phase of this one.  A queue entry holds the sample's
// batch offset in its low 10 bits and u_0 with those bits cleared in the
// rest; the first gate follows from that unless a table entry of row 0 falls
// between the truncated and the full u_0, and only then is u_0 drawn again.
// The bound uses the exact count of slots in use plus the
// batch's non-empty samples, so the stopping points depend only on the
// samples and every pass over the same bitstring empties the table at the
// same samples.  Counts of the batch's non-empty samples (which are also the
// queue positions) and of the slots each batch claims live in three rotating
// LDS counters each (cnt[0..2], cnt[3..5]), read only after the barrier that
// follows their last update and cleared two batches before their next use;
// the queue alternates between two buffers (the list and pivot scratch, free
// while sampling).  Whole workgroup; s.T / s.gkey loaded (load_tables); the table
// cleared (clear_table) before the first call and between calls.
template <int NT = kThreads>
__device__ __forceinline__ bool sample_until_flush(const DevPlan &p, const RawSmem &s, int *cnt,
                                                   uint32_t slot0, int64_t b, uint32_t t, uint32_t k0,
                                                   uint32_t k1, Sampler &st, unsigned long long &blocks) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const uint32_t blo = (uint32_t)b, bhi = (uint32_t)((uint64_t)b >> 32);
    const uint32_t any = p.k > 0 ? table_at(s, 0, p.k - 1) : 0u;   // T[0][k-1]
    int *pend = cnt, *added = cnt + 3;
    constexpr int NQ = (int)(kBatch / 4);   // first-draw blocks per batch
    constexpr uint32_t kOff = kBatch - 1;   // offset bits of a queue entry
    static_assert(NQ % 64 == 0 && NQ <= NT, "first draws by whole waves");
    static_assert((kBatch & kOff) == 0, "batch offsets are the low bits of a queue entry");
    const int q = tid - (NT - NQ);          // first-draw block of this thread, if >= 0
    for (; st.next < t; st.next += kBatch, ++st.j) {
        uint32_t *queue = (st.j & 1) ? (uint32_t *)s.piv : (uint32_t *)s.list;
        if (q >= 0) {
            // u_0 of samples next + 4 q + w is word w of block (next / 4 + q, 2^32 - 1)
            const uint4 r = philox10(make_uint4((st.next >> 2) + (uint32_t)q, 0xFFFFFFFFu, blo, bhi), k0, k1);
            if (st.next + 4u * (uint32_t)q < t) ++blocks;
            // live samples of the batch (offsets below lim)
            const uint32_t lim = min(kBatch, t - st.next);
            uint32_t ent[4];
            bool sel[4];
            uint64_t ball[4];
            int total = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t off = 4u * (uint32_t)q + (uint32_t)w;
                const uint32_t u = w == 0 ? r.x : (w == 1 ? r.y : (w == 2 ? r.z : r.w));
                ent[w] = (u & ~kOff) | off;
                sel[w] = (u < any) & (off < lim);
                ball[w] = __ballot(sel[w]);
                total += (int)__popcll(ball[w]);
            }
            int at = 0;
            if (lane == 0 && total) at = atomicAdd(&pend[st.j % 3], total);
            at = __shfl(at, 0, 64);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                // queue position: the selected samples of lower lanes (mbcnt of the ballot)
                const uint32_t below_sel = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(ball[w] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball[w], 0u));
                if (sel[w]) queue[at + (int)below_sel] = ent[w];
                at += (int)__popcll(ball[w]);
            }
        }
        __syncthreads();
        const int pending = pend[st.j % 3];
        st.claimed += added[(st.j + 2) % 3];
        if (tid == 0) {
            pend[(st.j + 2) % 3] = 0;
            added[(st.j + 1) % 3] = 0;
        }
        if (st.claimed > 1 && st.claimed + pending > kFlushAt) {
            // this batch is drawn again after the flush: count its first draws once
            if (q >= 0 && st.next + 4u * (uint32_t)q < t) --blocks;
            return false;
        }
        if (tid == 0) {
            const int live = (int)min((uint32_t)kBatch, t - st.next);
            if (live > pending) atomicAdd(&s.hcnt[slot0].x, live - pending);
        }
        int fresh = 0;
        for (int i = tid; i < pending; i += NT) {
            const uint32_t ent = queue[i];
            const uint32_t smp = st.next + (ent & kOff), hi = ent & ~kOff;
            // every u in [hi, hi | kOff] selects gate j0 first unless T[0][j0] lies in that range
            // (hi < T[0][k-1], so 0 <= j0 < k)
            int j0 = next_gate(s, p.k, 0, hi);
            if (table_at(s, 0, j0) <= (hi | kOff)) {
                const uint4 r0 = philox10(make_uint4(smp >> 2, 0xFFFFFFFFu, blo, bhi), k0, k1);
                const uint32_t w0 = smp & 3;
                j0 = next_gate(s, p.k, 0, w0 == 0 ? r0.x : (w0 == 1 ? r0.y : (w0 == 2 ? r0.z : r0.w)));
            }
            uint64_t key;
            uint32_t e;
            draw_rest(p, s, smp, j0, blo, bhi, k0, k1, key, e, blocks);
            uint32_t slot = hash_slot(key);
            while (true) {
                const unsigned long long prev = atomicCAS((unsigned long long *)&s.hkey[slot],
                                                          (unsigned long long)kEmptyKey, (unsigned long long)key);
                if (prev == kEmptyKey) {
                    ++fresh;
                    break;
                }
                if (prev == key) break;
                slot = (slot + 1) & (kHashSlots - 1);
            }
            // phase i^e: +-1 on the real (e even) or imaginary (e odd) count
            atomicAdd((e & 1) ? &s.hcnt[slot].y : &s.hcnt[slot].x, (e & 2) ? -1 : 1);
        }
        if (fresh) atomicAdd(&added[st.j % 3], fresh);
    }
    return true;
}

// Work done by one thread, kept in registers and added to the plan's device
// counters once at the end of a kernel: [0] distinct determinants, [1] sum of
// their correction ranks, [2] FP64-equivalent FLOPs of the evaluation, [3]
// bases whose lemma products ran on the FP32 matrix cores.  The other
// counters of a call: [4] Philox blocks of the sampling definition, [5]
// bitstrings the one-wave setup left to the workgroup setup, [6] bitstrings
// left to the pattern pass with lane groups of 32 (the passes that take them
// return at once when their counter is zero).
struct Work {
    unsigned long long terms = 0, rank = 0, flops = 0, fp32 = 0;
};

// Real FLOPs of the partial-pivot LU determinant of a complex m x m matrix.
__device__ __forceinline__ unsigned long long lu_flops(int m) {
    return (unsigned long long)((4 * (m - 1) * m * (2 * m - 1)) / 3 + 3 * m * (m - 1));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Every thread of the workgroup calls this.
__device__ __forceinline__ void flush_work(const Work &w, unsigned long long *nterm) {
    if (!nterm) return;
    const unsigned long long a = wave_sum(w.terms), b = wave_sum(w.rank), c = wave_sum(w.flops),
                             d = wave_sum(w.fp32);
    if ((threadIdx.x & 63) == 0) {
        if (a) atomicAdd(nterm, a);
        if (b) atomicAdd(nterm + 1, b);
        if (c) atomicAdd(nterm + 2, c);
        if (d) atomicAdd(nterm + 3, d);
    }
}

// Gauss-Jordan inverse with partial pivoting (same pivot rule as lu_det).
// On return lane r (< m) holds row pos of M^-1 in v, where pos is the step at
// which its row was the pivot; det = sign * prod(pivots).  Returns false for
// an exactly singular matrix.
template <int G>
__device__ __forceinline__ bool gj_invert(double2 (&a)[G], double2 (&v)[G], int m, int lane,
                                          double2 *pv, double2 &det, int &pos) {
    bool active = lane < m;
    bool live = true;
    bool neg = false;
    pos = lane;
    det = make_double2(1.0, 0.0);
#pragma unroll
    for (int j = 0; j < G; ++j) v[j] = make_double2((j == lane && lane < m) ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int c = 0; c < G; ++c) {
        if (c < m && live) {
            double best = active ? fma(a[c].x, a[c].x, a[c].y * a[c].y) : -1.0;
            int idx = lane;
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const double vo = __shfl_xor(best, off, G);
                const int io = __shfl_xor(idx, off, G);
                if (vo > best || (vo == best && io < idx)) {
                    best = vo;
                    idx = io;
                }
            }
            if (best > 0.0) {
                const int ppos = __shfl(pos, idx, G);
                neg ^= (ppos != c);
                if (pos == c) pos = ppos;
                if (lane == idx) {
                    pos = c;
                    active = false;
                    const double2 u = a[c];
                    const double inv = 1.0 / fma(u.x, u.x, u.y * u.y);
                    const double2 ui = make_double2(u.x * inv, -u.y * inv);
                    pv[c] = u;
#pragma unroll
                    for (int j = c + 1; j < G; ++j) pv[j] = c_mul(a[j], ui);
#pragma unroll
                    for (int j = 0; j < G; ++j) pv[G + j] = c_mul(v[j], ui);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                det = c_mul(det, pv[c]);
                if (lane == idx) {
#pragma unroll
                    for (int j = c + 1; j < G; ++j) a[j] = pv[j];
#pragma unroll
                    for (int j = 0; j < G; ++j) v[j] = pv[G + j];
                    a[c] = make_double2(1.0, 0.0);
                } else if (lane < m) {
                    const double2 l = make_double2(-a[c].x, -a[c].y);
#pragma unroll
                    for (int j = c + 1; j < G; ++j) a[j] = c_fma(a[j], l, pv[j]);
#pragma unroll
                    for (int j = 0; j < G; ++j) v[j] = c_fma(v[j], l, pv[G + j]);
                    a[c] = make_double2(0.0, 0.0);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                live = false;
            }
        }
    }
    if (neg) det = make_double2(-det.x, -det.y);
    return live;
}

// ---------------------------------------------------------------------------
// Determinant-lemma evaluation (one CPhase layer).
//
// Every submatrix of a bitstring shares the base M_0 = P[R, :]:
//   M_N = M_0 - 2 A1[R, N] Phi0[N, :]
//   det M_N = det M_0 * det(I_r - 2 H[N, N]),  H = Phi0[act, :] M_0^-1 A1[R, act]
// over the modes `act` the CPhase gates touch (the key's bit positions).  The
// per-bitstring work is one Gauss-Jordan inverse and two thin products; each
// distinct key then costs an r x r determinant (r = flipped modes): one lane
// for r <= kLemmaMaxRank, a lane group above.  Bitstrings with
// kappa_1(M_0) > 1e4 (or an exactly singular M_0) use the LU of M_N instead.
// ---------------------------------------------------------------------------
constexpr int kLemmaMaxRank = 4;
constexpr double kLemmaMaxCond = 1e4;

// Bytes of the lemma's persistent LDS: P rows (G x G) and H (kb x kb), FP64.
__host__ __device__ __forceinline__ size_t lemma_bytes(int G, int kb) {
    return (size_t)G * G * 16 + align16((size_t)kb * kb * 16);
}

// Inverse and determinant of the m x m matrix W (LDS, row stride G, m <= G <=
// 16) by Gauss-Jordan on the augmented rows [W | I], held in the registers of
// one wave: lane 16 q + i holds columns q G/2 .. q G/2 + G/2 - 1 of row i.
// Pivoting as in lu_det (the unused row with the largest |a|^2 in the
// column, lowest row on ties; a DPP max and a ballot); rows stay in their
// lanes, so row p_c (the pivot of column c) ends as u_c e_c on the left and
// as u_c times row c of W^-1 on the right.  Each step sends the pivot row and
// the multiplier column through LDS (xbuf: 2 (2G + 16) entries, one half per
// step parity).  det W = sign(c -> p_c) prod u_c.  Writes W^-1 to Minv (row
// stride G) and returns true, or returns false without writing when a pivot
// column is exactly zero.  Whole wave, wave-uniform m.
template <int G>
__device__ __forceinline__ bool gj_inverse_wave(const double2 *W, int m, double2 *Minv, double2 *xbuf,
                                                double2 &det_out) {
    static_assert(G % 2 == 0 && G <= 16, "four quarters of G / 2 columns per row");
    constexpr int CPL = G / 2;
    const int lane = threadIdx.x & 63, q = lane >> 4, i = lane & 15;
    double2 a[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int col = q * CPL + j;
        double2 v = make_double2(0.0, 0.0);
        if (i < m) v = col < G ? W[i * G + col] : make_double2(col - G == i ? 1.0 : 0.0, 0.0);
        a[j] = v;
    }
    bool active = i < m, live = true;
    unsigned inversions = 0;
    double2 det = make_double2(1.0, 0.0), pinv = make_double2(0.0, 0.0);
    int pstep = 0;
#pragma unroll
    for (int c = 0; c < G; ++c) {
        if (c < m && live) {
            const int qc = c / CPL, jc = c % CPL;
            const double v = (active && q == qc) ? fma(a[jc].x, a[jc].x, a[jc].y * a[jc].y) : -1.0;
            const double vmax = group_max<16>(v);
            const uint64_t hit = (__ballot(q == qc && active && v == vmax && vmax > 0.0) >> (16 * qc)) & 0xFFFFull;
            if (hit == 0) {
                live = false;
            } else {
                const int p = __ffsll((long long)hit) - 1;
                inversions += __popcll(__ballot(active) & ((1ull << p) - 1));
                double2 *prow = xbuf + (c & 1) * (2 * G + 16);
                double2 *mcol = prow + 2 * G;
                if (i == p) {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) prow[q * CPL + j] = a[j];
                }
                if (q == qc) mcol[i] = a[jc];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const double2 u = mcol[p];
                const double2 mi = mcol[i];
                double2 r[CPL];
#pragma unroll
                for (int j = 0; j < CPL; ++j) r[j] = prow[q * CPL + j];
                det = c_mul(det, u);
                const double inv = 1.0 / fma(u.x, u.x, u.y * u.y);
                const double2 ui = make_double2(u.x * inv, -u.y * inv);
                if (i == p) {
                    pstep = c;
                    pinv = ui;
                    active = false;
                } else if (i < m) {
                    const double2 l = c_mul(mi, ui);
#pragma unroll
                    for (int j = 0; j < CPL; ++j)
                        a[j] = make_double2(a[j].x - (l.x * r[j].x - l.y * r[j].y),
                                            a[j].y - (l.x * r[j].y + l.y * r[j].x));
                }
            }
        }
    }
    if (!live) return false;
    if (q >= 2 && i < m) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) Minv[pstep * G + (q - 2) * CPL + j] = c_mul(a[j], pinv);
    }
    det_out = (inversions & 1) ? make_double2(-det.x, -det.y) : det;
    return true;
}

struct LemmaBits {
    double2 detB;   // det M_0
    int ok;         // lemma usable for this bitstring
};

// Per-bitstring setup; whole workgroup; FP64 throughout.  M_0 = P[R, :] is
// copied to sP; wave 0 inverts it (gj_inverse_wave) into the not yet used
// hash keys, while the other waves copy the operands of X and H.  Then X = M_0^-1 A1[R, act]
// (after V in the hash keys) and H = Phi0[act, :] X into sH.  When
// m * |act| <= 512 the operands A1[R, act] and Phi0[act, :] are first copied
// to the hash counts (their loads overlap the elimination).
// s_flag: two ints of LDS (inverse found; conditioning acceptable).
template <int G>
__device__ __forceinline__ LemmaBits lemma_setup(const DevPlan &p, const RawSmem &s, double2 *sH,
                                                 int *s_flag, double2 *s_det, Work &wk) {
    const int tid = threadIdx.x, m = p.m, n = p.n, kb = p.keybits;
    double2 *W = s.sP;                        // m x G, left half
    double2 *V = (double2 *)s.hkey;           // m x G, right half -> M_0^-1
    double2 *X = V + G * G;                   // m x kb
    const bool staged = m * kb <= 512;
    double2 *A1s = (double2 *)s.hcnt;         // m x kb: A1[R, act]
    double2 *Phs = A1s + 512;                 // kb x m: Phi0[act, :]
    for (int i = tid; i < m * G; i += kThreads) {
        const int r = i / G, c = i % G;
        W[i] = p.P[(size_t)s.Rb[r] * G + c];
    }
    if (tid == 0) {
        *s_flag = 1;
        *s_det = make_double2(1.0, 0.0);
    }
    __syncthreads();
    if (tid >= 64) {
        // waves 1..3 copy the operands of X and H while wave 0 eliminates
        if (staged) {
            for (int i = tid - 64; i < m * kb; i += kThreads - 64) {
                const int l = i / kb, q = i % kb;
                A1s[i] = p.A1[(size_t)s.Rb[l] * n + p.keymode[q]];
                const int q2 = i / m, j = i % m;
                Phs[i] = p.Phi0[(size_t)p.keymode[q2] * G + j];
            }
        }
    } else {
        const int lane = tid;
        // ||M_0||_1 (largest column sum of moduli), kept in red[G]
        double cs = 0.0;
        if (lane < m)
            for (int i = 0; i < m; ++i) {
                const double2 x = W[i * G + lane];
                cs += sqrt(x.x * x.x + x.y * x.y);
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
        if (lane == 0) s.red[G].x = cs;
        double2 det = make_double2(0.0, 0.0);
        const bool ok = gj_inverse_wave<G>(W, m, V, s.piv, det);
        if (lane == 0) {
            *s_flag = ok ? 1 : 0;
            *s_det = det;
        }
    }
    __syncthreads();
    LemmaBits lb;
    lb.ok = *s_flag;
    lb.detB = *s_det;
    if (!lb.ok) {
        lb.detB = make_double2(0.0, 0.0);
        __syncthreads();
        return lb;
    }
    // kappa_1 = ||M_0||_1 ||M_0^-1||_1, into its own flag (s_flag[0] may
    // still be read by other waves)
    if (tid < 64) {
        double cs = 0.0;
        if (tid < m)
            for (int i = 0; i < m; ++i) {
                const double2 x = V[i * G + tid];
                cs += sqrt(x.x * x.x + x.y * x.y);
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
        if (tid == 0) s_flag[1] = cs * s.red[G].x <= kLemmaMaxCond ? 1 : 0;
    }
    __syncthreads();
    lb.ok = s_flag[1];
    if (tid == 0) {
        // elimination (multipliers, updates of the m - 1 other rows over the
        // remaining left columns and the right half), scaling by the pivots
        unsigned long long f = 6ull * m * m;
        for (int c = 0; c < m; ++c) f += 7 + 6ull * (m - 1) + 8ull * (m - 1) * (2 * m - 1 - c);
        if (lb.ok) f += 8ull * m * m * kb + 8ull * m * kb * kb;   // X and H
        wk.flops += f;
    }
    if (!lb.ok) return lb;
    // X = M_0^-1 A1[R, act]
    for (int i = tid; i < m * kb; i += kThreads) {
        const int j = i / kb, q = i % kb;
        double2 acc = make_double2(0.0, 0.0);
        if (staged) {
            for (int l = 0; l < m; ++l) acc = c_fma(acc, V[j * G + l], A1s[l * kb + q]);
        } else {
            const int c = p.keymode[q];
            for (int l = 0; l < m; ++l) acc = c_fma(acc, V[j * G + l], p.A1[(size_t)s.Rb[l] * n + c]);
        }
        X[j * kb + q] = acc;
    }
    __syncthreads();
    // H = Phi0[act, :] X
    for (int i = tid; i < kb * kb; i += kThreads) {
        const int q = i / kb, q2 = i % kb;
        double2 acc = make_double2(0.0, 0.0);
        if (staged) {
            for (int j = 0; j < m; ++j) acc = c_fma(acc, Phs[q * m + j], X[j * kb + q2]);
        } else {
            const int c = p.keymode[q];
            for (int j = 0; j < m; ++j) acc = c_fma(acc, p.Phi0[(size_t)c * G + j], X[j * kb + q2]);
        }
        sH[q * kb + q2] = acc;
    }
    __syncthreads();
    return lb;
}

// det(I_r - 2 H[N, N]) for the r <= kLemmaMaxRank set bits of key (one lane):
// LU with partial pivoting (largest |a|^2, lowest row on ties) by row swaps
// through static-index selects; rows and columns >= r are left untouched.
__device__ __forceinline__ double2 lemma_small_det(uint64_t key, const double2 *sH, int kb) {
    constexpr int RM = kLemmaMaxRank;
    int pos[RM];
    uint64_t mm = key;
    int r = 0;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        pos[i] = mm ? __ffsll((long long)mm) - 1 : 0;
        if (mm) ++r;
        mm &= mm - 1;
    }
    double2 a[RM][RM];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RM; ++j) {
            double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
            if (i < r && j < r) {
                const double2 h = sH[pos[i] * kb + pos[j]];
                v.x -= 2.0 * h.x;
                v.y -= 2.0 * h.y;
            }
            a[i][j] = v;
        }
    bool neg = false;
    double2 det = make_double2(1.0, 0.0);
#pragma unroll
    for (int c = 0; c < RM; ++c) {
        if (c < r) {
            int piv = c;
            double best = fma(a[c][c].x, a[c][c].x, a[c][c].y * a[c][c].y);
#pragma unroll
            for (int i = c + 1; i < RM; ++i) {
                const double v = fma(a[i][c].x, a[i][c].x, a[i][c].y * a[i][c].y);
                if (i < r && v > best) {
                    best = v;
                    piv = i;
                }
            }
            if (!(best > 0.0)) return make_double2(0.0, 0.0);
            neg ^= piv != c;
#pragma unroll
            for (int i = c + 1; i < RM; ++i) {
                if (piv == i) {
#pragma unroll
                    for (int j = c; j < RM; ++j) {
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
            for (int i = c + 1; i < RM; ++i) {
                if (i < r) {
                    const double2 l = c_mul(a[i][c], ui);
#pragma unroll
                    for (int j = c + 1; j < RM; ++j) a[i][j] = c_fma(a[i][j], l, a[c][j]);
                }
            }
        }
    }
    return neg ? make_double2(-det.x, -det.y) : det;
}



// Rows of I - 2 H[N, N] for the r set bits of key, one row per lane of a
// group of GS lanes (rows and columns >= r are those of the identity).
template <int GS>
__device__ __forceinline__ void lemma_rows(uint64_t key, int r, int lane, const double2 *sH, int kb,
                                           double2 (&a)[GS]) {
    uint64_t mm = key;
    int own = 0;
#pragma unroll
    for (int i = 0; i < GS; ++i) {
        const int q = mm ? __ffsll((long long)mm) - 1 : 0;
        if (i == lane) own = q;
        mm &= mm - 1;
    }
    mm = key;
#pragma unroll
    for (int j = 0; j < GS; ++j) {
        const int q = mm ? __ffsll((long long)mm) - 1 : 0;
        mm &= mm - 1;
        double2 v = make_double2(j == lane ? 1.0 : 0.0, 0.0);
        if (lane < r && j < r) {
            const double2 h = sH[own * kb + q];
            v.x -= 2.0 * h.x;
            v.y -= 2.0 * h.y;
        }
        a[j] = v;
    }
}


// Evaluation of one table under the determinant lemma.  The entries are
// first classified by r, the number of flipped modes:
//   easy (r <= kLemmaMaxRank): one lane each, taken in order of r (counting
//      sort) so that the lanes of a wave run the same number of steps;
//   mid (kLemmaMaxRank < r <= 8): the r x r matrix I - 2 H[N, N] factored by
//      8-lane groups;
//   hard (8 < r <= G): the same with G-lane groups.
// A table with a larger pattern (r > G, nine or more flipped CPhase gates,
// or more mid and hard patterns than the short list holds) is not
// evaluated: the call returns false and the bitstring is left to the LU
// kernel, which keeps the composition of M_N out of this kernel.  Values go
// into the slots and are added to the bitstring's sum.
constexpr int kLemmaMid = 8;

template <int G>
__device__ __forceinline__ bool sum_entries_lemma(const DevPlan &p, const RawSmem &s, int nl,
                                                  const double2 *sH, const LemmaBits &lb, Work &wk,
                                                  uint64_t *sacc) {
    const int tid = threadIdx.x;
    const int kb = p.keybits;
    int *cnt = (int *)s.red;  // [0..4] easy bins, 7 easy, 8 mid, 9 larger, 10 mid / 11 hard cursor, 12 hard
    uint16_t *order = (uint16_t *)s.piv;  // easy entries by r (the pivot scratch is free until then)
    uint16_t *mid = (uint16_t *)s.red + 32;
    constexpr int kMidCap = (kThreads * 16 - 64) / 2;   // u16 entries after 64 B of counters
    constexpr int kHardMax = G > kLemmaMid ? G : kLemmaMid;
    if (tid < 13) cnt[tid] = 0;
    __syncthreads();
    for (int e = tid; e < nl; e += kThreads) {
        const int r = __popcll(s.hkey[s.list[e]]);
        atomicAdd(&cnt[r <= kLemmaMaxRank ? r : (r <= kLemmaMid ? 8 : (r <= kHardMax ? 12 : 9))], 1);
    }
    __syncthreads();
    if (cnt[9] > 0 || cnt[8] + cnt[12] > kMidCap) return false;
    if (tid == 0) {
        int acc = 0;
        for (int r = 0; r <= kLemmaMaxRank; ++r) {
            const int h = cnt[r];
            cnt[r] = acc;
            acc += h;
        }
        cnt[7] = acc;
        cnt[10] = 0;
        cnt[11] = cnt[8];
    }
    __syncthreads();
    const int n_easy = cnt[7], n_mid = cnt[8], n_hard = cnt[12];
    for (int e = tid; e < nl; e += kThreads) {
        const uint16_t slot = s.list[e];
        const int r = __popcll(s.hkey[slot]);
        if (r <= kLemmaMaxRank) order[atomicAdd(&cnt[r], 1)] = slot;
        else mid[atomicAdd(&cnt[r <= kLemmaMid ? 10 : 11], 1)] = slot;
    }
    __syncthreads();
    for (int i = tid; i < n_easy; i += kThreads) {
        const uint16_t slot = order[i];
        const uint64_t key = s.hkey[slot];
        const int r = __popcll(key);
        const int2 c = s.hcnt[slot];
        const double2 d = c_mul(lb.detB, lemma_small_det(key, sH, kb));
        s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
        *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
        wk.rank += (unsigned)r;
        wk.flops += lu_flops(r) + 6;
    }
    __syncthreads();
    {
        const int l8 = tid & 7, g8 = tid >> 3;
        for (int i = g8; i < n_mid; i += kThreads / 8) {
            const uint16_t slot = mid[i];
            const uint64_t key = s.hkey[slot];
            const int r = __popcll(key);
            const int2 c = s.hcnt[slot];
            double2 a[kLemmaMid];
            lemma_rows<kLemmaMid>(key, r, l8, sH, kb, a);
            const double2 d = c_mul(lb.detB, lu_det<kLemmaMid>(a, r, l8, s.piv + g8 * kLemmaMid));
            if (l8 == 0) {
                s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
                *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
                wk.rank += (unsigned)r;
                wk.flops += lu_flops(r) + 6;
            }
        }
        __syncthreads();
    }
    if constexpr (G > kLemmaMid) {
        const int lane = tid % G, grp = tid / G;
        for (int i = n_mid + grp; i < n_mid + n_hard; i += kThreads / G) {
            const uint16_t slot = mid[i];
            const uint64_t key = s.hkey[slot];
            const int r = __popcll(key);
            const int2 c = s.hcnt[slot];
            double2 a[G];
            lemma_rows<G>(key, r, lane, sH, kb, a);
            const double2 d = c_mul(lb.detB, lu_det<G>(a, r, lane, s.piv + grp * G));
            if (lane == 0) {
                s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
                *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
                wk.rank += (unsigned)r;
                wk.flops += lu_flops(r) + 6;
            }
        }
        __syncthreads();
    }
    if (tid == 0) wk.terms += (unsigned)nl;
    accumulate_slots(s, nl, sacc);
    return true;
}

// Sum over the entries of count * det.  Each group evaluates entries
// e = grp, grp + NG, ...; the product is left in the entry's slot and added
// to the bitstring's LDS sum.
template <int G, bool MIXED, bool STAGE>
__device__ __forceinline__ void sum_entries(const DevPlan &p, const RawSmem &s, int nl, Work &wk,
                                            uint64_t *sacc) {
    const int tid = threadIdx.x;
    const int lane = tid % G, grp = tid / G;
    constexpr int NG = kThreads / G;
    const int m = p.m;
    for (int e = grp; e < nl; e += NG) {
        const uint16_t slot = s.list[e];
        if (slot >= kHashSlots) continue;   // unreachable: the list holds slot indices
        const uint64_t key = s.hkey[slot];
        const int2 c = s.hcnt[slot];
        int rank;
        double2 d;
        if constexpr (STAGE) d = term_det_staged<G, MIXED>(p, key, s, lane, s.piv + grp * G, &rank);
        else d = term_det<G, MIXED>(p, key, s.Rb, lane, s.piv + grp * G, &rank);
        if (lane == 0) {
            s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
            *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
            wk.rank += (unsigned)rank;
            wk.flops += lu_flops(m) + 8ull * m * m * rank;
        }
    }
    __syncthreads();
    if (tid == 0) wk.terms += (unsigned)nl;
    accumulate_slots(s, nl, sacc);
}

template <int NT = kThreads>
__device__ __forceinline__ void load_tables(const DevPlan &p, const RawSmem &s) {
    const int tid = threadIdx.x;
    const int k = p.k;
    const int kp = s.kpad, tr = s.trow;
    // row a: [ 32 guide bytes | T[a][4 c + 3], c < kp / 4 | T[a][j], j < kp ],
    // entries past k all-ones; the guide bytes from the entries in LDS
    for (int i = tid; i < k * tr; i += NT) {
        const int a = i / tr, w = i % tr;
        if (w < 8) continue;
        const int j = w < 8 + kp / 4 ? 4 * (w - 8) + 3 : w - 8 - kp / 4;
        s.T[i] = j < k ? p.T[a * k + j] : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int i = tid; i < k * 8; i += NT) {
        const int a = i >> 3, w = i & 7;
        const uint32_t *ent = s.T + a * tr + 8 + kp / 4;
        const int sh = bucket_shift(ent[k - 1]);
        uint32_t word = 0;
        for (int b = 0; b < 4; ++b) {
            const uint32_t start = (uint32_t)(4 * w + b) << sh;
            int c = 0;
            for (int j = 0; j < k; ++j) c += ent[j] <= start;
            word |= (uint32_t)c << (8 * b);
        }
        s.T[a * tr + w] = word;
    }
    for (int i = tid; i < k; i += NT) s.gkey[i] = p.gkey[i] | ((uint64_t)(p.gneg[i] != 0) << 63);
}

// The sampler kernel runs eight waves per workgroup: its LDS (the table) then
// serves twice the waves, and its few registers allow them.
constexpr int kSamplerThreads = 512;

__host__ __device__ __forceinline__ size_t sampler_head_bytes(int k) {
    return align16((size_t)kHashSlots * (8 + 8 + 2) + (size_t)kThreads * 16 + 64 + (size_t)k * 8);
}
__host__ __device__ __forceinline__ size_t sampler_lds_bytes(int k) {
    return sampler_head_bytes(k) + (size_t)k * table_row_words(k) * 4;
}

// Sampler layout: the hash, the two sample queues (pivot scratch and list)
// and the tables; no reduction scratch or factor copies.
__device__ __forceinline__ RawSmem carve_sampler(unsigned char *smem, int k) {
    RawSmem s;
    s.hkey = (uint64_t *)smem;
    s.hcnt = (int2 *)(s.hkey + kHashSlots);
    s.piv = (double2 *)(s.hcnt + kHashSlots);
    s.red = nullptr;
    s.list = (uint16_t *)(s.piv + kThreads);
    s.Rb = (uint8_t *)(s.list + kHashSlots);
    s.gkey = (uint64_t *)(s.Rb + 64);
    s.kpad = table_stride(k);
    s.trow = table_row_words(k);
    s.T = (uint32_t *)(smem + sampler_head_bytes(k));
    s.sP = nullptr;
    s.sA1 = nullptr;
    s.sPhi = nullptr;
    return s;
}

constexpr int kMaxGrid = 1 << 20;
constexpr size_t kMaxLds = 159 * 1024;

// LDS copies of the factor rows pay off for one CPhase layer and small eta,
// when they fit beside the table.
__host__ __forceinline__ bool use_stage(const DevPlan &p, bool mixed) {
    return p.L == 1 && p.G <= 16 && raw_lds_bytes(p.k, p.n, p.G, mixed, true) <= kMaxLds;
}

__host__ __forceinline__ size_t lemma_lds(const DevPlan &p) {
    return raw_lds_bytes(0, p.n, p.G, false, false) + lemma_bytes(p.G, p.keybits);
}

// The lemma needs one CPhase layer, compressed flip-pattern keys and room for
// H.  It runs in FP64 for both precisions: its per-pattern work is an r x r
// determinant, too small for FP32 to pay, and H in FP32 loses up to
// ||M_0^-1|| more digits than the direct FP32 correction.
__host__ __forceinline__ bool lemma_applies(const DevPlan &p) {
    return p.L == 1 && p.G <= 16 && p.keykind == 0 && p.keybits >= 1 && lemma_lds(p) <= kMaxLds &&
           sampler_lds_bytes(p.k) <= kMaxLds;
}

}  // namespace
}  // namespace xf
