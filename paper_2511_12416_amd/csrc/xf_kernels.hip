// gfx950 kernels of the Born-rule probability path.
//
// One workgroup (four wave64s) owns one output bitstring b at a time:
//   1. Raw Estimate: every lane draws trajectories (Philox4x32-10 words fed to
//      the next-selected-gate inverse-transform table, Sec. III-B Eq. 10-12),
//      reduces each to its flip-pattern key and adds its phase i^e to a
//      Gaussian-integer counter in an LDS hash keyed by the pattern (the
//      determinant table of Sec. IV-B).  Trajectories with no d_1 choice
//      (the common case at small angles) are counted with one ballot per wave.
//      Exact: the keys and weights come from the plan's shared term list.
//   2. The distinct keys are sorted, and each is evaluated by a group of G
//      lanes (G >= eta, one row of the eta x eta submatrix per lane): the row
//      is composed by the low-rank update of Sec. IV-B Eq. 19 (two-layer form
//      for L = 2), then an LU with partial pivoting runs in registers with the
//      pivot row broadcast through LDS; det = sign * prod(pivots) in FP64.
//   3. weight * det is summed in a fixed order, so results are bitwise
//      reproducible, and p_b = |A_b|^2.
#include <hip/hip_runtime.h>

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
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t hash_slot(uint64_t key) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53) & (kHashSlots - 1);
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

// Determinant of the m x m matrix whose row `lane` (< m) is held by lane
// `lane` of a group of G consecutive lanes (rows >= m are padding).  Partial
// pivoting: the pivot of column c is the active row with the largest
// re^2 + im^2 (lowest lane on ties); rows stay in their lanes and the pivot
// row is broadcast through `piv` (G entries of LDS private to the group).
// The permutation sign is tracked by virtual row swaps.  Exactly zero pivot
// column => det = 0.  Every lane of the group returns the determinant.
template <int G>
__device__ __forceinline__ double2 lu_det(double2 (&a)[G], int m, int lane, double2 *piv) {
    bool active = lane < m;
    bool live = true;   // false once a zero pivot column was met (group-uniform)
    int pos = lane;
    bool neg = false;
    double2 det = make_double2(1.0, 0.0);
#pragma unroll
    for (int c = 0; c < G; ++c) {
        if (c < m && live) {
            double v = active ? fma(a[c].x, a[c].x, a[c].y * a[c].y) : -1.0;
            int idx = lane;
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const double vo = __shfl_xor(v, off, G);
                const int io = __shfl_xor(idx, off, G);
                if (vo > v || (vo == v && io < idx)) {
                    v = vo;
                    idx = io;
                }
            }
            if (v > 0.0) {
                const int ppos = __shfl(pos, idx, G);
                neg ^= (ppos != c);
                if (pos == c) pos = ppos;
                if (lane == idx) {
                    pos = c;
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
    return neg ? make_double2(-det.x, -det.y) : det;
}

// det of the trajectory submatrix for `key`, evaluated by a group of G lanes.
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

// Loads bitstring b; returns false (and writes p = 0) if its weight is not
// eta or it has bits at or above n.  Fills Rb with the occupied modes.
__device__ bool load_bitstring(const DevPlan &p, const uint64_t *bits, int64_t b, uint8_t *Rb,
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
    return *s_ok != 0;
}

// Fixed-order sum of out[0..cnt): each thread adds a contiguous chunk, then a
// fixed tree over the workgroup.  Result valid in thread 0.
__device__ double2 ordered_sum(const double2 *out, int cnt, double2 *red) {
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

struct RawSmem {
    double2 *out;
    uint64_t *hkey;
    int2 *hcnt;
    double2 *piv;
    double2 *red;
    uint16_t *list;
    uint8_t *Rb;
    uint64_t *gkey;
    uint8_t *gneg;
    uint32_t *T;
};

__device__ __forceinline__ RawSmem carve_raw(unsigned char *smem, int k) {
    RawSmem s;
    s.out = (double2 *)smem;
    s.hkey = (uint64_t *)(s.out + kHashSlots);
    s.hcnt = (int2 *)(s.hkey + kHashSlots);
    s.piv = (double2 *)(s.hcnt + kHashSlots);
    s.red = s.piv + kThreads;
    s.list = (uint16_t *)(s.red + kThreads);
    s.Rb = (uint8_t *)(s.list + kHashSlots);
    s.gkey = (uint64_t *)(s.Rb + 64);
    s.gneg = (uint8_t *)(s.gkey + k);
    s.T = (uint32_t *)(s.gneg + ((k + 7) & ~7));
    return s;
}

__device__ __forceinline__ uint64_t list_key(const RawSmem &s, uint16_t idx) {
    return idx == 0xFFFFu ? kEmptyKey : s.hkey[idx];
}

// Sorts, evaluates and sums the current hash content; clears the table and
// re-reserves the empty pattern.  Called by the whole workgroup.
template <int G, bool MIXED>
__device__ double2 flush_table(const DevPlan &p, const RawSmem &s, int *s_n, int *s_claimed,
                               int slot0, unsigned long long *nterm) {
    const int tid = threadIdx.x;
    if (tid == 0) *s_n = 0;
    __syncthreads();
    for (int i = tid; i < kHashSlots; i += kThreads) {
        if (s.hkey[i] != kEmptyKey && (s.hcnt[i].x != 0 || s.hcnt[i].y != 0))
            s.list[atomicAdd(s_n, 1)] = (uint16_t)i;
    }
    __syncthreads();
    const int nl = *s_n;
    int np = 1;
    while (np < nl) np <<= 1;
    for (int i = nl + tid; i < np; i += kThreads) s.list[i] = 0xFFFFu;
    __syncthreads();
    // bitonic sort of slot indices by key (keys are distinct)
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < (np >> 1); i += kThreads) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint16_t a = s.list[lo], b = s.list[hi];
                if ((list_key(s, a) > list_key(s, b)) == asc) {
                    s.list[lo] = b;
                    s.list[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    const int lane = tid % G, grp = tid / G;
    constexpr int NG = kThreads / G;
    unsigned rank_sum = 0;
    for (int e = grp; e < nl; e += NG) {
        const uint16_t slot = s.list[e];
        int rank;
        const double2 d = term_det<G, MIXED>(p, s.hkey[slot], s.Rb, lane, s.piv + grp * G, &rank);
        if (lane == 0) {
            const int2 c = s.hcnt[slot];
            s.out[e] = make_double2((double)c.x * d.x - (double)c.y * d.y,
                                    (double)c.x * d.y + (double)c.y * d.x);
            rank_sum += (unsigned)rank;
        }
    }
    __syncthreads();
    const double2 sum = ordered_sum(s.out, nl, s.red);
    if (nterm) {
        if (tid == 0) atomicAdd(nterm, (unsigned long long)nl);
        if (lane == 0 && rank_sum) atomicAdd(nterm + 1, (unsigned long long)rank_sum);
    }
    for (int i = tid; i < kHashSlots; i += kThreads) {
        s.hkey[i] = kEmptyKey;
        s.hcnt[i] = make_int2(0, 0);
    }
    __syncthreads();
    if (tid == 0) {
        s.hkey[slot0] = 0;
        *s_claimed = 1;
    }
    __syncthreads();
    return sum;
}

template <int G, bool MIXED>
__global__ void __launch_bounds__(kThreads)
k_raw_estimate(DevPlan p, const uint64_t *__restrict__ bits, int64_t B, uint32_t t, uint64_t seed,
               double *__restrict__ prob, double *__restrict__ amp, unsigned long long *nterm) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_n, s_claimed;
    const RawSmem s = carve_raw(smem, p.k);
    const int tid = threadIdx.x;
    const int k = p.k;
    for (int i = tid; i < k * k; i += kThreads) s.T[i] = p.T[i];
    for (int i = tid; i < k; i += kThreads) {
        s.gkey[i] = p.gkey[i];
        s.gneg[i] = p.gneg[i];
    }
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t slot0 = hash_slot(0);

    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        if (!load_bitstring(p, bits, b, s.Rb, &s_ok)) {
            if (tid == 0) {
                prob[b] = 0.0;
                if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
            }
            __syncthreads();
            continue;
        }
        for (int i = tid; i < kHashSlots; i += kThreads) {
            s.hkey[i] = kEmptyKey;
            s.hcnt[i] = make_int2(0, 0);
        }
        __syncthreads();
        if (tid == 0) {
            s.hkey[slot0] = 0;
            s_claimed = 1;
        }
        __syncthreads();

        double2 total = make_double2(0.0, 0.0);
        const uint32_t blo = (uint32_t)b, bhi = (uint32_t)((uint64_t)b >> 32);
        for (uint32_t base = 0; base < t; base += kThreads) {
            if (s_claimed + kThreads > (3 * kHashSlots) / 4) {
                const double2 part = flush_table<G, MIXED>(p, s, &s_n, &s_claimed, slot0, nterm);
                total.x += part.x;
                total.y += part.y;
            }
            const uint32_t smp = base + tid;
            const bool valid = smp < t;
            uint64_t key = 0;
            uint32_t e = 0;
            bool empty = true;
            if (valid && k > 0) {
                uint32_t blk = 0;
                uint4 r = philox10(make_uint4(smp, 0u, blo, bhi), k0, k1);
                uint32_t d = 0;
                int a = 0;
                while (a < k) {
                    if ((d >> 2) != blk) {
                        blk = d >> 2;
                        r = philox10(make_uint4(smp, blk, blo, bhi), k0, k1);
                    }
                    const uint32_t w = d & 3;
                    const uint32_t u = w == 0 ? r.x : (w == 1 ? r.y : (w == 2 ? r.z : r.w));
                    ++d;
                    const uint32_t *Ta = s.T + a * k;
                    if (!(u < Ta[k - 1])) break;
                    int lo = a, hi = k - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (u < Ta[mid]) hi = mid;
                        else lo = mid + 1;
                    }
                    key ^= s.gkey[lo];
                    e += 1u + 2u * s.gneg[lo];
                    empty = false;
                    a = lo + 1;
                }
            }
            const unsigned long long ball = __ballot(valid && empty);
            if ((tid & 63) == 0 && ball) atomicAdd(&s.hcnt[slot0].x, (int)__popcll(ball));
            if (valid && !empty) {
                uint32_t slot = hash_slot(key);
                while (true) {
                    const unsigned long long prev =
                        atomicCAS((unsigned long long *)&s.hkey[slot], (unsigned long long)kEmptyKey,
                                  (unsigned long long)key);
                    if (prev == kEmptyKey) {
                        atomicAdd(&s_claimed, 1);
                        break;
                    }
                    if (prev == key) break;
                    slot = (slot + 1) & (kHashSlots - 1);
                }
                e &= 3;
                if (e == 0) atomicAdd(&s.hcnt[slot].x, 1);
                else if (e == 1) atomicAdd(&s.hcnt[slot].y, 1);
                else if (e == 2) atomicAdd(&s.hcnt[slot].x, -1);
                else atomicAdd(&s.hcnt[slot].y, -1);
            }
            __syncthreads();
        }
        const double2 part = flush_table<G, MIXED>(p, s, &s_n, &s_claimed, slot0, nterm);
        total.x += part.x;
        total.y += part.y;
        if (tid == 0) {
            const double ax = total.x * p.scale, ay = total.y * p.scale;
            prob[b] = ax * ax + ay * ay;
            if (amp) { amp[2 * b] = ax; amp[2 * b + 1] = ay; }
        }
        __syncthreads();
    }
}

template <int G, bool MIXED>
__global__ void __launch_bounds__(kThreads)
k_exact(DevPlan p, const uint64_t *__restrict__ keys, const double2 *__restrict__ w, int64_t nkeys,
        const uint64_t *__restrict__ bits, int64_t B, double *__restrict__ prob,
        double *__restrict__ amp, unsigned long long *nterm) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok;
    double2 *out = (double2 *)smem;
    double2 *piv = out + kExactChunk;
    double2 *red = piv + kThreads;
    uint8_t *Rb = (uint8_t *)(red + kThreads);
    const int tid = threadIdx.x;
    const int lane = tid % G, grp = tid / G;
    constexpr int NG = kThreads / G;
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        if (!load_bitstring(p, bits, b, Rb, &s_ok)) {
            if (tid == 0) {
                prob[b] = 0.0;
                if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
            }
            __syncthreads();
            continue;
        }
        double2 total = make_double2(0.0, 0.0);
        unsigned rank_sum = 0;
        for (int64_t c0 = 0; c0 < nkeys; c0 += kExactChunk) {
            const int ncur = (int)min((int64_t)kExactChunk, nkeys - c0);
            for (int e = grp; e < ncur; e += NG) {
                int rank;
                const double2 d = term_det<G, MIXED>(p, keys[c0 + e], Rb, lane, piv + grp * G, &rank);
                if (lane == 0) {
                    out[e] = c_mul(w[c0 + e], d);
                    rank_sum += (unsigned)rank;
                }
            }
            __syncthreads();
            const double2 part = ordered_sum(out, ncur, red);
            total.x += part.x;
            total.y += part.y;
        }
        if (tid == 0) {
            prob[b] = total.x * total.x + total.y * total.y;
            if (amp) { amp[2 * b] = total.x; amp[2 * b + 1] = total.y; }
            if (nterm) atomicAdd(nterm, (unsigned long long)nkeys);
        }
        if (nterm && lane == 0 && rank_sum) atomicAdd(nterm + 1, (unsigned long long)rank_sum);
        __syncthreads();
    }
}

__global__ void k_zero_u64(unsigned long long *p) {
    p[0] = 0ull;
    p[1] = 0ull;
}

constexpr int kMaxGrid = 1 << 20;

template <int G, bool MIXED>
hipError_t launch_raw_t(const DevPlan &p, const uint64_t *bits, int64_t B, int64_t t, uint64_t seed,
                        double *prob, double *amp, unsigned long long *nterm, hipStream_t s) {
    const size_t lds = raw_estimate_lds_bytes(p);
    const int grid = (int)(B < kMaxGrid ? B : kMaxGrid);
    hipLaunchKernelGGL((k_raw_estimate<G, MIXED>), dim3(grid), dim3(kThreads), lds, s, p, bits, B,
                       (uint32_t)t, seed, prob, amp, nterm);
    return hipGetLastError();
}

template <int G, bool MIXED>
hipError_t launch_exact_t(const DevPlan &p, const uint64_t *keys, const double2 *w, int64_t nkeys,
                          const uint64_t *bits, int64_t B, double *prob, double *amp,
                          unsigned long long *nterm, hipStream_t s) {
    const size_t lds = exact_lds_bytes(p);
    const int grid = (int)(B < kMaxGrid ? B : kMaxGrid);
    hipLaunchKernelGGL((k_exact<G, MIXED>), dim3(grid), dim3(kThreads), lds, s, p, keys, w, nkeys,
                       bits, B, prob, amp, nterm);
    return hipGetLastError();
}

template <int G>
hipError_t set_lds_limits() {
    const int big = 160 * 1024 - 1024;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_raw_estimate<G, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_raw_estimate<G, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_exact<G, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)k_exact<G, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace

size_t raw_estimate_lds_bytes(const DevPlan &p) {
    const size_t k = (size_t)p.k;
    return kHashSlots * (16 + 8 + 8 + 2) + 2 * kThreads * 16 + 64 + k * 8 + ((k + 7) & ~(size_t)7) +
           k * k * 4;
}

size_t exact_lds_bytes(const DevPlan &) { return kExactChunk * 16 + 2 * kThreads * 16 + 64; }

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

hipError_t prepare_kernels(int G) {
    switch (G) {
        case 4: return set_lds_limits<4>();
        case 8: return set_lds_limits<8>();
        case 16: return set_lds_limits<16>();
        case 32: return set_lds_limits<32>();
        case 64: return set_lds_limits<64>();
    }
    return hipErrorInvalidValue;
}

#define XF_DISPATCH_G(G, CALL) \
    switch (G) {               \
        case 4: CALL(4); break; \
        case 8: CALL(8); break; \
        case 16: CALL(16); break; \
        case 32: CALL(32); break; \
        case 64: CALL(64); break; \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_raw_estimate(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t B,
                               int64_t t, uint64_t seed, double *prob, double *amp,
                               unsigned long long *nterm, hipStream_t s) {
    hipError_t e = hipSuccess;
#define XF_RAW(GG) \
    e = mixed ? launch_raw_t<GG, true>(p, bits, B, t, seed, prob, amp, nterm, s) \
              : launch_raw_t<GG, false>(p, bits, B, t, seed, prob, amp, nterm, s)
    XF_DISPATCH_G(p.G, XF_RAW)
#undef XF_RAW
    return e;
}

hipError_t launch_exact(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w,
                        int64_t nkeys, const uint64_t *bits, int64_t B, double *prob, double *amp,
                        unsigned long long *nterm, hipStream_t s) {
    hipError_t e = hipSuccess;
#define XF_EX(GG) \
    e = mixed ? launch_exact_t<GG, true>(p, keys, w, nkeys, bits, B, prob, amp, nterm, s) \
              : launch_exact_t<GG, false>(p, keys, w, nkeys, bits, B, prob, amp, nterm, s)
    XF_DISPATCH_G(p.G, XF_EX)
#undef XF_EX
    return e;
}

}  // namespace xf
