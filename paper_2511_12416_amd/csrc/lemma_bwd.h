// Adjoint under the determinant lemma (one CPhase layer, eta <= 16).
//
// With M_0 = P[R, :], X = M_0^-1 A1[R, act], Y = Phi0[act, :] M_0^-1 and
// H = Y A1[R, act] = Phi0[act, :] X, every distinct pattern e of bitstring b
// (count c_e, flipped positions N_e) has det M_e = det M_0 det S_e with
// S_e = I - 2 H[N_e, N_e].  By Jacobi's formula (d det S = tr(adj(S) dS)),
// the unscaled sum A = sum_e c_e det M_e has the holomorphic adjoints
//   Gbar_H[n_i, n_j] = -2 det M_0 sum_e c_e adj(S_e)[j][i],
//   Gbar_M0 = A M_0^-T - Y^T Gbar_H X^T,
//   Gbar_A1[R, act] = Y^T Gbar_H,   Gbar_Phi0[act, :] = Gbar_H X^T,
// since dH = dPhi0_a X + Y dA1_a - Y dM_0 X.  With coef = g_b / A (the Raw
// Estimate scale cancels in d log |A|^2), the bitstring adds coef times these
// to Gbar_P[R, :], Gbar_A1 and Gbar_Phi0.
//
// The sum over patterns of c_e adj(S_e) is accumulated exactly: every value
// is split into a multiple of 2^-16 and a remainder in units of 2^-60, both
// added as 64-bit integers with LDS atomics, so the result does not depend on
// the order in which lanes add their patterns.  Each workgroup adds its
// bitstrings' adjoints into its own partial buffer in a fixed order; a
// fixed-order reduction over the workgroups follows.  The backward is
// therefore bitwise reproducible.
#pragma once
#include "xf_device.h"

namespace xf {
namespace {

// Units of the two integer words of an exactly accumulated real value.
constexpr double kFxHi = 65536.0;                  // 2^16
constexpr double kFxLo = 1152921504606846976.0;    // 2^60
constexpr int kFxFoldShift = 44;                   // 2^60 / 2^16
// Largest |adj(S)| component accepted: with counts summing to at most
// t < 2^31 in modulus, the high words stay below 2^16 2^31 2^15 = 2^62.
constexpr double kFxMaxAdj = 32768.0;

// w[0] += round(v 2^16), w[1] += round((v - that) 2^60).  The remainder is
// exact in FP64; the rounding error is below 2^-61.
__device__ __forceinline__ void fx_add(unsigned long long *w, double v) {
    const double h = rint(v * kFxHi);
    const double rem = v - h * (1.0 / kFxHi);
    const double l = rint(rem * kFxLo);
    atomicAdd(&w[0], (unsigned long long)(long long)h);
    atomicAdd(&w[1], (unsigned long long)(long long)l);
}

// Moves the multiples of 2^44 of the low word into the high word (single
// owner, between barriers).
__device__ __forceinline__ void fx_fold(unsigned long long *w) {
    const long long lo = (long long)w[1];
    const long long q = lo >> kFxFoldShift;
    w[0] = (unsigned long long)((long long)w[0] + q);
    w[1] = (unsigned long long)(lo - (q * (1ll << kFxFoldShift)));
}

__device__ __forceinline__ double fx_value(const unsigned long long *w) {
    return (double)(long long)w[0] * (1.0 / kFxHi) + (double)(long long)w[1] * (1.0 / kFxLo);
}

// Adds c * a to the accumulator of Gbar_H[row][col] (4 words: re hi, re lo,
// im hi, im lo).  Returns false if a component of a exceeds kFxMaxAdj.
__device__ __forceinline__ bool fx_add_c(unsigned long long *acc, int kb, int row, int col, int2 c, double2 a) {
    if (!(fabs(a.x) <= kFxMaxAdj && fabs(a.y) <= kFxMaxAdj)) return false;
    const double2 v = c_mul(make_double2((double)c.x, (double)c.y), a);
    unsigned long long *w = acc + 4 * ((size_t)row * kb + col);
    fx_add(w, v.x);
    fx_add(w + 2, v.y);
    return true;
}

// Determinant and adjugate of S = I - 2 H[N, N] for the r <= kLemmaMaxRank
// set bits of key (one lane).  Gauss-Jordan on [S | I] with the pivot rule of
// lemma_small_det: the rows below the pivot are updated with the same
// expressions, so the pivots, and the determinant, are those of
// lemma_small_det.  The left half ends diagonal (u_c) and the right half is
// E with E S = diag(u); adj(S) = det(S) S^-1 has rows
// sign * prod_{c' != c} u_c' * E[c, :], formed without dividing by a pivot.
// Returns false (det = 0, adj unset) for an exactly singular S.
__device__ __forceinline__ bool lemma_small_adj(uint64_t key, const double2 *sH, int kb, int (&pos)[kLemmaMaxRank],
                                                int &r, double2 &det, double2 (&adj)[kLemmaMaxRank][kLemmaMaxRank]) {
    constexpr int RM = kLemmaMaxRank;
    uint64_t mm = key;
    r = 0;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        pos[i] = mm ? __ffsll((long long)mm) - 1 : 0;
        if (mm) ++r;
        mm &= mm - 1;
    }
    double2 a[RM][RM], e[RM][RM];
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
            e[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        }
    bool neg = false;
    double2 u[RM];
    det = make_double2(1.0, 0.0);
#pragma unroll
    for (int c = 0; c < RM; ++c) {
        u[c] = make_double2(1.0, 0.0);
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
            if (!(best > 0.0)) {
                det = make_double2(0.0, 0.0);
                return false;
            }
            neg ^= piv != c;
#pragma unroll
            for (int i = c + 1; i < RM; ++i) {
                if (piv == i) {
#pragma unroll
                    for (int j = 0; j < RM; ++j) {
                        double2 t = a[c][j];
                        a[c][j] = a[i][j];
                        a[i][j] = t;
                        t = e[c][j];
                        e[c][j] = e[i][j];
                        e[i][j] = t;
                    }
                }
            }
            u[c] = a[c][c];
            det = c_mul(det, a[c][c]);
            const double inv = 1.0 / best;
            const double2 ui = make_double2(-a[c][c].x * inv, a[c][c].y * inv);
#pragma unroll
            for (int i = 0; i < RM; ++i) {
                if (i != c && i < r) {
                    const double2 l = c_mul(a[i][c], ui);
#pragma unroll
                    for (int j = c + 1; j < RM; ++j) a[i][j] = c_fma(a[i][j], l, a[c][j]);
#pragma unroll
                    for (int j = 0; j < RM; ++j) e[i][j] = c_fma(e[i][j], l, e[c][j]);
                }
            }
        }
    }
    if (neg) det = make_double2(-det.x, -det.y);
#pragma unroll
    for (int c = 0; c < RM; ++c) {
        double2 f = make_double2(neg ? -1.0 : 1.0, 0.0);
#pragma unroll
        for (int c2 = 0; c2 < RM; ++c2)
            if (c2 != c && c2 < r) f = c_mul(f, u[c2]);
#pragma unroll
        for (int j = 0; j < RM; ++j) adj[c][j] = c_mul(f, e[c][j]);
    }
    return true;
}

// Positions (bit indices) of the first GS set bits of key, in ascending order.
template <int GS>
__device__ __forceinline__ void key_positions(uint64_t key, int (&q)[GS]) {
    uint64_t mm = key;
#pragma unroll
    for (int i = 0; i < GS; ++i) {
        q[i] = mm ? __ffsll((long long)mm) - 1 : 0;
        mm &= mm - 1;
    }
}

// Bytes of LDS beyond lemma_lds(p) that k_bwd_entries uses: M_0^-1 (G x G),
// X (G x kb), Y (kb x G), the exact Gbar_H accumulator (kb x kb x 4 words)
// and the lane-group Gauss-Jordan scratch (2 x 256 entries).
__host__ __device__ __forceinline__ size_t bwd_lemma_extra(int G, int kb) {
    return (size_t)G * G * 16 + (size_t)G * kb * 16 + (size_t)kb * G * 16 + (size_t)kb * kb * 32 +
           2 * (size_t)kThreads * 16;
}

// One group-evaluated pattern (r in (kLemmaMaxRank, GS]): Gauss-Jordan of S
// by GS lanes (lane i ends with row pos_i of S^-1), adj = det S^-1 added for
// the group's rows.  Returns the determinant of S (0 if exactly singular).
template <int GS>
__device__ __forceinline__ double2 group_adjugate(uint64_t key, int r, int lane, const double2 *sH, int kb,
                                                  int2 c, double2 *pv, unsigned long long *gacc, bool &bad) {
    double2 a[GS], v[GS], dS;
    int gp, q[GS];
    lemma_rows<GS>(key, r, lane, sH, kb, a);
    key_positions<GS>(key, q);
    const bool nonsingular = gj_invert<GS>(a, v, r, lane, pv, dS, gp);
    if (!nonsingular) return make_double2(0.0, 0.0);
    if (lane < r) {
        // this lane holds row gp of S^-1: adj[gp][j] goes to Gbar_H[n_j][n_gp]
        int pr = 0;
#pragma unroll
        for (int j = 0; j < GS; ++j)
            if (j == gp) pr = q[j];
#pragma unroll
        for (int j = 0; j < GS; ++j)
            if (j < r) bad |= !fx_add_c(gacc, kb, q[j], pr, c, c_mul(dS, v[j]));
    }
    return dS;
}

// One table (nl entries in the hash slots) of a bitstring: count * det M_e of
// every entry goes into its slot (summed afterwards as in the forward pass)
// and c_e adj(S_e) into the Gbar_H accumulator.  Returns false if a pattern
// is larger than the lane groups take (the bitstring is then left to the LU
// backward); sets *s_bad for an adjugate entry outside the accumulator range
// (the bitstring is then left to the LU backward as well).
template <int G>
__device__ __forceinline__ bool bwd_entries_lemma(const DevPlan &p, const RawSmem &s, int nl, const double2 *sH,
                                                  const LemmaBits &lb, unsigned long long *gacc,
                                                  double2 *gpv, int *s_bad, uint64_t *sacc) {
    const int tid = threadIdx.x;
    const int kb = p.keybits;
    int *cnt = (int *)s.red;
    uint16_t *order = (uint16_t *)s.piv;
    uint16_t *mid = (uint16_t *)s.red + 32;
    constexpr int kMidCap = (kThreads * 16 - 64) / 2;
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
    bool bad = false;
    for (int i = tid; i < n_easy; i += kThreads) {
        const uint16_t slot = order[i];
        const uint64_t key = s.hkey[slot];
        const int2 c = s.hcnt[slot];
        int pos[kLemmaMaxRank], r;
        double2 dS, adj[kLemmaMaxRank][kLemmaMaxRank];
        const bool nonsingular = lemma_small_adj(key, sH, kb, pos, r, dS, adj);
        const double2 d = c_mul(lb.detB, dS);
        if (nonsingular) {
#pragma unroll
            for (int a = 0; a < kLemmaMaxRank; ++a)
#pragma unroll
                for (int b2 = 0; b2 < kLemmaMaxRank; ++b2)
                    if (a < r && b2 < r) bad |= !fx_add_c(gacc, kb, pos[b2], pos[a], c, adj[a][b2]);
        }
        s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
        *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
    }
    __syncthreads();
    {
        const int l8 = tid & 7, g8 = tid >> 3;
        for (int i = g8; i < n_mid; i += kThreads / 8) {
            const uint16_t slot = mid[i];
            const uint64_t key = s.hkey[slot];
            const int2 c = s.hcnt[slot];
            const double2 dS = group_adjugate<kLemmaMid>(key, __popcll(key), l8, sH, kb, c,
                                                         gpv + g8 * 2 * kLemmaMid, gacc, bad);
            const double2 d = c_mul(lb.detB, dS);
            if (l8 == 0) {
                s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
                *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
            }
        }
        __syncthreads();
    }
    if constexpr (G > kLemmaMid) {
        const int lane = tid % G, grp = tid / G;
        for (int i = n_mid + grp; i < n_mid + n_hard; i += kThreads / G) {
            const uint16_t slot = mid[i];
            const uint64_t key = s.hkey[slot];
            const int2 c = s.hcnt[slot];
            const double2 dS = group_adjugate<G>(key, __popcll(key), lane, sH, kb, c, gpv + grp * 2 * G, gacc, bad);
            const double2 d = c_mul(lb.detB, dS);
            if (lane == 0) {
                s.hkey[slot] = (uint64_t)__double_as_longlong((double)c.x * d.x - (double)c.y * d.y);
                *(double *)&s.hcnt[slot] = (double)c.x * d.y + (double)c.y * d.x;
            }
        }
        __syncthreads();
    }
    if (bad) *s_bad = 1;
    accumulate_slots(s, nl, sacc);
    // fold the low words (at most kHashSlots entries were added since the last fold)
    for (int e = tid; e < 2 * kb * kb; e += kThreads) fx_fold(gacc + 2 * e);
    __syncthreads();
    return true;
}

template <int G>
__global__ void __launch_bounds__(kThreads, 1)
k_bwd_entries(DevPlan p, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb,
              const uint64_t *__restrict__ ekey, const int2 *__restrict__ ecnt, uint32_t *__restrict__ ecount,
              uint64_t cap, const double *__restrict__ g, double2 *__restrict__ part, GradLayout lay) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_flag[2], s_bad;
    __shared__ double2 s_det;
    __shared__ uint64_t s_acc[kAccWords];
    const RawSmem s = carve_raw(smem, 0, p.n, G, false);
    const int m = p.m, n = p.n, kb = p.keybits;
    double2 *sH = (double2 *)((unsigned char *)s.sP + (size_t)G * G * 16);
    unsigned char *ext = (unsigned char *)sH + align16((size_t)kb * kb * 16);
    double2 *sV = (double2 *)ext;                                             // G x G: M_0^-1
    double2 *sX = sV + G * G;                                                 // G x kb
    double2 *sY = sX + (size_t)G * kb;                                        // kb x G
    unsigned long long *gacc = (unsigned long long *)(sY + (size_t)kb * G);   // kb x kb x 4
    double2 *gpv = (double2 *)(gacc + 4 * (size_t)kb * kb);                  // 2 x kThreads
    const int tid = threadIdx.x;
    double2 *gp = part + (size_t)blockIdx.x * lay.stride;
    Work wk;
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = b0 + i;
        const uint32_t ne = ecount[i];
        // wrong weight, or patterns that overflowed the workspace region (the
        // LU backward resamples those)
        if (ne == kEntryInvalid || ne == kEntryDeferred) continue;
        const double gb = g[b];
        if (gb == 0.0) continue;
        load_bitstring(p, bits, b, s.Rb, &s_ok);
        const LemmaBits lb = lemma_setup<G>(p, s, sH, s_flag, &s_det, wk);
        if (!lb.ok) {
            if (tid == 0) ecount[i] = kEntryDeferred;
            __syncthreads();
            continue;
        }
        // keep M_0^-1 and X (in the hash keys until the entries arrive), form Y
        const double2 *V = (const double2 *)s.hkey;
        const double2 *X = V + G * G;
        for (int e = tid; e < m * G; e += kThreads) sV[e] = V[e];
        for (int e = tid; e < m * kb; e += kThreads) sX[e] = X[e];
        for (int e = tid; e < kb * m; e += kThreads) {
            const int q = e / m, j = e % m;
            const double2 *phi = p.Phi0 + (size_t)p.keymode[q] * G;
            double2 acc = make_double2(0.0, 0.0);
            for (int l = 0; l < m; ++l) acc = c_fma(acc, phi[l], V[l * G + j]);
            sY[q * G + j] = acc;
        }
        for (int e = tid; e < 4 * kb * kb; e += kThreads) gacc[e] = 0ull;
        if (tid == 0) s_bad = 0;
        acc_clear(s_acc);
        __syncthreads();
        bool ok = true;
        const uint64_t *kin = ekey + (size_t)i * cap;
        const int2 *cin = ecnt + (size_t)i * cap;
        for (uint32_t c0 = 0; ok && c0 < ne; c0 += kHashSlots) {
            const int nc = (int)min((uint32_t)kHashSlots, ne - c0);
            for (int e = tid; e < nc; e += kThreads) {
                s.hkey[e] = kin[c0 + e];
                s.hcnt[e] = cin[c0 + e];
                s.list[e] = (uint16_t)e;
            }
            __syncthreads();
            ok = bwd_entries_lemma<G>(p, s, nc, sH, lb, gacc, gpv, &s_bad, s_acc);
        }
        if (!ok || s_bad) {
            // a pattern larger than the lane groups, or an adjugate entry
            // outside the exact accumulator's range: the LU backward takes it
            if (tid == 0) ecount[i] = kEntryDeferred;
            __syncthreads();
            continue;
        }
        const double2 A = acc_value(s_acc);
        const double a2 = A.x * A.x + A.y * A.y;
        if (a2 == 0.0) {
            __syncthreads();
            continue;
        }
        // coef = g_b / A; phi = -2 det M_0 coef; Gbar_H = phi * accumulator
        const double2 coef = make_double2(gb * A.x / a2, -gb * A.y / a2);
        const double2 phi = c_mul(make_double2(-2.0 * lb.detB.x, -2.0 * lb.detB.y), coef);
        double2 *GH = sH;   // H is no longer needed
        for (int e = tid; e < kb * kb; e += kThreads) {
            const unsigned long long *w = gacc + 4 * (size_t)e;
            GH[e] = c_mul(phi, make_double2(fx_value(w), fx_value(w + 2)));
        }
        __syncthreads();
        // Z = Gbar_H X^T (kb x m): the Phi0[act, :] adjoint, kept in the hash keys
        double2 *Z = (double2 *)s.hkey;
        for (int e = tid; e < kb * m; e += kThreads) {
            const int q = e / m, j = e % m;
            double2 acc = make_double2(0.0, 0.0);
            for (int q2 = 0; q2 < kb; ++q2) acc = c_fma(acc, GH[q * kb + q2], sX[j * kb + q2]);
            Z[q * m + j] = acc;
            double2 *dst = gp + lay.oPhi + (size_t)p.keymode[q] * G + j;
            dst->x += acc.x;
            dst->y += acc.y;
        }
        __syncthreads();
        // Gbar_A1[R_l, act_q'] += (Y^T Gbar_H)[l][q']
        for (int e = tid; e < m * kb; e += kThreads) {
            const int l = e / kb, q2 = e % kb;
            double2 acc = make_double2(0.0, 0.0);
            for (int q = 0; q < kb; ++q) acc = c_fma(acc, sY[q * G + l], GH[q * kb + q2]);
            double2 *dst = gp + lay.oA1 + (size_t)s.Rb[l] * n + p.keymode[q2];
            dst->x += acc.x;
            dst->y += acc.y;
        }
        // Gbar_P[R_i, j] += g_b M_0^-1[j][i] - (Y^T Z)[i][j]
        for (int e = tid; e < m * m; e += kThreads) {
            const int i2 = e / m, j = e % m;
            double2 acc = make_double2(0.0, 0.0);
            for (int q = 0; q < kb; ++q) acc = c_fma(acc, sY[q * G + i2], Z[q * m + j]);
            const double2 v = sV[j * G + i2];
            double2 *dst = gp + lay.oP + (size_t)s.Rb[i2] * G + j;
            dst->x += gb * v.x - acc.x;
            dst->y += gb * v.y - acc.y;
        }
        if (tid == 0) gp[lay.oG].x += gb;
        __syncthreads();
    }
}

}  // namespace
}  // namespace xf
