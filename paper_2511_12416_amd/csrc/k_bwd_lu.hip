// Adjoint kernels that differentiate through the LU evaluation: every
// distinct trajectory submatrix is recomposed and inverted (Jacobi's formula).
#include "xf_device.h"

namespace xf {
namespace {
// ---------------------------------------------------------------------------
// Adjoint (gradient of L = sum_b g_b log p_b)
//
// d log p_b = 2 Re(dA_b / A_b) and d det M = det M tr(M^-1 dM) (Jacobi), so
// every distinct entry e of bitstring b contributes the holomorphic adjoint
// Gbar_M = beta_e M_e^-T, beta_e = (g_b / A_b) c_e det M_e, which is pushed
// back through the low-rank composition M = P[R,:] - 2 A1[R,N] Phi0[N,:]:
//   Gbar_P[R_i, :]   += Gbar_M[i, :]
//   Gbar_A1[R_i, c]  += -2 Gbar_M[i, :] . Phi0[c, :]      (c in N)
//   Gbar_Phi0[c, :]  += -2 sum_i A1[R_i, c] Gbar_M[i, :]   (c in N)
// The submatrix is recomputed, not stored.  M^-1 comes from Gauss-Jordan in
// the same one-row-per-lane layout as the forward LU; an LDS tile per lane
// group turns the permuted rows of M^-1 into both the rows and the columns
// of Gbar_M.  Every lane group accumulates into its own partial buffer, in
// which each of its lanes owns the entries it adds to (its row R_i, its
// column of Phi0, its angles), so the adds are plain read-modify-writes in
// program order; a fixed-order reduction over all partials follows.  The
// result is bitwise reproducible.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void add_c(double2 *dst, double2 v) {
    dst->x += v.x;
    dst->y += v.y;
}

struct GradOut {
    double2 *P, *Phi0, *A1, *W;   // this lane group's partial (see GradLayout)
    double *gsum;
};

// One entry's adjoint, evaluated by a group of G lanes.  coef = g_b / A_b
// (times the Raw Estimate scale), ce = the entry's weight.  Adds its row of
// Gbar_M into srow (summed over entries, scattered into Gbar_P per bitstring).
// dw (exact mode, nullable): derivatives of the weight with respect to every
// angle, k values.
template <int G, bool MIXED>
__device__ __forceinline__ void adjoint_entry(const DevPlan &p, uint64_t key, double2 ce, double2 coef,
                              const double2 *dw, const uint8_t *Rb, int lane, double2 *pv,
                              double2 *tile, double2 (&srow)[G], const GradOut &go) {
    double2 det;
    int pos;
    const Flips f = decode_key(p, key);
    {
        double2 a[G], v[G];
        if (lane < p.m) {
            compose_row<G, MIXED>(p, Rb[lane], f, a);
        } else {
#pragma unroll
            for (int j = 0; j < G; ++j) a[j] = make_double2(j == lane ? 1.0 : 0.0, 0.0);
        }
        if (!gj_invert<G>(a, v, p.m, lane, pv, det, pos)) return;   // det = 0: no contribution
        if (lane < p.m) {
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (j < p.m) tile[pos * G + j] = v[j];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // weight derivatives (exact mode): dL/dtheta_j gets 2 Re(coef dw_j det)
    if (dw) {
        const double2 cd = c_mul(coef, det);
        for (int j = lane; j < p.k; j += G) add_c(go.W + j, c_mul(cd, dw[j]));
    }
    const double2 beta = c_mul(c_mul(coef, ce), det);
    if (lane < p.m) {
        double2 gr[G], gc[G];   // row `lane` and column `lane` of Gbar_M
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (j < p.m) {
                gr[j] = c_mul(beta, tile[j * G + lane]);
                gc[j] = c_mul(beta, tile[lane * G + j]);
            } else {
                gr[j] = gc[j] = make_double2(0.0, 0.0);
            }
            srow[j].x += gr[j].x;
            srow[j].y += gr[j].y;
        }
        if (p.L == 1) {
            const int Ri = Rb[lane];
            for (int w = 0; w < 2; ++w) {
                for (uint64_t mm = f.n0[w]; mm; mm &= mm - 1) {
                    const int c = 64 * w + __ffsll((long long)mm) - 1;
                    const double2 *phi = p.Phi0 + (size_t)c * G;
                    double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
#pragma unroll
                    for (int j = 0; j < G; ++j) {
                        s1 = c_fma(s1, gr[j], phi[j]);
                        if (j < p.m) s2 = c_fma(s2, p.A1[(size_t)Rb[j] * p.n + c], gc[j]);
                    }
                    add_c(go.A1 + (size_t)Ri * p.n + c, make_double2(-2.0 * s1.x, -2.0 * s1.y));
                    add_c(go.Phi0 + (size_t)c * G + lane, make_double2(-2.0 * s2.x, -2.0 * s2.y));
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Partial of lane group grp of this workgroup (kThreads / G groups each).
__device__ __forceinline__ GradOut grad_out(double2 *part, const GradLayout &L, int ngroups, int grp) {
    double2 *base = part + ((size_t)blockIdx.x * ngroups + grp) * L.stride;
    GradOut g;
    g.P = base + L.oP;
    g.Phi0 = base + L.oPhi;
    g.A1 = base + L.oA1;
    g.W = base + L.oW;
    g.gsum = (double *)(base + L.oG);
    return g;
}

template <int G>
__device__ __forceinline__ void flush_srow(const DevPlan &p, const uint8_t *Rb, int lane, double2 (&srow)[G],
                           const GradOut &go) {
    if (lane < p.m) {
        double2 *row = go.P + (size_t)Rb[lane] * G;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j < p.m) add_c(row + j, srow[j]);
    }
}

template <int G, bool MIXED>
__global__ void __launch_bounds__(kThreads)
k_raw_estimate_bwd(DevPlan p, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb, uint32_t t, uint64_t seed,
                   const double *__restrict__ g, double2 *part, GradLayout lay, const uint32_t *__restrict__ only) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_n;
    __shared__ int s_cnt[6];
    __shared__ uint64_t s_acc[kAccWords];
    const RawSmem s = carve_raw(smem, p.k, p.n, G, MIXED);
    constexpr int NG = kThreads / G;
    double2 *tiles = (double2 *)(smem + raw_lds_bytes(p.k, p.n, G, MIXED, false));
    double2 *pvs = tiles + NG * G * G;
    const int tid = threadIdx.x;
    const int lane = tid % G, grp = tid / G;
    load_tables(p, s);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t slot0 = hash_slot(0);
    const GradOut go = grad_out(part, lay, NG, grp);

    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        // with `only`, just the bitstrings the lemma backward deferred
        if (only && only[i] != kEntryDeferred) continue;
        const int64_t b = b0 + i;
        if (!load_bitstring(p, bits, b, s.Rb, &s_ok)) continue;
        const double gb = g[b];
        if (gb == 0.0) continue;
        Sampler st;
        unsigned long long blocks = 0;   // not reported here
        acc_clear(s_acc);
        clear_table(s, s_cnt, slot0, st);
        while (true) {
            const bool done = sample_until_flush(p, s, s_cnt, slot0, b, t, k0, k1, st, blocks);
            const int nl = gather_list(s, &s_n);
            Work unused;
            sum_entries<G, MIXED, false>(p, s, nl, unused, s_acc);
            if (done) break;
            clear_table(s, s_cnt, slot0, st);
        }
        const double2 total = acc_value(s_acc);
        const double ax = total.x * p.scale, ay = total.y * p.scale;
        const double a2 = ax * ax + ay * ay;
        if (a2 == 0.0) continue;
        // coef = g_b / A_b * scale
        const double2 coef = make_double2(gb * ax / a2 * p.scale, -gb * ay / a2 * p.scale);
        double2 srow[G];
#pragma unroll
        for (int j = 0; j < G; ++j) srow[j] = make_double2(0.0, 0.0);
        st = Sampler();
        clear_table(s, s_cnt, slot0, st);
        while (true) {
            const bool done = sample_until_flush(p, s, s_cnt, slot0, b, t, k0, k1, st, blocks);
            const int nl = gather_list(s, &s_n);
            for (int e = grp; e < nl; e += NG) {
                const uint16_t slot = s.list[e];
                const int2 c = s.hcnt[slot];
                adjoint_entry<G, MIXED>(p, s.hkey[slot], make_double2((double)c.x, (double)c.y), coef,
                                        nullptr, s.Rb, lane, pvs + grp * 2 * G, tiles + grp * G * G,
                                        srow, go);
            }
            __syncthreads();
            if (done) break;
            clear_table(s, s_cnt, slot0, st);
        }
        flush_srow<G>(p, s.Rb, lane, srow, go);
        if (tid == 0) *go.gsum += gb;
        __syncthreads();
    }
}

template <int G, bool MIXED>
__global__ void __launch_bounds__(kThreads)
k_exact_bwd(DevPlan p, const uint64_t *__restrict__ keys, const double2 *__restrict__ w,
            const double2 *__restrict__ dw, int64_t nkeys, const uint64_t *__restrict__ bits, int64_t B,
            const double *__restrict__ g, double2 *part, GradLayout lay) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok;
    constexpr int NG = kThreads / G;
    double2 *out = (double2 *)smem;
    double2 *piv = out + kExactChunk;
    double2 *red = piv + kThreads;
    double2 *tiles = red + kThreads;
    double2 *pvs = tiles + NG * G * G;
    uint8_t *Rb = (uint8_t *)(pvs + NG * 2 * G);
    const int tid = threadIdx.x;
    const int lane = tid % G, grp = tid / G;
    const GradOut go = grad_out(part, lay, NG, grp);
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        if (!load_bitstring(p, bits, b, Rb, &s_ok)) continue;
        const double gb = g[b];
        if (gb == 0.0) continue;
        double2 total = make_double2(0.0, 0.0);
        for (int64_t c0 = 0; c0 < nkeys; c0 += kExactChunk) {
            const int ncur = (int)min((int64_t)kExactChunk, nkeys - c0);
            for (int e = grp; e < ncur; e += NG) {
                int rank;
                const double2 d = term_det<G, MIXED>(p, keys[c0 + e], Rb, lane, piv + grp * G, &rank);
                if (lane == 0) out[e] = c_mul(w[c0 + e], d);
            }
            __syncthreads();
            const double2 ps = ordered_sum(out, ncur, red);
            total.x += ps.x;
            total.y += ps.y;
        }
        if (tid == 0) red[0] = total;
        __syncthreads();
        total = red[0];
        __syncthreads();
        const double a2 = total.x * total.x + total.y * total.y;
        if (a2 == 0.0) continue;
        const double2 coef = make_double2(gb * total.x / a2, -gb * total.y / a2);
        double2 srow[G];
#pragma unroll
        for (int j = 0; j < G; ++j) srow[j] = make_double2(0.0, 0.0);
        for (int64_t e = grp; e < nkeys; e += NG)
            adjoint_entry<G, MIXED>(p, keys[e], w[e], coef, dw + (size_t)e * p.k, Rb, lane,
                                    pvs + grp * 2 * G, tiles + grp * G * G, srow, go);
        flush_srow<G>(p, Rb, lane, srow, go);
        if (tid == 0) *go.gsum += gb;
        __syncthreads();
    }
}

template <int G, bool MIXED>
hipError_t launch_raw_bwd_t(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                            uint64_t seed, const double *g, double2 *part, int nwg, const GradLayout &lay,
                            const uint32_t *only, hipStream_t s) {
    const size_t lds = raw_estimate_bwd_lds_bytes(p, MIXED);
    hipLaunchKernelGGL((k_raw_estimate_bwd<G, MIXED>), dim3(nwg), dim3(kThreads), lds, s, p, bits, b0, nb,
                       (uint32_t)t, seed, g, part, lay, only);
    return hipGetLastError();
}

template <int G, bool MIXED>
hipError_t launch_exact_bwd_t(const DevPlan &p, const uint64_t *keys, const double2 *w, const double2 *dw,
                              int64_t nkeys, const uint64_t *bits, int64_t B, const double *g,
                              double2 *part, int nparts, const GradLayout &lay, hipStream_t s) {
    const size_t lds = exact_bwd_lds_bytes(p);
    hipLaunchKernelGGL((k_exact_bwd<G, MIXED>), dim3(nparts), dim3(kThreads), lds, s, p, keys, w, dw,
                       nkeys, bits, B, g, part, lay);
    return hipGetLastError();
}

template <int G>
hipError_t set_lds_limits_bwd() {
    const int big = (int)kMaxLds;
    hipError_t e;
    for (const void *f : {(const void *)k_raw_estimate_bwd<G, false>, (const void *)k_raw_estimate_bwd<G, true>,
                          (const void *)k_exact_bwd<G, false>, (const void *)k_exact_bwd<G, true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

size_t raw_estimate_bwd_lds_bytes(const DevPlan &p, bool mixed) {
    const size_t NG = kThreads / p.G;
    return raw_lds_bytes(p.k, p.n, p.G, mixed, false) + NG * p.G * p.G * 16 + NG * 2 * p.G * 16;
}

size_t exact_bwd_lds_bytes(const DevPlan &p) {
    const size_t NG = kThreads / p.G;
    return kExactChunk * 16 + 2 * kThreads * 16 + NG * p.G * p.G * 16 + NG * 2 * p.G * 16 + 64;
}

hipError_t launch_raw_estimate_bwd(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb,
                                   int64_t t, uint64_t seed, const double *g, double2 *part, int nwg,
                                   const GradLayout &lay, const uint32_t *only, hipStream_t s) {
    hipError_t e = hipSuccess;
#define XF_RB(GG) \
    e = mixed ? launch_raw_bwd_t<GG, true>(p, bits, b0, nb, t, seed, g, part, nwg, lay, only, s) \
              : launch_raw_bwd_t<GG, false>(p, bits, b0, nb, t, seed, g, part, nwg, lay, only, s)
    switch (p.G) {
        case 4: XF_RB(4); break;
        case 8: XF_RB(8); break;
        case 16: XF_RB(16); break;
        default: return hipErrorInvalidValue;
    }
#undef XF_RB
    return e;
}

hipError_t launch_exact_bwd(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w,
                            const double2 *dw, int64_t nkeys, const uint64_t *bits, int64_t B,
                            const double *g, double2 *part, int nparts, const GradLayout &lay,
                            hipStream_t s) {
    hipError_t e = hipSuccess;
#define XF_EB(GG) \
    e = mixed ? launch_exact_bwd_t<GG, true>(p, keys, w, dw, nkeys, bits, B, g, part, nparts, lay, s) \
              : launch_exact_bwd_t<GG, false>(p, keys, w, dw, nkeys, bits, B, g, part, nparts, lay, s)
    switch (p.G) {
        case 4: XF_EB(4); break;
        case 8: XF_EB(8); break;
        case 16: XF_EB(16); break;
        default: return hipErrorInvalidValue;
    }
#undef XF_EB
    return e;
}

hipError_t prepare_bwd(int G) {
    switch (G) {
        case 4: return set_lds_limits_bwd<4>();
        case 8: return set_lds_limits_bwd<8>();
        case 16: return set_lds_limits_bwd<16>();
    }
    return hipSuccess;
}

}  // namespace xf
