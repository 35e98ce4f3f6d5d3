// Fused per-bitstring kernels that factorise every distinct trajectory
// submatrix directly (the paper's per-pattern determinant, Sec. IV-B Eq. 19
// and Sec. V-B): Raw Estimate with sampling and evaluation in one kernel, and
// exact mode over the plan's shared term list.  Used where the determinant
// lemma does not apply, when the LU evaluation is selected, and for the
// bitstrings the lemma kernels defer.
#include "xf_device.h"

namespace xf {
namespace {
// Raw Estimate with the LU per distinct pattern, sampling and evaluation fused
// per bitstring.  KIND: 0 = factors read from global memory, 1 = the
// bitstring's factor rows staged in LDS.  Up to G = 16 the LDS footprint
// allows two workgroups per CU; registers are capped to match (a few
// loop-invariant values spill around the bitstring loop).
template <int G, bool MIXED, int KIND>
__global__ void __launch_bounds__(kThreads, G <= 16 ? 2 : 1)
k_raw_estimate(DevPlan p, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb, uint32_t t, uint64_t seed,
               double *__restrict__ prob, double *__restrict__ amp, double *__restrict__ logp,
               unsigned long long *nterm, const uint32_t *__restrict__ only) {
    constexpr bool STAGE = KIND == 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_n;
    __shared__ int s_cnt[6];
    __shared__ uint64_t s_acc[kAccWords];
    const RawSmem s = carve_raw(smem, p.k, p.n, G, MIXED);
    const int tid = threadIdx.x;
    Work wk;
    bool loaded = false;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t slot0 = hash_slot(0);

    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        // with `only`, just the bitstrings the lemma kernels deferred
        if (only && only[i] != kEntryDeferred) continue;
        const int64_t b = b0 + i;
        if (!loaded) {
            load_tables(p, s);
            if constexpr (STAGE) stage_phi<MIXED>(p, s);
            loaded = true;
        }
        if (!load_bitstring(p, bits, b, s.Rb, &s_ok)) {
            if (tid == 0) {
                prob[b] = 0.0;
                if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
                if (logp) logp[b] = -INFINITY;
            }
            __syncthreads();
            continue;
        }
        if constexpr (STAGE) stage_rows<MIXED>(p, s);
        Sampler st;
        unsigned long long blocks = 0;   // not reported here
        acc_clear(s_acc);
        clear_table(s, s_cnt, slot0, st);
        while (true) {
            const bool done = sample_until_flush(p, s, s_cnt, slot0, b, t, k0, k1, st, blocks);
            const int nl = gather_list(s, &s_n);
            sum_entries<G, MIXED, STAGE>(p, s, nl, wk, s_acc);
            if (done) break;
            clear_table(s, s_cnt, slot0, st);
        }
        const double2 total = acc_value(s_acc);
        if (tid == 0) {
            const double ax = total.x * p.scale, ay = total.y * p.scale;
            const double pb = ax * ax + ay * ay;
            prob[b] = pb;
            if (amp) { amp[2 * b] = ax; amp[2 * b + 1] = ay; }
            if (logp) logp[b] = log(pb);
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

template <int G, bool MIXED>
__global__ void __launch_bounds__(kThreads)
k_exact(DevPlan p, const uint64_t *__restrict__ keys, const double2 *__restrict__ w, int64_t nkeys,
        const uint64_t *__restrict__ bits, int64_t B, double *__restrict__ prob,
        double *__restrict__ amp, double *__restrict__ logp, unsigned long long *nterm,
        const uint32_t *__restrict__ only) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok;
    double2 *out = (double2 *)smem;
    double2 *piv = out + kExactChunk;
    double2 *red = piv + kThreads;
    uint8_t *Rb = (uint8_t *)(red + kThreads);
    const int tid = threadIdx.x;
    const int lane = tid % G, grp = tid / G;
    constexpr int NG = kThreads / G;
    Work wk;
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        // with `only`, just the bitstrings the lemma evaluation deferred
        if (only && only[b] != kEntryDeferred) continue;
        if (!load_bitstring(p, bits, b, Rb, &s_ok)) {
            if (tid == 0) {
                prob[b] = 0.0;
                if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
                if (logp) logp[b] = -INFINITY;
            }
            __syncthreads();
            continue;
        }
        double2 total = make_double2(0.0, 0.0);
        for (int64_t c0 = 0; c0 < nkeys; c0 += kExactChunk) {
            const int ncur = (int)min((int64_t)kExactChunk, nkeys - c0);
            for (int e = grp; e < ncur; e += NG) {
                int rank;
                const double2 d = term_det<G, MIXED>(p, keys[c0 + e], Rb, lane, piv + grp * G, &rank);
                if (lane == 0) {
                    out[e] = c_mul(w[c0 + e], d);
                    wk.rank += (unsigned)rank;
                    wk.flops += lu_flops(p.m) + 8ull * p.m * p.m * rank;
                }
            }
            __syncthreads();
            const double2 part = ordered_sum(out, ncur, red);
            total.x += part.x;
            total.y += part.y;
        }
        if (tid == 0) {
            const double pb = total.x * total.x + total.y * total.y;
            prob[b] = pb;
            if (amp) { amp[2 * b] = total.x; amp[2 * b + 1] = total.y; }
            if (logp) logp[b] = log(pb);
            wk.terms += (unsigned long long)nkeys;
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

// Bitstrings [b0, b0 + nb) (only: those with only[i] == kEntryDeferred) on a
// grid of `grid` workgroups.
template <int G, bool MIXED>
hipError_t launch_raw_t(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t, uint64_t seed,
                        double *prob, double *amp, double *logp, unsigned long long *nterm, const uint32_t *only,
                        int grid, hipStream_t s) {
    if constexpr (G <= 16) {
        if (use_stage(p, MIXED)) {
            const size_t lds = raw_lds_bytes(p.k, p.n, G, MIXED, true);
            hipLaunchKernelGGL((k_raw_estimate<G, MIXED, 1>), dim3(grid), dim3(kThreads), lds, s, p, bits, b0, nb,
                               (uint32_t)t, seed, prob, amp, logp, nterm, only);
            return hipGetLastError();
        }
    }
    const size_t lds = raw_lds_bytes(p.k, p.n, G, MIXED, false);
    hipLaunchKernelGGL((k_raw_estimate<G, MIXED, 0>), dim3(grid), dim3(kThreads), lds, s, p, bits, b0, nb,
                       (uint32_t)t, seed, prob, amp, logp, nterm, only);
    return hipGetLastError();
}

template <int G, bool MIXED>
hipError_t launch_exact_t(const DevPlan &p, const uint64_t *keys, const double2 *w, int64_t nkeys,
                          const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                          unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s) {
    const size_t lds = exact_lds_bytes(p);
    hipLaunchKernelGGL((k_exact<G, MIXED>), dim3(grid), dim3(kThreads), lds, s, p, keys, w, nkeys,
                       bits, B, prob, amp, logp, nterm, only);
    return hipGetLastError();
}

template <int G>
hipError_t set_lds_limits_raw() {
    const int big = (int)kMaxLds;
    hipError_t e;
    for (const void *f : {(const void *)k_raw_estimate<G, false, 0>, (const void *)k_raw_estimate<G, true, 0>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess) return e;
    if constexpr (G <= 16) {
        for (const void *f : {(const void *)k_raw_estimate<G, false, 1>, (const void *)k_raw_estimate<G, true, 1>})
            if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
                return e;
    }
    return hipSuccess;
}

template <int G>
hipError_t set_lds_limits_exact() {
    const int big = (int)kMaxLds;
    hipError_t e;
    for (const void *f : {(const void *)k_exact<G, false>, (const void *)k_exact<G, true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace
}  // namespace xf
