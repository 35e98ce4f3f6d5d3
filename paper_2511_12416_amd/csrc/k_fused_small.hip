// Instantiations of the fused LU kernels for lane groups of 4, 8, 16 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_small(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t B, int64_t t, uint64_t seed,
                         double *prob, double *amp, double *logp, unsigned long long *nterm, hipStream_t s) {
    switch (p.G) {
        case 4: return mixed ? launch_raw_t<4, true>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s)
                         : launch_raw_t<4, false>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s);
        case 8: return mixed ? launch_raw_t<8, true>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s)
                         : launch_raw_t<8, false>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s);
        case 16: return mixed ? launch_raw_t<16, true>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s)
                         : launch_raw_t<16, false>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s);
    }
    return hipErrorInvalidValue;
}

hipError_t fused_exact_small(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, hipStream_t s) {
    switch (p.G) {
        case 4: return mixed ? launch_exact_t<4, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s)
                         : launch_exact_t<4, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s);
        case 8: return mixed ? launch_exact_t<8, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s)
                         : launch_exact_t<8, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s);
        case 16: return mixed ? launch_exact_t<16, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s)
                         : launch_exact_t<16, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_fused_small(int G) {
    switch (G) {
        case 4: {
            const hipError_t e = set_lds_limits_raw<4>();
            return e != hipSuccess ? e : set_lds_limits_exact<4>();
        }
        case 8: {
            const hipError_t e = set_lds_limits_raw<8>();
            return e != hipSuccess ? e : set_lds_limits_exact<8>();
        }
        case 16: {
            const hipError_t e = set_lds_limits_raw<16>();
            return e != hipSuccess ? e : set_lds_limits_exact<16>();
        }
    }
    return hipSuccess;
}

size_t raw_estimate_lds_bytes(const DevPlan &p, bool mixed) {
    return raw_lds_bytes(p.k, p.n, p.G, mixed, p.G <= 16 && use_stage(p, mixed));
}

size_t exact_lds_bytes(const DevPlan &) { return kExactChunk * 16 + 2 * kThreads * 16 + 64; }

hipError_t launch_raw_deferred(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                               uint64_t seed, double *prob, double *amp, double *logp,
                               unsigned long long *nterm, const uint32_t *ecount, int grid, hipStream_t s) {
#define XF_DEF(GG)                                                                                             \
    do {                                                                                                       \
        if (use_stage(p, false))                                                                               \
            hipLaunchKernelGGL((k_raw_estimate<GG, false, 1>), dim3(grid), dim3(kThreads),                     \
                               raw_lds_bytes(p.k, p.n, GG, false, true), s, p, bits, b0, nb, (uint32_t)t, seed,   \
                               prob, amp, logp, nterm, ecount);                                                \
        else                                                                                                   \
            hipLaunchKernelGGL((k_raw_estimate<GG, false, 0>), dim3(grid), dim3(kThreads),                     \
                               raw_lds_bytes(p.k, p.n, GG, false, false), s, p, bits, b0, nb, (uint32_t)t, seed,  \
                               prob, amp, logp, nterm, ecount);                                                \
    } while (0)
    switch (p.G) {
        case 4: XF_DEF(4); break;
        case 8: XF_DEF(8); break;
        case 16: XF_DEF(16); break;
        default: return hipErrorInvalidValue;
    }
#undef XF_DEF
    return hipGetLastError();
}


}  // namespace xf
