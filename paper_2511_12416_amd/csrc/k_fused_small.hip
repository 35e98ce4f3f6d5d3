// Instantiations of the fused LU kernels for lane groups of 4, 8, 16 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_small(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                         uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                         const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 4: return mixed ? launch_raw_t<4, true>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s)
                         : launch_raw_t<4, false>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
        case 8: return mixed ? launch_raw_t<8, true>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s)
                         : launch_raw_t<8, false>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
        case 16: return mixed ? launch_raw_t<16, true>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s)
                         : launch_raw_t<16, false>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t fused_exact_small(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 4: return mixed ? launch_exact_t<4, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s)
                         : launch_exact_t<4, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
        case 8: return mixed ? launch_exact_t<8, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s)
                         : launch_exact_t<8, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
        case 16: return mixed ? launch_exact_t<16, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s)
                         : launch_exact_t<16, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
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



}  // namespace xf
