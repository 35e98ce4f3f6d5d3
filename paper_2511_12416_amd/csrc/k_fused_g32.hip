// Instantiations of the fused LU kernels for lane groups of 32 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_g32(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                         uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                         const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 32: return mixed ? launch_raw_t<32, true>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s)
                         : launch_raw_t<32, false>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t fused_exact_g32(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 32: return mixed ? launch_exact_t<32, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s)
                         : launch_exact_t<32, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_fused_g32(int G) {
    switch (G) {
        case 32: {
            const hipError_t e = set_lds_limits_raw<32>();
            return e != hipSuccess ? e : set_lds_limits_exact<32>();
        }
    }
    return hipSuccess;
}

}  // namespace xf
