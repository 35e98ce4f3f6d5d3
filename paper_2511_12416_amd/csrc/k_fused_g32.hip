// Instantiations of the fused LU kernels for lane groups of 32 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_g32(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t B, int64_t t, uint64_t seed,
                         double *prob, double *amp, double *logp, unsigned long long *nterm, hipStream_t s) {
    switch (p.G) {
        case 32: return mixed ? launch_raw_t<32, true>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s)
                         : launch_raw_t<32, false>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s);
    }
    return hipErrorInvalidValue;
}

hipError_t fused_exact_g32(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, hipStream_t s) {
    switch (p.G) {
        case 32: return mixed ? launch_exact_t<32, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s)
                         : launch_exact_t<32, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, s);
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
