// Instantiations of the fused LU kernels (Raw Estimate) for lane groups of 64 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_g64(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t B, int64_t t, uint64_t seed,
                         double *prob, double *amp, double *logp, unsigned long long *nterm, hipStream_t s) {
    switch (p.G) {
        case 64: return mixed ? launch_raw_t<64, true>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s)
                         : launch_raw_t<64, false>(p, 0, bits, B, t, seed, prob, amp, logp, nterm, s);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_fused_g64(int G) {
    switch (G) {
        case 64: return set_lds_limits_raw<64>();
    }
    return hipSuccess;
}

}  // namespace xf
