// Instantiations of the fused LU kernels (Raw Estimate) for lane groups of 64 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_raw_g64(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                         uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                         const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 64: return mixed ? launch_raw_t<64, true>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s)
                         : launch_raw_t<64, false>(p, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
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
