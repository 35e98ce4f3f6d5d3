// Instantiations of the fused LU kernels (exact mode) for lane groups of 64 lanes.
#include "fused_kernels.h"

namespace xf {

hipError_t fused_exact_g64(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s) {
    switch (p.G) {
        case 64: return mixed ? launch_exact_t<64, true>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s)
                         : launch_exact_t<64, false>(p, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_fused_g64x(int G) { return G == 64 ? set_lds_limits_exact<64>() : hipSuccess; }

}  // namespace xf
