// Prefix-tree kernel of exact mode (lemma_tree.h): one wave per bitstring.
#include "lemma_tree.h"

namespace xf {

hipError_t launch_gen_tree(const DevPlan &p, const GenPlan &g, const DevTree &tr, int64_t nb, uint32_t *flags,
                           const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    const int grid = (int)(nb < 65536 ? nb : 65536);
    if (g.multi)
        hipLaunchKernelGGL(k_gen_tree<true>, dim3(grid), dim3(64), (size_t)tr.lds, s, p, g, tr, nb, flags, hbuf, rec,
                           prob, amp, logp, nterm);
    else
        hipLaunchKernelGGL(k_gen_tree<false>, dim3(grid), dim3(64), (size_t)tr.lds, s, p, g, tr, nb, flags, hbuf, rec,
                           prob, amp, logp, nterm);
    return hipGetLastError();
}

hipError_t prepare_gen_tree() {
    hipError_t e;
    for (const void *f : {(const void *)k_gen_tree<false>, (const void *)k_gen_tree<true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024)) != hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace xf
