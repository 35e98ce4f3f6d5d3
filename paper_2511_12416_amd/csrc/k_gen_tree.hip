// Prefix-tree kernel of exact mode (lemma_tree.h): one wave per bitstring.
#include "lemma_tree.h"

namespace xf {

hipError_t launch_gen_tree(const DevPlan &p, const GenPlan &g, const DevTree &tr, int64_t nb, int parts,
                           uint32_t *flags, const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, uint64_t *part, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    const int64_t items = nb * (int64_t)parts;
    const int grid = (int)(items < 65536 ? items : 65536);
    if (g.multi)
        hipLaunchKernelGGL(k_gen_tree<true>, dim3(grid), dim3(64), (size_t)tr.lds, s, p, g, tr, nb, parts, flags, hbuf,
                           rec, prob, amp, logp, nterm, part);
    else
        hipLaunchKernelGGL(k_gen_tree<false>, dim3(grid), dim3(64), (size_t)tr.lds, s, p, g, tr, nb, parts, flags, hbuf,
                           rec, prob, amp, logp, nterm, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || parts <= 1) return e;
    hipLaunchKernelGGL(k_gen_tree_reduce, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb, parts, tr.npat, flags,
                       (const GenRec *)rec, (const uint64_t *)part, prob, amp, logp, nterm);
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
