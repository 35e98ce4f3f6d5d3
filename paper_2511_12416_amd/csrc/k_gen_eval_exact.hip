// Pattern-evaluation kernels of the general determinant lemma in exact mode
// (lemma_gen.h, k_gen_eval): with lane groups of 32 where a block has more
// than 16 active positions, without otherwise.
#include "lemma_gen.h"

namespace xf {

hipError_t launch_gen_eval_exact(const DevPlan &p, const GenPlan &g, bool multi, bool wide, int64_t nb,
                                 const uint64_t *xkeys, const double2 *xw, int64_t nkeys, uint32_t *flags,
                                 const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                                 unsigned long long *nterm, int nseg, uint64_t *part, int grid_cap, hipStream_t s) {
    const size_t lds = gen_lds_bytes(g, true), lds16 = gen_lds_bytes(g, false);
    const int64_t items = nb * nseg;
    const int64_t cap = grid_cap > 0 ? grid_cap : kMaxGrid;
    const int grid = (int)(items < cap ? items : cap);
#define XF_EVAL(MULTI, BIG)                                                                                     \
    hipLaunchKernelGGL((k_gen_eval<true, MULTI, BIG, false>), dim3(grid), dim3(kThreads), BIG ? lds : lds16, s, p, \
                       g, (int64_t)0, nb, nullptr, nullptr, flags, (uint64_t)0, xkeys, xw, nkeys, hbuf, rec, prob,  \
                       amp, logp, nterm, nseg, part)
    if (multi) {
        if (wide) XF_EVAL(true, true);
        else XF_EVAL(true, false);
    } else {
        if (wide) XF_EVAL(false, true);
        else XF_EVAL(false, false);
    }
#undef XF_EVAL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nseg <= 1) return e;
    hipLaunchKernelGGL(k_gen_reduce_segments, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb, nseg, flags, 0u,
                       (const uint64_t *)part, prob, amp, logp);
    return hipGetLastError();
}

hipError_t prepare_gen_eval_exact() {
    hipError_t e;
    for (const void *f : {(const void *)k_gen_eval<true, false, false, false>, (const void *)k_gen_eval<true, false, true, false>,
                          (const void *)k_gen_eval<true, true, false, false>, (const void *)k_gen_eval<true, true, true, false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGenMaxLds)) != hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace xf
