// Pattern-evaluation kernels of the general determinant lemma under Raw
// Estimate (lemma_gen.h, k_gen_eval): a pass without lane groups of 32 over
// every bitstring, then, where a block has more than 16 active positions, a
// pass with them over the bitstrings the first left (kEntryWide).
#include "lemma_gen.h"

namespace xf {

hipError_t launch_gen_eval_raw(const DevPlan &p, const GenPlan &g, bool multi, bool wide, int64_t b0, int64_t nb,
                               const uint64_t *ekey, const int2 *ecnt, uint32_t *ecount, uint64_t cap,
                               const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                               unsigned long long *nterm, int grid, hipStream_t s) {
    const size_t lds = gen_lds_bytes(g, true), lds16 = gen_lds_bytes(g, false);
    const int grid2 = grid < 2048 ? grid : 2048;
#define XF_EVAL(MULTI, BIG, WIDE, GRID)                                                                           \
    hipLaunchKernelGGL((k_gen_eval<false, MULTI, BIG, WIDE>), dim3(GRID), dim3(kThreads), BIG ? lds : lds16, s, p, g, \
                       b0, nb, ekey,                                                                            \
                       ecnt, ecount, cap, nullptr, nullptr, (int64_t)0, hbuf, rec, prob, amp, logp, nterm, 1, nullptr)
    if (multi) {
        XF_EVAL(true, false, false, grid);
        if (wide) XF_EVAL(true, true, true, grid2);
    } else {
        XF_EVAL(false, false, false, grid);
        if (wide) XF_EVAL(false, true, true, grid2);
    }
#undef XF_EVAL
    return hipGetLastError();
}

hipError_t prepare_gen_eval_raw() {
    hipError_t e;
    for (const void *f : {(const void *)k_gen_eval<false, false, false, false>, (const void *)k_gen_eval<false, false, true, true>,
                          (const void *)k_gen_eval<false, true, false, false>, (const void *)k_gen_eval<false, true, true, true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGenMaxLds)) != hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace xf
