// Instantiations and launchers of the general determinant-lemma evaluation
// (lemma_gen.h): exact mode and Raw Estimate, FP64 and mixed precision.
#include "lemma_gen.h"
#include "sample_entries.h"

namespace xf {
namespace {

size_t gen_lds_bytes(const GenPlan &g) { return kGenBaseBytes + gen_tables_bytes(g); }

// Dynamic LDS limit of k_gen_eval: the static per-bitstring state takes the
// rest of the 160 KiB.
constexpr size_t kGenMaxLds = 150 * 1024;

template <bool EXACT, bool MIXED>
void launch_gen_t(const DevPlan &p, const GenPlan &g, const uint64_t *bits, int64_t b0, int64_t nb,
                  const uint64_t *ekey, const int2 *ecnt, uint32_t *ecount, uint64_t cap, const uint64_t *xkeys,
                  const double2 *xw, int64_t nkeys, double *prob, double *amp, double *logp,
                  unsigned long long *nterm, hipStream_t s) {
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    hipLaunchKernelGGL((k_gen_eval<EXACT, MIXED>), dim3(grid), dim3(kThreads), gen_lds_bytes(g), s, p, g, bits, b0,
                       nb, ekey, ecnt, ecount, cap, xkeys, xw, nkeys, prob, amp, logp, nterm);
}

}  // namespace

bool gen_applies(const DevPlan &p, const GenPlan &g) {
    if (p.L < 1 || p.L > 2 || p.keykind < 0 || g.nblk < 1 || g.nblk > 2) return false;
    for (int b = 0; b < g.nblk; ++b) {
        const int m = g.mb[b], kb = g.kb[b];
        if (m > kGenMaxM || kb > kGenMaxKb) return false;
        if (align16((size_t)m * 2 * m * 16) + (size_t)m * kb * 16 > kGenSetupBytes) return false;
    }
    return gen_lds_bytes(g) <= kGenMaxLds && sampler_lds_bytes(p.k) <= kMaxLds;
}

hipError_t launch_gen_chunk(const DevPlan &p, const GenPlan &g, bool mixed, const uint64_t *bits, int64_t b0,
                            int64_t nb, int64_t t, uint64_t seed, uint64_t *ekey, int2 *ecnt, uint32_t *ecount,
                            uint64_t cap, double *prob, double *amp, double *logp, unsigned long long *nterm,
                            hipEvent_t ev_mid, hipStream_t s) {
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    hipLaunchKernelGGL((k_sample_entries<kSamplerThreads>), dim3(grid), dim3(kSamplerThreads),
                       sampler_lds_bytes(p.k), s, p, bits, b0, nb, (uint32_t)t, seed, ekey, ecnt, ecount, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
    if (mixed)
        launch_gen_t<false, true>(p, g, bits, b0, nb, ekey, ecnt, ecount, cap, nullptr, nullptr, 0, prob, amp, logp,
                                  nterm, s);
    else
        launch_gen_t<false, false>(p, g, bits, b0, nb, ekey, ecnt, ecount, cap, nullptr, nullptr, 0, prob, amp, logp,
                                   nterm, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // then the bitstrings the evaluation deferred, on a smaller grid (its
    // workgroups skip the other bitstrings at once)
    hipLaunchKernelGGL((k_gen_lu<false>), dim3(grid < 2048 ? grid : 2048), dim3(kThreads),
                       raw_lds_bytes(p.k, p.n, 4, false, false), s, p, g, bits, b0, nb, (uint32_t)t, seed, ecount,
                       nullptr, nullptr, (int64_t)0, prob, amp, logp, nterm);
    return hipGetLastError();
}

hipError_t launch_gen_exact(const DevPlan &p, const GenPlan &g, bool mixed, const uint64_t *keys, const double2 *w,
                            int64_t nkeys, const uint64_t *bits, int64_t B, uint32_t *flags, double *prob,
                            double *amp, double *logp, unsigned long long *nterm, hipEvent_t ev_mid,
                            hipStream_t s) {
    if (mixed)
        launch_gen_t<true, true>(p, g, bits, 0, B, nullptr, nullptr, flags, 0, keys, w, nkeys, prob, amp, logp,
                                 nterm, s);
    else
        launch_gen_t<true, false>(p, g, bits, 0, B, nullptr, nullptr, flags, 0, keys, w, nkeys, prob, amp, logp,
                                  nterm, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
    const int grid = (int)(B < 2048 ? B : 2048);
    hipLaunchKernelGGL((k_gen_lu<true>), dim3(grid), dim3(kThreads), raw_lds_bytes(0, p.n, 4, false, false), s, p, g,
                       bits, (int64_t)0, B, 0u, (uint64_t)0, flags, keys, w, nkeys, prob, amp, logp, nterm);
    return hipGetLastError();
}

hipError_t prepare_gen() {
    hipError_t e;
    for (const void *f : {(const void *)k_gen_eval<false, false>, (const void *)k_gen_eval<false, true>,
                          (const void *)k_gen_eval<true, false>, (const void *)k_gen_eval<true, true>,
                          (const void *)k_gen_lu<false>, (const void *)k_gen_lu<true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGenMaxLds)) != hipSuccess)
            return e;
    return hipFuncSetAttribute((const void *)k_sample_entries<kSamplerThreads>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

}  // namespace xf
