// Instantiations and launchers of the general determinant-lemma evaluation
// (lemma_gen.h): exact mode and Raw Estimate, FP64 and mixed precision.
#include "lemma_gen.h"
#include "sample_entries.h"

namespace xf {

hipError_t launch_gen_eval_raw(const DevPlan &p, const GenPlan &g, bool multi, bool wide, int64_t b0, int64_t nb,
                               const uint64_t *ekey, const int2 *ecnt, uint32_t *ecount, uint64_t cap,
                               const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                               unsigned long long *nterm, int grid, hipStream_t s);
hipError_t launch_gen_eval_exact(const DevPlan &p, const GenPlan &g, bool multi, bool wide, int64_t nb,
                                 const uint64_t *xkeys, const double2 *xw, int64_t nkeys, uint32_t *flags,
                                 const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                                 unsigned long long *nterm, int nseg, uint64_t *part, int grid_cap, hipStream_t s);
hipError_t launch_gen_tree(const DevPlan &p, const GenPlan &g, const DevTree &tr, int64_t nb, int parts,
                           uint32_t *flags, const double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, uint64_t *part, hipStream_t s);
hipError_t prepare_gen_eval_raw();
hipError_t prepare_gen_eval_exact();
hipError_t prepare_gen_tree();

namespace {

size_t gen_lu_lds_bytes(const DevPlan &p, const GenPlan &g, bool exact) {
    return raw_lds_bytes(exact ? 0 : p.k, p.n, 4, false, false) + (g.multi ? kGenMultiLuBytes : 0);
}

// The setup kernels: one wave per bitstring, then the workgroup setup over
// the bases it left (on a smaller grid: its workgroups pass over the other
// bitstrings at once, or return at once when there are none).
template <bool EXACT, bool MIXED, bool MULTI>
void launch_gen_setup_tm(const DevPlan &p, const GenPlan &g, const uint64_t *bits, int64_t b0, int64_t nb,
                         uint32_t *ecount, double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                         unsigned long long *nterm, hipStream_t s) {
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    hipLaunchKernelGGL((k_gen_setup_wave<EXACT, MIXED, MULTI>), dim3(grid), dim3(64), gen_setup_wave_lds(g), s, p, g,
                       bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm);
    hipLaunchKernelGGL((k_gen_setup<EXACT, MIXED, MULTI>), dim3(grid < 2048 ? grid : 2048), dim3(kThreads),
                       kGenSetupLds, s, p, g, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, 1);
}

template <bool EXACT>
void launch_gen_setup_t(const DevPlan &p, const GenPlan &g, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb,
                        uint32_t *ecount, double2 *hbuf, GenRec *rec, double *prob, double *amp, double *logp,
                        unsigned long long *nterm, hipStream_t s) {
    if (g.multi) {
        if (mixed) launch_gen_setup_tm<EXACT, true, true>(p, g, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, s);
        else launch_gen_setup_tm<EXACT, false, true>(p, g, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, s);
    } else {
        if (mixed) launch_gen_setup_tm<EXACT, true, false>(p, g, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, s);
        else launch_gen_setup_tm<EXACT, false, false>(p, g, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, s);
    }
}

// patterns of more than 16 flipped positions in a block can occur only
// where a block has more than 16 active positions
bool gen_wide(const GenPlan &g) {
    bool wide = false;
    for (int b = 0; b < g.nblk; ++b) wide = wide || g.kb[b] > 16;
    return wide;
}

}  // namespace

bool gen_applies(const DevPlan &p, const GenPlan &g) {
    if (p.L < 1 || p.keykind < 0 || g.nblk < 1 || g.nblk > 2) return false;
    if (p.L > 2 && (!g.multi || p.keykind != 1)) return false;
    if (gen_lu_lds_bytes(p, g, false) > kGenMaxLds) return false;
    for (int b = 0; b < g.nblk; ++b) {
        const int m = g.mb[b], kb = g.kb[b];
        if (m > kGenMaxM || kb > kGenMaxKb) return false;
        if (align16((size_t)m * 2 * m * 16) + (size_t)m * kb * 16 > kGenSetupBytes) return false;
    }
    return gen_lds_bytes(g, true) <= kGenMaxLds && sampler_lds_bytes(p.k) <= kMaxLds;
}

size_t gen_setup_bytes(const GenPlan &g) { return (size_t)g.hsize * 16 + sizeof(GenRec); }

int gen_exact_segments(int64_t B, int64_t nkeys) {
    if (B <= 0 || B >= 1024) return 1;
    const int64_t want = (4096 + B - 1) / B, most = (nkeys + 255) / 256;
    return (int)(want < most ? want : (most > 0 ? most : 1));
}

int gen_tree_left_segments(int64_t nkeys) {
    const int64_t most = (nkeys + 255) / 256;
    return (int)(most < 16 ? (most > 0 ? most : 1) : 16);
}

int gen_tree_parts(int64_t B, int64_t nkeys) {
    const int64_t want = (kTreeWaves + B - 1) / (B > 0 ? B : 1), most = (nkeys + 255) / 256;
    const int64_t p = want < most ? want : most;
    return (int)(p < 1 ? 1 : p);
}

int gen_exact_part_segments(int64_t B, int64_t nkeys, bool tree) {
    const int a = gen_exact_segments(B, nkeys);
    if (!tree) return a;
    const int b = a > 1 ? a : gen_tree_left_segments(nkeys), c = gen_tree_parts(B, nkeys);
    return b > c ? b : c;
}

hipError_t launch_gen_chunk(const DevPlan &p, const GenPlan &g, bool mixed, bool all_lu, const uint64_t *bits,
                            int64_t b0, int64_t nb, int64_t t, uint64_t seed, uint64_t *ekey, int2 *ecnt,
                            uint32_t *ecount, uint64_t cap, void *setup, double *prob, double *amp, double *logp,
                            unsigned long long *nterm, hipEvent_t ev_mid, hipStream_t s) {
    double2 *hbuf = (double2 *)setup;
    GenRec *rec = (GenRec *)(hbuf + (size_t)nb * g.hsize);
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    hipError_t e;
    if (all_lu) {
        // every bitstring to the fallback, which samples it itself
        if ((e = launch_fill_u32(ecount, nb, kEntryDeferred, s)) != hipSuccess) return e;
        if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_gen_lu<false>), dim3(grid < 2048 ? grid : 2048), dim3(kThreads),
                           gen_lu_lds_bytes(p, g, false), s, p, g, bits, b0, nb, (uint32_t)t, seed, ecount, nullptr,
                           nullptr, (int64_t)0, prob, amp, logp, nterm, 1, nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_sample_entries<kSamplerThreads>), dim3(grid), dim3(kSamplerThreads),
                       sampler_lds_bytes(p.k), s, p, bits, b0, nb, (uint32_t)t, seed, ekey, ecnt, ecount, cap,
                       nterm ? nterm + 4 : nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
    launch_gen_setup_t<false>(p, g, mixed, bits, b0, nb, ecount, hbuf, rec, prob, amp, logp, nterm, s);
    launch_gen_eval_raw(p, g, g.multi, gen_wide(g), b0, nb, ekey, ecnt, ecount, cap, hbuf, rec, prob, amp, logp,
                        nterm, grid, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // then the bitstrings the evaluation deferred, on a smaller grid (its
    // workgroups skip the other bitstrings at once)
    hipLaunchKernelGGL((k_gen_lu<false>), dim3(grid < 2048 ? grid : 2048), dim3(kThreads),
                       gen_lu_lds_bytes(p, g, false), s, p, g, bits, b0, nb, (uint32_t)t, seed, ecount, nullptr,
                       nullptr, (int64_t)0, prob, amp, logp, nterm, 1, nullptr);
    return hipGetLastError();
}

hipError_t launch_gen_exact(const DevPlan &p, const GenPlan &g, bool mixed, bool all_lu, const uint64_t *keys,
                            const double2 *w, int64_t nkeys, const uint64_t *bits, int64_t B, uint32_t *flags,
                            void *setup, double *prob, double *amp, double *logp, unsigned long long *nterm,
                            hipEvent_t ev_mid, hipStream_t s, const DevTree *tree) {
    hipError_t e;
    double2 *hbuf = (double2 *)setup;
    GenRec *rec = (GenRec *)(hbuf + (size_t)B * g.hsize);
    // few bitstrings: each term list split over segments so that about 4096
    // workgroups take part; their partial sums follow the records
    // the tree: each bitstring's walk split into parts (at most the plan's)
    // so that about kTreeWaves waves share the call, each with at least
    // about 256 terms' work; their partial sums are added after
    int nseg = gen_exact_segments(B, nkeys);
    const bool use_tree = tree && !all_lu;
    const int tp = gen_tree_parts(B, nkeys);
    const int tparts = !use_tree ? 0 : (tp < tree->nparts ? tp : tree->nparts);
    if (use_tree && nseg <= 1) nseg = gen_tree_left_segments(nkeys);
    uint64_t *part = (uint64_t *)(rec + B);
    if (all_lu) {
        if ((e = launch_fill_u32(flags, B, kEntryDeferred, s)) != hipSuccess) return e;
    } else {
        launch_gen_setup_t<true>(p, g, mixed, bits, 0, B, flags, hbuf, rec, prob, amp, logp, nterm, s);
        if (use_tree) launch_gen_tree(p, g, *tree, B, tparts, flags, hbuf, rec, prob, amp, logp, nterm, part, s);
        launch_gen_eval_exact(p, g, g.multi, gen_wide(g), B, keys, w, nkeys, flags, hbuf, rec, prob, amp, logp, nterm,
                              nseg, part, use_tree ? 2048 : 0, s);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
    const int64_t items = B * (int64_t)nseg;
    const int grid = (int)(items < 2048 ? items : 2048);
    hipLaunchKernelGGL((k_gen_lu<true>), dim3(grid), dim3(kThreads), gen_lu_lds_bytes(p, g, true), s, p, g, bits,
                       (int64_t)0, B, 0u, (uint64_t)0, flags, keys, w, nkeys, prob, amp, logp, nterm, nseg, part);
    if ((e = hipGetLastError()) != hipSuccess || nseg <= 1) return e;
    hipLaunchKernelGGL(k_gen_reduce_segments, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, B, nseg, flags,
                       kEntryDeferred, (const uint64_t *)part, prob, amp, logp);
    return hipGetLastError();
}

hipError_t prepare_gen() {
    hipError_t e;
    if ((e = prepare_gen_eval_raw()) != hipSuccess || (e = prepare_gen_eval_exact()) != hipSuccess ||
        (e = prepare_gen_tree()) != hipSuccess)
        return e;
    for (const void *f : {(const void *)k_gen_setup<false, false, false>, (const void *)k_gen_setup<false, true, false>,
                          (const void *)k_gen_setup<true, false, false>, (const void *)k_gen_setup<true, true, false>,
                          (const void *)k_gen_setup<false, false, true>, (const void *)k_gen_setup<false, true, true>,
                          (const void *)k_gen_setup<true, false, true>, (const void *)k_gen_setup<true, true, true>,
                          (const void *)k_gen_setup_wave<false, false, false>,
                          (const void *)k_gen_setup_wave<false, true, false>,
                          (const void *)k_gen_setup_wave<true, false, false>,
                          (const void *)k_gen_setup_wave<true, true, false>,
                          (const void *)k_gen_setup_wave<false, false, true>,
                          (const void *)k_gen_setup_wave<false, true, true>,
                          (const void *)k_gen_setup_wave<true, false, true>,
                          (const void *)k_gen_setup_wave<true, true, true>,
                          (const void *)k_gen_lu<false>, (const void *)k_gen_lu<true>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGenMaxLds)) != hipSuccess)
            return e;
    return hipFuncSetAttribute((const void *)k_sample_entries<kSamplerThreads>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

}  // namespace xf
