// Raw Estimate under the determinant lemma for one CPhase layer and
// eta <= 16: a sampling kernel that writes each bitstring's distinct flip
// patterns with their Gaussian-integer counts to a workspace, and an
// evaluation kernel that forms the bitstring's H once and takes an r x r
// determinant per pattern; and the adjoint of the same evaluation
// (k_bwd_entries, lemma_bwd.h).
#include "lemma_bwd.h"
#include "sample_entries.h"
#include "xf_device.h"

namespace xf {
namespace {
// ---------------------------------------------------------------------------
// Raw Estimate under the determinant lemma, in two kernels per chunk of
// bitstrings, so that each runs at its own occupancy: the sampler needs few
// registers and no evaluation scratch (three workgroups per CU), the
// evaluation needs the registers of the per-lane determinants.
//   k_sample_entries: draws the t trajectories of each bitstring and writes
//     its distinct (flip pattern, Gaussian-integer count) entries, one table
//     flush after another, to the bitstring's region of the workspace.
//   k_eval_entries: forms H for the bitstring and evaluates the entries in
//     chunks of kHashSlots, summing count * det exactly.
// ---------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kThreads, 2)
k_eval_entries(DevPlan p, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb,
               const uint64_t *__restrict__ ekey, const int2 *__restrict__ ecnt,
               uint32_t *__restrict__ ecount, uint64_t cap, double *__restrict__ prob,
               double *__restrict__ amp, double *__restrict__ logp, unsigned long long *nterm) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_flag[2];
    __shared__ double2 s_det;
    __shared__ uint64_t s_acc[kAccWords];
    const RawSmem s = carve_raw(smem, 0, p.n, G, false);
    double2 *sH = (double2 *)((unsigned char *)s.sP + (size_t)G * G * 16);
    const int tid = threadIdx.x;
    Work wk;
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = b0 + i;
        const uint32_t ne = ecount[i];
        if (ne == kEntryInvalid) {
            if (tid == 0) {
                prob[b] = 0.0;
                if (amp) { amp[2 * b] = 0.0; amp[2 * b + 1] = 0.0; }
                if (logp) logp[b] = -INFINITY;
            }
            continue;
        }
        // patterns that overflowed the workspace region: the LU kernel takes it
        if (ne == kEntryDeferred) continue;
        load_bitstring(p, bits, b, s.Rb, &s_ok);
        double2 total;
        {
            const LemmaBits lb = lemma_setup<G>(p, s, sH, s_flag, &s_det, wk);
            bool ok = lb.ok;
            acc_clear(s_acc);
            const uint64_t *kin = ekey + (size_t)i * cap;
            const int2 *cin = ecnt + (size_t)i * cap;
            for (uint32_t c0 = 0; ok && c0 < ne; c0 += kHashSlots) {
                const int nc = (int)min((uint32_t)kHashSlots, ne - c0);
                for (int e = tid; e < nc; e += kThreads) {
                    s.hkey[e] = kin[c0 + e];
                    s.hcnt[e] = cin[c0 + e];
                    s.list[e] = (uint16_t)e;
                }
                __syncthreads();
                ok = sum_entries_lemma<G>(p, s, nc, sH, lb, wk, s_acc);
            }
            if (!ok) {
                // ill-conditioned base or a pattern with r > G: the LU kernel
                // that follows recomputes this bitstring
                if (tid == 0) ecount[i] = kEntryDeferred;
                __syncthreads();
                continue;
            }
            total = acc_value(s_acc);
        }
        if (tid == 0) {
            const double ax = total.x * p.scale, ay = total.y * p.scale;
            const double pb = ax * ax + ay * ay;
            prob[b] = pb;
            if (amp) { amp[2 * b] = ax; amp[2 * b + 1] = ay; }
            if (logp) logp[b] = log(pb);
        }
        __syncthreads();
    }
    flush_work(wk, nterm);
}

template <int G>
hipError_t set_lds_limits_lemma() {
    const int big = (int)kMaxLds;
    hipError_t e;
    for (const void *f : {(const void *)k_eval_entries<G>, (const void *)k_sample_entries<kSamplerThreads>,
                          (const void *)k_bwd_entries<G>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

bool raw_estimate_uses_lemma(const DevPlan &p, int algorithm) {
    return algorithm != 1 && lemma_applies(p);
}

// Entries of a bitstring's workspace region: enough for every pattern of t
// samples (with the tables' reserved empty-pattern slots), at most
// kEntryCapMax; a bitstring with more distinct patterns is left to the LU
// kernels.
uint64_t lemma_entry_cap(int64_t t) {
    const uint64_t full = (uint64_t)t + (uint64_t)t / 511 + 2;
    return full < kEntryCapMax ? full : kEntryCapMax;
}

hipError_t launch_lemma_chunk(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                              uint64_t seed, uint64_t *ekey, int2 *ecnt, uint32_t *ecount, uint64_t cap,
                              double *prob, double *amp, double *logp, unsigned long long *nterm,
                              hipEvent_t ev_mid, hipStream_t s) {
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    hipLaunchKernelGGL((k_sample_entries<kSamplerThreads>), dim3(grid), dim3(kSamplerThreads),
                       sampler_lds_bytes(p.k), s, p, bits, b0, nb, (uint32_t)t, seed, ekey, ecnt, ecount, cap,
                       nterm ? nterm + 4 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid && (e = hipEventRecord(ev_mid, s)) != hipSuccess) return e;
    switch (p.G) {
        case 4:
            hipLaunchKernelGGL((k_eval_entries<4>), dim3(grid), dim3(kThreads), lemma_lds(p), s, p, bits, b0, nb,
                               ekey, ecnt, ecount, cap, prob, amp, logp, nterm);
            break;
        case 8:
            hipLaunchKernelGGL((k_eval_entries<8>), dim3(grid), dim3(kThreads), lemma_lds(p), s, p, bits, b0, nb,
                               ekey, ecnt, ecount, cap, prob, amp, logp, nterm);
            break;
        case 16:
            hipLaunchKernelGGL((k_eval_entries<16>), dim3(grid), dim3(kThreads), lemma_lds(p), s, p, bits, b0, nb,
                               ekey, ecnt, ecount, cap, prob, amp, logp, nterm);
            break;
        default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // then the LU kernel for the bitstrings the evaluation deferred, on a
    // smaller grid (its workgroups skip the other bitstrings at once; the
    // deferred ones are rare)
    return launch_raw_estimate(p, false, bits, b0, nb, t, seed, prob, amp, logp, nterm, ecount,
                               grid < 2048 ? grid : 2048, s);
}

size_t bwd_lemma_lds(const DevPlan &p) { return lemma_lds(p) + bwd_lemma_extra(p.G, p.keybits); }

bool backward_uses_lemma(const DevPlan &p, int algorithm) {
    return algorithm != 1 && lemma_applies(p) && bwd_lemma_lds(p) <= kMaxLds;
}

hipError_t launch_lemma_bwd_chunk(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                                  uint64_t seed, uint64_t *ekey, int2 *ecnt, uint32_t *ecount, uint64_t cap,
                                  const double *g, double2 *part, int nparts, const GradLayout &lay,
                                  bool resample, hipStream_t s) {
    const int grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    if (resample) {
        hipLaunchKernelGGL((k_sample_entries<kSamplerThreads>), dim3(grid), dim3(kSamplerThreads),
                           sampler_lds_bytes(p.k), s, p, bits, b0, nb, (uint32_t)t, seed, ekey, ecnt, ecount, cap,
                           nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int bg = nparts < nb ? nparts : (int)nb;
    const size_t lds = bwd_lemma_lds(p);
    switch (p.G) {
        case 4:
            hipLaunchKernelGGL((k_bwd_entries<4>), dim3(bg), dim3(kThreads), lds, s, p, bits, b0, nb, ekey, ecnt,
                               ecount, cap, g, part, lay);
            break;
        case 8:
            hipLaunchKernelGGL((k_bwd_entries<8>), dim3(bg), dim3(kThreads), lds, s, p, bits, b0, nb, ekey, ecnt,
                               ecount, cap, g, part, lay);
            break;
        case 16:
            hipLaunchKernelGGL((k_bwd_entries<16>), dim3(bg), dim3(kThreads), lds, s, p, bits, b0, nb, ekey, ecnt,
                               ecount, cap, g, part, lay);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t prepare_lemma(int G) {
    switch (G) {
        case 4: return set_lds_limits_lemma<4>();
        case 8: return set_lds_limits_lemma<8>();
        case 16: return set_lds_limits_lemma<16>();
    }
    return hipSuccess;
}

}  // namespace xf
