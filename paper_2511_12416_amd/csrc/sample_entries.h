// The sampling kernel of the determinant-lemma paths: draws the t
// trajectories of each bitstring (Sec. III-B Eq. 10-12, the sampler defined in
// the public header), reduces them to distinct flip patterns with
// Gaussian-integer phase counts in an LDS hash (the determinant table of
// Sec. IV-B), and writes each table's entries to the bitstring's region of a
// workspace, one flush after another.
#pragma once
#include "xf_device.h"

namespace xf {
namespace {

template <int NT>
__global__ void __launch_bounds__(NT)
k_sample_entries(DevPlan p, const uint64_t *__restrict__ bits, int64_t b0, int64_t nb, uint32_t t, uint64_t seed,
                 uint64_t *__restrict__ ekey, int2 *__restrict__ ecnt, uint32_t *__restrict__ ecount,
                 uint64_t cap, unsigned long long *nblocks) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_ok, s_n;
    __shared__ int s_cnt[6];
    const RawSmem s = carve_sampler(smem, p.k);
    const int tid = threadIdx.x;
    load_tables<NT>(p, s);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t slot0 = hash_slot(0);
    unsigned long long blocks = 0;   // Philox blocks the sampling definition draws
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t b = b0 + i;
        if (!load_bitstring(p, bits, b, s.Rb, &s_ok)) {
            if (tid == 0) ecount[i] = kEntryInvalid;
            continue;
        }
        uint64_t *kout = ekey + (size_t)i * cap;
        int2 *cout = ecnt + (size_t)i * cap;
        uint64_t cursor = 0;
        bool overflow = false;
        Sampler st;
        clear_table<NT>(s, s_cnt, slot0, st);
        while (true) {
            const bool done = sample_until_flush<NT>(p, s, s_cnt, slot0, b, t, k0, k1, st, blocks);
            const int nl = gather_list<NT>(s, &s_n);
            if (cursor + (uint64_t)nl <= cap) {
                for (int e = tid; e < nl; e += NT) {
                    const uint16_t slot = s.list[e];
                    kout[cursor + e] = s.hkey[slot];
                    cout[cursor + e] = s.hcnt[slot];
                }
            } else {
                overflow = true;
            }
            cursor += (uint64_t)nl;
            if (done) break;
            clear_table<NT>(s, s_cnt, slot0, st);
        }
        // a bitstring whose patterns overflow its region is left to the LU kernels
        if (tid == 0) ecount[i] = overflow ? kEntryDeferred : (uint32_t)cursor;
    }
    if (nblocks) {
        const unsigned long long w = wave_sum(blocks);
        if ((tid & 63) == 0 && w) atomicAdd(nblocks, w);
    }
}

}  // namespace
}  // namespace xf
