// Small utility kernels: zero and value fills, fixed-order reduction of per-workgroup
// partial sums (overwrites the partials), counter reset.
#include "xf_device.h"

namespace xf {
namespace {
__global__ void k_fill_zero(double *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Fixed-order sum of the partials part[q][e], q < nparts, in two levels:
// k_reduce_chunks adds each chunk of `len` consecutive partials in order and
// stores the sum in the chunk's first row (blockIdx.y = chunk);
// k_reduce_parts then adds the chunks' sums in chunk order into out[e].
// The association does not depend on the launch, so results repeat bitwise.
__global__ void k_reduce_chunks(double2 *__restrict__ part, int nparts, int stride, int len) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int q0 = blockIdx.y * len;
    if (e >= stride || q0 >= nparts) return;
    const int q1 = min(nparts, q0 + len);
    double2 acc = make_double2(0.0, 0.0);
    for (int q = q0; q < q1; ++q) {
        const double2 v = part[(size_t)q * stride + e];
        acc.x += v.x;
        acc.y += v.y;
    }
    part[(size_t)q0 * stride + e] = acc;
}

__global__ void k_reduce_parts(const double2 *__restrict__ part, int nparts, int stride, int len, double2 *out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= stride) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < nparts; q += len) {
        const double2 v = part[(size_t)q * stride + e];
        acc.x += v.x;
        acc.y += v.y;
    }
    out[e] = acc;
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x < 8) p[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s) {
    const int grid = (int)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, p, (size_t)count, v);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(double2 *part, int nparts, int stride, double2 *out, hipStream_t s) {
    // chunks of 32 partials: enough workgroups to read the partials at the
    // memory's rate, few enough chunk sums for the second level
    const int len = 32, chunks = (nparts + len - 1) / len;
    const unsigned gx = (unsigned)((stride + 255) / 256);
    if (chunks > 1) {
        hipLaunchKernelGGL(k_reduce_chunks, dim3(gx, (unsigned)chunks), dim3(256), 0, s, part, nparts, stride, len);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(gx), dim3(256), 0, s, (const double2 *)part, nparts, stride,
                       chunks > 1 ? len : 1, out);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t prepare_kernels(int G) {
    hipError_t e;
    if ((e = prepare_fused_small(G)) != hipSuccess) return e;
    if ((e = prepare_fused_g32(G)) != hipSuccess) return e;
    if ((e = prepare_fused_g64(G)) != hipSuccess) return e;
    if ((e = prepare_fused_g64x(G)) != hipSuccess) return e;
    if ((e = prepare_lemma(G)) != hipSuccess) return e;
    if ((e = prepare_gen()) != hipSuccess) return e;
    return prepare_bwd(G);
}

size_t raw_estimate_lds_bytes(const DevPlan &p, bool mixed) {
    return raw_lds_bytes(p.k, p.n, p.G, mixed, p.G <= 16 && use_stage(p, mixed));
}

size_t exact_lds_bytes(const DevPlan &) { return kExactChunk * 16 + 2 * kThreads * 16 + 64; }

hipError_t launch_raw_estimate(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                               uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                               const uint32_t *only, int grid, hipStream_t s) {
    if (grid <= 0) grid = (int)(nb < kMaxGrid ? nb : kMaxGrid);
    if (p.G <= 16) return fused_raw_small(p, mixed, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
    if (p.G == 32) return fused_raw_g32(p, mixed, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
    return fused_raw_g64(p, mixed, bits, b0, nb, t, seed, prob, amp, logp, nterm, only, grid, s);
}

hipError_t launch_exact(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                        const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                        unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s) {
    if (grid <= 0) grid = (int)(B < kMaxGrid ? B : kMaxGrid);
    if (p.G <= 16) return fused_exact_small(p, mixed, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
    if (p.G == 32) return fused_exact_g32(p, mixed, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
    return fused_exact_g64(p, mixed, keys, w, nkeys, bits, B, prob, amp, logp, nterm, only, grid, s);
}

}  // namespace xf
