// Small support kernels: a fill (used instead of hipMemsetAsync so the whole
// path stays capturable into a HIP graph) and a one-workgroup exclusive scan.
#include "hough_internal.h"

namespace hough {

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, size_t n)
{
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += size_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Exclusive prefix of n counts -> offsets[0..n] (offsets[n] = total).  When
// out_strided is set, out_strided[i / stride] = offsets[i] for every i that
// is a multiple of stride (i = n included), e.g. per-event offsets.
__global__ void __launch_bounds__(1024)
k_scan_counts(const uint32_t *__restrict__ counts, uint64_t n, uint64_t *__restrict__ offsets,
              uint64_t stride, uint64_t *__restrict__ out_strided)
{
    __shared__ uint64_t part[1024];
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint64_t per = (n + nt - 1) / nt;
    const uint64_t b = min(uint64_t(t) * per, n), e = min(b + per, n);
    uint64_t s = 0;
    for (uint64_t i = b; i < e; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < nt; off <<= 1) {
        const uint64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint64_t run = t ? part[t - 1] : 0;
    for (uint64_t i = b; i < e; ++i) {
        offsets[i] = run;
        if (out_strided && i % stride == 0) out_strided[i / stride] = run;
        run += counts[i];
    }
    if (t == nt - 1) {
        offsets[n] = part[nt - 1];
        if (out_strided) out_strided[n / stride] = part[nt - 1];
    }
}

// Copies event i's hits from [src_off[i], +len[i]) to [dst_off[i], +len[i]).
// blockIdx.y strides over events, (blockIdx.x, threadIdx.x) over hits.
__global__ void __launch_bounds__(256)
k_gather_events(const uint8_t *__restrict__ sl, const uint32_t *__restrict__ sp, const int32_t *__restrict__ sz,
                const uint64_t *__restrict__ src_off, const uint64_t *__restrict__ len,
                const uint64_t *__restrict__ dst_off, uint32_t n, uint8_t *__restrict__ dl,
                uint32_t *__restrict__ dp, int32_t *__restrict__ dz)
{
    for (uint32_t e = blockIdx.y; e < n; e += gridDim.y) {
        const uint64_t s0 = src_off[e], d0 = dst_off[e], m = len[e];
        for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
             i += uint64_t(gridDim.x) * blockDim.x) {
            dl[d0 + i] = sl[s0 + i];
            dp[d0 + i] = sp[s0 + i];
            if (sz) dz[d0 + i] = sz[s0 + i];
        }
    }
}

hipError_t launch_gather_events(const uint8_t *sl, const uint32_t *sp, const int32_t *sz, const uint64_t *src_off,
                                const uint64_t *len, const uint64_t *dst_off, uint32_t n, uint8_t *dl,
                                uint32_t *dp, int32_t *dz, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_events, dim3(64, std::min(n, 65535u)), dim3(256), 0, s, sl, sp, sz, src_off, len,
                       dst_off, n, dl, dp, dz);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hough_ctx *c, uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    KernelTimer t;
    prof_begin(c, "fill_u32", s, &t);
    const uint32_t blocks = uint32_t(std::min<size_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, v, n);
    prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_scan_counts(hough_ctx *c, const uint32_t *counts, uint64_t n, uint64_t *offsets,
                              uint64_t stride_out, uint64_t *out_strided, hipStream_t s)
{
    KernelTimer t;
    prof_begin(c, "scan_counts", s, &t);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, n, offsets,
                       stride_out ? stride_out : 1, out_strided);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
