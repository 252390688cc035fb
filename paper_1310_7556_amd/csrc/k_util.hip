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
template <class T>
__global__ void __launch_bounds__(1024)
k_scan_counts(const T *__restrict__ counts, uint64_t n, uint64_t *__restrict__ offsets,
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

// Large scans in three launches: per-block sums of kScanBlock counts, the
// one-workgroup scan of those sums, then a block-wide scan of each block's
// counts offset by its sum's prefix.
constexpr uint32_t kScanThreads = 1024, kScanPer = 4, kScanBlock = kScanThreads * kScanPer;

__device__ __forceinline__ uint64_t thread_counts(const uint32_t *__restrict__ counts, uint64_t n, uint64_t i0,
                                                  uint32_t v[kScanPer])
{
    uint64_t s = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) {
        v[j] = i0 + j < n ? counts[i0 + j] : 0u;
        s += v[j];
    }
    return s;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_partials(const uint32_t *__restrict__ counts, uint64_t n, uint64_t *__restrict__ partials)
{
    __shared__ uint64_t ws[kScanThreads / 64];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t v[kScanPer];
    uint64_t s = thread_counts(counts, n, uint64_t(blockIdx.x) * kScanBlock + uint64_t(t) * kScanPer, v);
    for (uint32_t off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) ws[wave] = s;
    __syncthreads();
    if (t == 0) {
        uint64_t total = 0;
        for (uint32_t w = 0; w < kScanThreads / 64; ++w) total += ws[w];
        partials[blockIdx.x] = total;
    }
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const uint32_t *__restrict__ counts, uint64_t n, const uint64_t *__restrict__ block_off,
             uint64_t *__restrict__ offsets, uint64_t stride, uint64_t *__restrict__ out_strided)
{
    __shared__ uint64_t ws[kScanThreads / 64];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint64_t i0 = uint64_t(blockIdx.x) * kScanBlock + uint64_t(t) * kScanPer;
    uint32_t v[kScanPer];
    const uint64_t s = thread_counts(counts, n, i0, v);
    // inclusive wave scan of the thread sums, then the waves' totals
    uint64_t inc = s;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    uint64_t wbase = 0;
    for (uint32_t w = 0; w < wave; ++w) wbase += ws[w];
    uint64_t run = block_off[blockIdx.x] + wbase + inc - s;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) {
        const uint64_t i = i0 + j;
        if (i < n) {
            offsets[i] = run;
            if (out_strided && i % stride == 0) out_strided[i / stride] = run;
            run += v[j];
            if (i == n - 1) {
                offsets[n] = run;
                if (out_strided) out_strided[n / stride] = run;
            }
        }
    }
}

// Copies event i's hits from [src_off[i], +len[i]) to [dst_off[i], +len[i]).
// blockIdx.y strides over events, (blockIdx.x, threadIdx.x) over hits.
__global__ void __launch_bounds__(256)
k_gather_events(const uint8_t *__restrict__ sl, const uint32_t *__restrict__ sp, const int32_t *__restrict__ sz,
                const uint64_t *__restrict__ src_off, const uint64_t *__restrict__ len,
                const uint64_t *__restrict__ dst_off, uint32_t n, uint8_t *__restrict__ dl,
                uint32_t *__restrict__ dp, int32_t *__restrict__ dz, uint64_t cap)
{
    for (uint32_t e = blockIdx.y; e < n; e += gridDim.y) {
        const uint64_t s0 = src_off[e], d0 = min(dst_off[e], cap);
        const uint64_t m = min(len[e], cap - d0);   // nothing lands at or past cap
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
                                uint32_t *dp, int32_t *dz, uint64_t cap, hipStream_t s)
{
    if (n == 0 || cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_events, dim3(64, std::min(n, 65535u)), dim3(256), 0, s, sl, sp, sz, src_off, len,
                       dst_off, n, dl, dp, dz, cap);
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

uint64_t scan_blocks(uint64_t n)
{
    return (n + kScanBlock - 1) / kScanBlock;
}

hipError_t launch_scan_counts(hough_ctx *c, const uint32_t *counts, uint64_t n, uint64_t *offsets,
                              uint64_t stride_out, uint64_t *out_strided, hipStream_t s, uint64_t *scan_part,
                              uint64_t *scan_off, uint64_t blocks_max, bool timed)
{
    KernelTimer t;
    t.name = nullptr;
    const uint64_t stride = stride_out ? stride_out : 1;
    const uint64_t nb = scan_blocks(n);
    if (timed) prof_begin(c, "scan_counts", s, &t);
    if (nb <= 2 || nb > blocks_max) {
        hipLaunchKernelGGL(k_scan_counts<uint32_t>, dim3(1), dim3(1024), 0, s, counts, n, offsets, stride,
                           out_strided);
    } else {
        hipLaunchKernelGGL(k_scan_partials, dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, counts, n, scan_part);
        hipLaunchKernelGGL(k_scan_counts<uint64_t>, dim3(1), dim3(1024), 0, s, scan_part, nb, scan_off,
                           uint64_t(1), static_cast<uint64_t *>(nullptr));
        hipLaunchKernelGGL(k_scan_apply, dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, counts, n, scan_off,
                           offsets, stride, out_strided);
    }
    if (timed) prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_scan_counts(hough_ctx *c, const uint32_t *counts, uint64_t n, uint64_t *offsets,
                              uint64_t stride_out, uint64_t *out_strided, hipStream_t s)
{
    return launch_scan_counts(c, counts, n, offsets, stride_out, out_strided, s, c->d_scan_part, c->d_scan_off,
                              c->scan_blocks_max, true);
}

}  // namespace hough
