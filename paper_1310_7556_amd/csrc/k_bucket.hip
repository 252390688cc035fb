// Hit ingest: per-event counting sorts that group hits by layer (so a vote
// wavefront works on one layer at a time and the layer bit and the offset
// of a row are wave-uniform), and, for the rz stage, by (layer, coarse
// azimuth bucket) so the member hits of a candidate cell are found in a few
// buckets.  Order inside a group is unspecified: votes are OR/count updates
// and every result is independent of hit order.
#include "hough_internal.h"

namespace hough {

__device__ __forceinline__ void event_range(const uint64_t *offs, uint32_t e, uint64_t n_hits,
                                            uint64_t &b, uint64_t &end)
{
    b = min(offs[e], n_hits);
    end = min(offs[e + 1], n_hits);
    if (end < b) end = b;
}

// One workgroup per event: layer histogram, prefix, scatter.
template <bool WITH_Z>
__global__ void __launch_bounds__(1024)
k_bucket_layers(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
                const int32_t *__restrict__ z, const uint64_t *__restrict__ offs, uint64_t n_hits,
                uint32_t n_layers, uint32_t *__restrict__ out_phi, int32_t *__restrict__ out_z,
                uint32_t *__restrict__ layer_off)
{
    __shared__ uint32_t cnt[kMaxLayers], cur[kMaxLayers];
    const uint32_t e = blockIdx.x, t = threadIdx.x;
    uint64_t b, end;
    event_range(offs, e, n_hits, b, end);
    if (t < kMaxLayers) cnt[t] = 0;
    __syncthreads();
    for (uint64_t i = b + t; i < end; i += blockDim.x) {
        const uint32_t l = layer[i];
        if (l < n_layers) atomicAdd(&cnt[l], 1u);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        uint32_t *lo = layer_off + size_t(e) * (n_layers + 1);
        for (uint32_t l = 0; l < n_layers; ++l) {
            cur[l] = run;
            lo[l] = run;
            run += cnt[l];
        }
        lo[n_layers] = run;
    }
    __syncthreads();
    for (uint64_t i = b + t; i < end; i += blockDim.x) {
        const uint32_t l = layer[i];
        if (l < n_layers) {
            const uint32_t pos = atomicAdd(&cur[l], 1u);
            out_phi[b + pos] = phi[i];
            if (WITH_Z) out_z[b + pos] = z[i];
        }
    }
}

// Split form of the layer sort for batches of few events: event e is cut
// into K parts of consecutive hits, one 256-thread workgroup each.
// k_layer_count counts a part's hits per layer (one ballot per layer per 64
// hits, no atomics); k_split_plan (one wave per event) turns the parts'
// counts into the event's layer offsets and each part's first position per
// layer; k_layer_scatter places a part's hits in input order.  The result
// is a stable counting sort, so the order inside a layer is the input order.
constexpr uint32_t kSplitThreads = 256;

__device__ __forceinline__ void part_range(const uint64_t *offs, uint32_t e, uint32_t k, uint32_t K, uint64_t n,
                                           uint64_t &pb, uint64_t &pe)
{
    uint64_t b, end;
    event_range(offs, e, n, b, end);
    const uint64_t len = end - b;
    pb = b + len * k / K;
    pe = b + len * (k + 1) / K;
}

__global__ void __launch_bounds__(kSplitThreads)
k_layer_count(const uint8_t *__restrict__ layer, const uint64_t *__restrict__ offs, uint64_t n_hits,
              uint32_t n_layers, uint32_t K, uint32_t *__restrict__ part_cnt)
{
    __shared__ uint32_t wc[kSplitThreads / 64][kMaxLayers];
    const uint32_t t = threadIdx.x, lane = t & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
    uint64_t pb, pe;
    part_range(offs, blockIdx.x / K, blockIdx.x % K, K, n_hits, pb, pe);
    uint32_t cnt[kMaxLayers];
#pragma unroll
    for (uint32_t q = 0; q < kMaxLayers; ++q) cnt[q] = 0;
    for (uint64_t i0 = pb + wave * 64; i0 < pe; i0 += kSplitThreads) {
        const uint64_t i = i0 + lane;
        const uint32_t l = i < pe ? layer[i] : 0xFFu;
#pragma unroll
        for (uint32_t q = 0; q < kMaxLayers; ++q)
            if (q < n_layers) cnt[q] += uint32_t(__popcll(__ballot(l == q)));
    }
    if (lane == 0) {
#pragma unroll
        for (uint32_t q = 0; q < kMaxLayers; ++q) wc[wave][q] = cnt[q];
    }
    __syncthreads();
    if (t < n_layers) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < kSplitThreads / 64; ++w) s += wc[w][t];
        part_cnt[size_t(blockIdx.x) * kSplitBins + t] = s;
    }
}

// One wave per event: for each of the event's bins (layers) in order, the
// bin's start is the sum of all earlier bins, and part k's first position
// in bin v is the start plus the counts of parts 0..k-1 in v.  bin_off
// receives the n_bins + 1 starts (relative to the event) when not null.
__global__ void __launch_bounds__(64)
k_split_plan(const uint32_t *__restrict__ part_cnt, uint32_t n_bins, uint32_t K, uint32_t *__restrict__ part_base,
             uint32_t *__restrict__ bin_off)
{
    const uint32_t e = blockIdx.x, lane = threadIdx.x;
    uint32_t run = 0;
    for (uint32_t v = 0; v < n_bins; ++v) {
        const uint32_t x = lane < K ? part_cnt[(size_t(e) * K + lane) * kSplitBins + v] : 0u;
        uint32_t incl = x;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, 64);
            incl += lane >= d ? y : 0u;
        }
        if (lane < K) part_base[(size_t(e) * K + lane) * kSplitBins + v] = run + incl - x;
        if (bin_off && lane == 0) bin_off[size_t(e) * (n_bins + 1) + v] = run;
        run += __shfl(incl, 63, 64);
    }
    if (bin_off && lane == 0) bin_off[size_t(e) * (n_bins + 1) + n_bins] = run;
}

template <bool WITH_Z>
__global__ void __launch_bounds__(kSplitThreads)
k_layer_scatter(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi, const int32_t *__restrict__ z,
                const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_layers, uint32_t K,
                const uint32_t *__restrict__ part_base, uint32_t *__restrict__ out_phi, int32_t *__restrict__ out_z)
{
    __shared__ uint32_t wc[kSplitThreads / 64][kMaxLayers];
    __shared__ uint32_t base[kMaxLayers];
    const uint32_t t = threadIdx.x, lane = t & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t e = blockIdx.x / K;
    uint64_t b, end, pb, pe;
    event_range(offs, e, n_hits, b, end);
    part_range(offs, e, blockIdx.x % K, K, n_hits, pb, pe);
    if (t < n_layers) base[t] = part_base[size_t(blockIdx.x) * kSplitBins + t];
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    // rounds of 256 consecutive hits, wave w taking the w-th 64
    for (uint64_t r0 = pb; r0 < pe; r0 += kSplitThreads) {
        const uint64_t i = r0 + t;
        const bool ok = i < pe;
        const uint32_t l = ok ? layer[i] : 0xFFu;
        const uint32_t ph = ok ? phi[i] : 0u;
        const int32_t zz = WITH_Z && ok ? z[i] : 0;
        uint32_t rank = 0;
#pragma unroll
        for (uint32_t q = 0; q < kMaxLayers; ++q) {
            if (q < n_layers) {
                const uint64_t m = __ballot(l == q);
                if (lane == 0) wc[wave][q] = uint32_t(__popcll(m));
                if (l == q) rank = uint32_t(__popcll(m & lt));
            }
        }
        __syncthreads();
        if (l < n_layers) {
            uint32_t pos = base[l] + rank;
            for (uint32_t w = 0; w < wave; ++w) pos += wc[w][l];
            out_phi[b + pos] = ph;
            if (WITH_Z) out_z[b + pos] = zz;
        }
        __syncthreads();
        if (t < n_layers) {
            uint32_t s = 0;
            for (uint32_t w = 0; w < kSplitThreads / 64; ++w) s += wc[w][t];
            base[t] += s;
        }
        __syncthreads();
    }
}

// Exclusive scan of n (<= 4 * blockDim) LDS counters in place; returns total.
__device__ uint32_t block_exclusive_scan(uint32_t *v, uint32_t n, uint32_t *tmp)
{
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t per = (n + nt - 1) / nt;
    const uint32_t b = min(t * per, n), e = min(b + per, n);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += v[i];
    tmp[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < nt; off <<= 1) {
        const uint32_t x = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += x;
        __syncthreads();
    }
    uint32_t run = t ? tmp[t - 1] : 0;
    const uint32_t total = tmp[nt - 1];
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    __syncthreads();
    return total;
}

// One workgroup per (event, layer): counting sort of the layer's hits by the
// top `bits` bits of phi (z moved along unless out_z is null).  bucket_off[(e * L + l) * (NB + 1) + i] = start of
// bucket i relative to the event start.
__global__ void __launch_bounds__(1024)
k_bucket_phi(const uint32_t *__restrict__ in_phi, const int32_t *__restrict__ in_z,
             const uint64_t *__restrict__ offs, uint64_t n_hits, const uint32_t *__restrict__ layer_off,
             uint32_t n_layers, uint32_t bits, uint32_t *__restrict__ out_phi,
             int32_t *__restrict__ out_z, uint32_t *__restrict__ bucket_off)
{
    __shared__ uint32_t hist[1u << kMaxBucketBits];
    __shared__ uint32_t tmp[1024];
    const uint32_t e = blockIdx.x / n_layers, l = blockIdx.x % n_layers, t = threadIdx.x;
    const uint32_t nb = 1u << bits, sh = 32 - bits;
    uint64_t b, end;
    event_range(offs, e, n_hits, b, end);
    const uint32_t *lo = layer_off + size_t(e) * (n_layers + 1);
    const uint32_t s0 = lo[l], s1 = lo[l + 1];
    for (uint32_t i = t; i < nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = s0 + t; i < s1; i += blockDim.x) atomicAdd(&hist[in_phi[b + i] >> sh], 1u);
    __syncthreads();
    block_exclusive_scan(hist, nb, tmp);
    uint32_t *bo = bucket_off + (size_t(e) * n_layers + l) * (nb + 1);
    for (uint32_t i = t; i < nb; i += blockDim.x) bo[i] = s0 + hist[i];
    if (t == 0) bo[nb] = s1;
    __syncthreads();
    for (uint32_t i = s0 + t; i < s1; i += blockDim.x) {
        const uint32_t ph = in_phi[b + i];
        const uint32_t pos = s0 + atomicAdd(&hist[ph >> sh], 1u);
        out_phi[b + pos] = ph;
        if (out_z) out_z[b + pos] = in_z[b + i];
    }
}

// Events ordered longest first (coarse: log2 size with 3 mantissa bits) for
// a longest-processing-time-first work queue.  One workgroup.
__global__ void __launch_bounds__(1024)
k_event_order(const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_events,
              uint32_t *__restrict__ order)
{
    __shared__ uint32_t hist[256];
    const uint32_t t = threadIdx.x;
    auto key = [&](uint32_t e) {
        uint64_t b, end;
        event_range(offs, e, n_hits, b, end);
        const uint64_t sz = end - b;
        if (sz == 0) return 255u;
        const uint32_t lg = 63 - __clzll(sz);
        const uint32_t sub = lg >= 3 ? uint32_t(sz >> (lg - 3)) & 7u : uint32_t(sz << (3 - lg)) & 7u;
        return 255u - min(lg * 8 + sub, 255u);        // descending size
    };
    for (uint32_t i = t; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (uint32_t e = t; e < n_events; e += blockDim.x) atomicAdd(&hist[key(e)], 1u);
    __syncthreads();
    // exclusive prefix sum of the 256 bins: four per lane of the first wave,
    // then a wave scan of the lanes' totals
    if (t < 64) {
        const uint32_t h0 = hist[4 * t], h1 = hist[4 * t + 1], h2 = hist[4 * t + 2], h3 = hist[4 * t + 3];
        const uint32_t tot = h0 + h1 + h2 + h3;
        uint32_t inc = tot;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(inc, d, 64);
            if (t >= d) inc += v;
        }
        const uint32_t ex = inc - tot;
        hist[4 * t] = ex;
        hist[4 * t + 1] = ex + h0;
        hist[4 * t + 2] = ex + h0 + h1;
        hist[4 * t + 3] = ex + h0 + h1 + h2;
    }
    __syncthreads();
    for (uint32_t e = t; e < n_events; e += blockDim.x) order[atomicAdd(&hist[key(e)], 1u)] = e;
}

hipError_t launch_bucket_layers(hough_ctx *c, const hough_hits *h, bool with_z, hipStream_t s)
{
    if (h->n_events == 0) return hipSuccess;
    KernelTimer t;
    prof_begin(c, "bucket_layers", s, &t);
    if (const uint32_t K = split_parts(c, h->n_events)) {
        const uint32_t parts = h->n_events * K, L = c->spec.n_layers;
        hipLaunchKernelGGL(k_layer_count, dim3(parts), dim3(kSplitThreads), 0, s, h->layer, h->event_offsets,
                           h->n_hits, L, K, c->d_part_cnt);
        hipError_t err = launch_split_plan(h->n_events, L, K, c->d_part_cnt, c->d_part_base, c->d_layer_off, s);
        if (err != hipSuccess) return err;
        if (with_z)
            hipLaunchKernelGGL(k_layer_scatter<true>, dim3(parts), dim3(kSplitThreads), 0, s, h->layer, h->phi,
                               h->z_um, h->event_offsets, h->n_hits, L, K, c->d_part_base, c->d_phi_a, c->d_z_a);
        else
            hipLaunchKernelGGL(k_layer_scatter<false>, dim3(parts), dim3(kSplitThreads), 0, s, h->layer, h->phi,
                               h->z_um, h->event_offsets, h->n_hits, L, K, c->d_part_base, c->d_phi_a, c->d_z_a);
        prof_end(c, s, &t);
        return hipGetLastError();
    }
    if (with_z)
        hipLaunchKernelGGL(k_bucket_layers<true>, dim3(h->n_events), dim3(1024), 0, s, h->layer,
                           h->phi, h->z_um, h->event_offsets, h->n_hits, c->spec.n_layers,
                           c->d_phi_a, c->d_z_a, c->d_layer_off);
    else
        hipLaunchKernelGGL(k_bucket_layers<false>, dim3(h->n_events), dim3(1024), 0, s, h->layer,
                           h->phi, h->z_um, h->event_offsets, h->n_hits, c->spec.n_layers,
                           c->d_phi_a, c->d_z_a, c->d_layer_off);
    prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_split_plan(uint32_t n_events, uint32_t n_bins, uint32_t K, const uint32_t *part_cnt,
                             uint32_t *part_base, uint32_t *bin_off, hipStream_t s)
{
    if (n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_plan, dim3(n_events), dim3(64), 0, s, part_cnt, n_bins, K, part_base, bin_off);
    return hipGetLastError();
}

hipError_t launch_bucket_phi(hough_ctx *c, const hough_hits *h, hipStream_t s, bool with_z)
{
    if (h->n_events == 0) return hipSuccess;
    KernelTimer t;
    prof_begin(c, "bucket_phi", s, &t);
    hipLaunchKernelGGL(k_bucket_phi, dim3(h->n_events * c->spec.n_layers), dim3(1024), 0, s,
                       c->d_phi_a, c->d_z_a, h->event_offsets, h->n_hits, c->d_layer_off,
                       c->spec.n_layers, c->bucket_bits, c->d_phi_b, with_z ? c->d_z_b : nullptr,
                       c->d_bucket_off);
    prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_event_order(hough_ctx *c, const hough_hits *h, hipStream_t s)
{
    KernelTimer t;
    prof_begin(c, "event_order", s, &t);
    hipLaunchKernelGGL(k_event_order, dim3(1), dim3(1024), 0, s, h->event_offsets, h->n_hits,
                       h->n_events, c->d_order);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
