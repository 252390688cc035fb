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
    if (t == 0) {
        uint32_t run = 0;
        for (uint32_t i = 0; i < 256; ++i) {
            const uint32_t x = hist[i];
            hist[i] = run;
            run += x;
        }
    }
    __syncthreads();
    for (uint32_t e = t; e < n_events; e += blockDim.x) order[atomicAdd(&hist[key(e)], 1u)] = e;
}

hipError_t launch_bucket_layers(hough_ctx *c, const hough_hits *h, bool with_z, hipStream_t s)
{
    if (h->n_events == 0) return hipSuccess;
    KernelTimer t;
    prof_begin(c, "bucket_layers", s, &t);
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
