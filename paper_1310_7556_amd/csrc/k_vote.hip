// Step 1 of the transform: every hit votes into every reachable row of the
// accumulator (Section 4, first step; the Discussion's indirect update
// A[B[i]] += 1, here in its layer-bitmask OR form).
//
// Work item = (event, tile of R consecutive rows).  A persistent grid pulls
// items from a global counter (events ordered longest first).  The tile of
// R x n_phi cells lives in LDS as one uint32 per cell; hits arrive grouped by
// layer so the layer bit and the R row offsets of a layer are wave-uniform
// scalars, and each vote is: subtract, shift, LDS atomic OR.  The finished
// tile is packed to uint16 and written to HBM once, with coalesced stores.
// This is the paper's GPU recipe (global atomics replaced by shared-memory
// atomics, Section 6.1) re-tiled for 64-wide wavefronts and 160 KB LDS.
#include "hough_internal.h"

namespace hough {

// COUNT: the paper's counting form A[B[i]] += 1 (Section 8) -- an atomic
// add of 1 per vote into the uint32 tile, written out as uint32 counts --
// instead of the OR of the layer bit packed to uint16 masks.
template <int R, bool COUNT>
__global__ void __launch_bounds__(1024)
k_vote_lds(const uint32_t *__restrict__ sphi, const uint64_t *__restrict__ offs, uint64_t n_hits,
           const uint32_t *__restrict__ layer_off, const uint32_t *__restrict__ O,
           const uint8_t *__restrict__ V, uint32_t n_layers, uint32_t rows, uint32_t nphi,
           uint32_t shift, int all_valid, uint32_t n_tiles, uint32_t n_items,
           const uint32_t *__restrict__ order, uint32_t *__restrict__ counter,
           void *__restrict__ out)
{
    HOUGH_DYNAMIC_LDS(uint32_t, tile);
    __shared__ uint32_t item_s[2];
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint64_t cells = uint64_t(rows) * nphi;
    for (;;) {
        // Work fetch without divergent control flow: all threads execute the
        // atomic, only thread 0 adds 1 and only its ticket lands in slot 0.
        const uint32_t mine = atomicAdd(counter, t == 0 ? 1u : 0u);
        item_s[t == 0 ? 0 : 1] = mine;
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(item_s[0]);
        if (item >= n_items) break;
        const uint32_t e = __builtin_amdgcn_readfirstlane(order[item / n_tiles]);
        const uint32_t r0 = (item % n_tiles) * R;
        const uint32_t nr = min(uint32_t(R), rows - r0);
        for (uint32_t i = t; i < uint32_t(R) * nphi; i += nt) tile[i] = 0;
        uint64_t b = min(offs[e], n_hits);
        b = __builtin_amdgcn_readfirstlane(uint32_t(b)) | (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(b >> 32))) << 32);
        const uint32_t *lo = layer_off + size_t(e) * (n_layers + 1);
        __syncthreads();
        for (uint32_t l = 0; l < n_layers; ++l) {
            const uint32_t hs = lo[l], he = lo[l + 1];
            const uint32_t bit = 1u << l;
            const uint32_t *Ol = O + size_t(l) * rows + r0;
            const uint8_t *Vl = V + size_t(l) * rows + r0;
            uint32_t o[R];
            bool ok[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool in = uint32_t(r) < nr;
                o[r] = in ? Ol[r] : 0u;
                ok[r] = in && (all_valid || Vl[r]);
            }
            for (uint32_t h = hs + t; h < he; h += nt) {
                const uint32_t ph = sphi[b + h];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (ok[r]) {
                        const uint32_t p = (ph - o[r]) >> shift;
                        if (COUNT)
                            atomicAdd(&tile[uint32_t(r) * nphi + p], 1u);
                        else
                            atomicOr(&tile[uint32_t(r) * nphi + p], bit);
                    }
                }
            }
        }
        __syncthreads();
        if (COUNT) {
            uint32_t *dst = static_cast<uint32_t *>(out) + uint64_t(e) * cells + uint64_t(r0) * nphi;
            for (uint32_t i = t; i < nr * nphi; i += nt) dst[i] = tile[i];
        } else {
            uint32_t *dst = reinterpret_cast<uint32_t *>(static_cast<uint16_t *>(out) + uint64_t(e) * cells +
                                                         uint64_t(r0) * nphi);
            const uint32_t nw = nr * nphi / 2;
            for (uint32_t i = t; i < nw; i += nt) dst[i] = tile[2 * i] | (tile[2 * i + 1] << 16);
        }
        __syncthreads();
    }
}

// Fallback for rows too wide for an LDS tile: global atomics straight into
// the (pre-cleared) accumulator.  One thread per hit, looping over rows.
template <bool COUNT>
__global__ void __launch_bounds__(256)
k_vote_global(const uint32_t *__restrict__ sphi, const uint64_t *__restrict__ offs, uint64_t n_hits,
              const uint32_t *__restrict__ layer_off, const uint32_t *__restrict__ O,
              const uint8_t *__restrict__ V, uint32_t n_layers, uint32_t rows, uint32_t nphi,
              uint32_t shift, uint32_t n_events, void *__restrict__ out)
{
  for (uint32_t e = blockIdx.y; e < n_events; e += gridDim.y) {
    const uint64_t b = min(offs[e], n_hits);
    const uint32_t *lo = layer_off + size_t(e) * (n_layers + 1);
    const uint32_t total = lo[n_layers];
    const uint64_t eb = uint64_t(e) * rows * nphi;
    for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < total; h += gridDim.x * blockDim.x) {
        uint32_t l = 0;
        while (l + 1 < n_layers && lo[l + 1] <= h) ++l;
        const uint32_t ph = sphi[b + h];
        for (uint32_t r = 0; r < rows; ++r) {
            const size_t ti = size_t(l) * rows + r;
            if (!V[ti]) continue;
            const uint64_t c = eb + uint64_t(r) * nphi + ((ph - O[ti]) >> shift);
            if (COUNT)
                atomicAdd(static_cast<uint32_t *>(out) + c, 1u);
            else
                atomicOr(reinterpret_cast<uint32_t *>(out) + (c >> 1), (1u << l) << ((c & 1) * 16));
        }
    }
  }
}

namespace {

template <int R, bool COUNT>
void launch_lds(hough_ctx *c, const hough_hits *h, void *out, uint32_t threads, hipStream_t s)
{
    const uint32_t n_tiles = (c->rows + R - 1) / R;
    const uint32_t n_items = n_tiles * h->n_events;
    const uint32_t per_cu = c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 2;
    const uint32_t grid = std::max(1u, std::min(n_items, uint32_t(c->n_cu) * per_cu));
    hipLaunchKernelGGL((k_vote_lds<R, COUNT>), dim3(grid), dim3(threads), size_t(R) * c->spec.n_phi * 4, s,
                       c->d_phi_a, h->event_offsets, h->n_hits, c->d_layer_off, c->d_O, c->d_V,
                       c->spec.n_layers, c->rows, c->spec.n_phi, c->shift, int(c->all_valid),
                       n_tiles, n_items, c->d_order, c->d_counters, out);
}

// The per-hit forms: layer bucketing, then LDS row tiles (or global atomics
// when a row is too wide for a tile).
template <bool COUNT>
hipError_t launch_vote_hits(hough_ctx *c, const hough_hits *h, void *out, hipStream_t s)
{
    hipError_t err;
    const uint32_t R = vote_rows(c);
    const bool lds = R > 0 && c->tun.vote_algo != 2;
    if (lds) {
        if ((err = launch_fill_u32(c, c->d_counters, 0, 1, s)) != hipSuccess) return err;
        if (h->n_events > 1) {
            if ((err = launch_event_order(c, h, s)) != hipSuccess) return err;
        } else if ((err = launch_fill_u32(c, c->d_order, 0, 1, s)) != hipSuccess) {
            return err;
        }
    }
    if ((err = launch_bucket_layers(c, h, false, s)) != hipSuccess) return err;
    KernelTimer t;
    if (!lds) {
        const size_t words = size_t(h->n_events) * c->cells / (COUNT ? 1 : 2);
        if ((err = launch_fill_u32(c, static_cast<uint32_t *>(out), 0, words, s)) != hipSuccess) return err;
        prof_begin(c, COUNT ? "vote_count_global" : "vote_global", s, &t);
        hipLaunchKernelGGL(k_vote_global<COUNT>, dim3(64, std::min(h->n_events, 65535u)), dim3(256), 0, s,
                           c->d_phi_a, h->event_offsets, h->n_hits, c->d_layer_off, c->d_O, c->d_V,
                           c->spec.n_layers, c->rows, c->spec.n_phi, c->shift, h->n_events, out);
        prof_end(c, s, &t);
        return hipGetLastError();
    }
    const uint32_t threads = c->tun.vote_threads ? c->tun.vote_threads : 256;
    prof_begin(c, COUNT ? "vote_count_lds" : "vote_lds", s, &t);
    switch (R) {
    case 1: launch_lds<1, COUNT>(c, h, out, threads, s); break;
    case 2: launch_lds<2, COUNT>(c, h, out, threads, s); break;
    case 4: launch_lds<4, COUNT>(c, h, out, threads, s); break;
    case 8: launch_lds<8, COUNT>(c, h, out, threads, s); break;
    case 16: launch_lds<16, COUNT>(c, h, out, threads, s); break;
    case 32: launch_lds<32, COUNT>(c, h, out, threads, s); break;
    default: launch_lds<64, COUNT>(c, h, out, threads, s); break;
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace

// Rows per LDS tile: the tuned value, else the largest power of two <= 64
// whose uint32 tile fits in 64 KB; 0 when even one row does not fit.
uint32_t vote_rows(const hough_ctx *c)
{
    uint32_t r = c->tun.vote_rows;
    if (!r) {
        r = 64;
        while (r > 0 && size_t(r) * c->spec.n_phi * 4 > c->max_lds) r >>= 1;
    }
    return r;
}

hipError_t launch_vote(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s)
{
    if (h->n_events == 0) return hipSuccess;
    if ((c->tun.vote_algo == 0 || c->tun.vote_algo == 5) && rank_vote_usable(c, acc))
        return launch_vote_rank(c, h, acc, s);
    if ((c->tun.vote_algo == 0 || c->tun.vote_algo == 4 || c->tun.vote_algo == 5) && direct_vote_usable(c))
        return launch_vote_direct(c, h, acc, s);
    if ((c->tun.vote_algo == 0 || c->tun.vote_algo == 3) && gap_vote_usable(c)) return launch_vote_gaps(c, h, acc, s);
    return launch_vote_hits<false>(c, h, acc, s);
}

hipError_t launch_vote_count(hough_ctx *c, const hough_hits *h, uint32_t *counts, hipStream_t s)
{
    if (h->n_events == 0) return hipSuccess;
    return launch_vote_hits<true>(c, h, counts, s);
}

}  // namespace hough
