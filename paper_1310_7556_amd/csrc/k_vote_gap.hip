// Step 1 of the transform in its exact gap form (Section 3, first step; the
// Discussion's A[B[i]] += 1 in layer-mask form), the default vote algorithm.
//
// A cell (row r, bin p) gets layer bit l iff some hit of layer l lies in the
// bin's azimuth interval [O[l][r] + p W, O[l][r] + (p+1) W), W = 2^32/n_phi.
// Equivalently the bit is absent iff that interval sits inside a gap
// between two cyclically consecutive hits of the layer: with a the hit
// before the gap and L its length (1 <= L <= 2^32), the bins emptied by the
// gap are exactly those whose start lies in [a + 1, a + L - W], and every
// empty bin belongs to exactly one gap.  A layer with many hits is therefore
// described by its few gaps longer than W instead of by its hits.
//
// A gap longer than W never lies inside one W-wide azimuth bucket: it runs
// from the largest hit of a non-empty bucket to the smallest hit of the next
// non-empty bucket (cyclically).  Per-bucket minima and maxima (LDS atomics)
// therefore give every such gap without sorting the hits.
//
// k_vote_scan (one workgroup per event) classifies each layer: empty,
// sparse (at most n_phi/2 hits: its hits are listed) or dense (its gaps
// longer than W are listed as {hit before the gap, length - 1}).  A layer's
// list holds at most as many entries as the layer has hits, so the lists of
// an event live in the event's own range of a hit-sized scratch buffer.
// k_vote_gaps (grid-stride over (event, R-row tile) items): every cell of a
// row starts with the bits of the dense layers that reach the row, sparse
// layers add their bits hit by hit, each (row, gap) pair of a dense layer
// clears that layer's bit in the bins the gap empties, and the tile is
// written once with coalesced stores.  The result is bit-identical to the
// per-hit vote, whatever the hit order.
#include "hough_internal.h"

namespace hough {

constexpr uint32_t kLayerEmpty = 0, kLayerSparse = 1, kLayerDense = 2;

// info[e][l] = {mode, entries, first list index, 0}.  Layers are scanned in
// groups whose bucket minima and maxima fit the LDS budget.
__global__ void __launch_bounds__(1024)
k_vote_scan(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
            const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_layers, uint32_t nphi,
            uint32_t shift, uint32_t group_layers, uint4 *__restrict__ info, uint2 *__restrict__ lists)
{
    HOUGH_DYNAMIC_LDS(uint32_t, lds);                // bmin[gl][nphi], bmax[gl][nphi]
    __shared__ uint32_t cnt[kMaxLayers], fill[kMaxLayers], start[kMaxLayers];
    const uint32_t e = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    const uint32_t scap = nphi / 2;
    const uint64_t W = uint64_t(1) << shift;
    const uint64_t b = min(offs[e], n_hits);
    uint64_t end = min(offs[e + 1], n_hits);
    if (end < b) end = b;
    if (t < kMaxLayers) {
        cnt[t] = 0;
        fill[t] = 0;
    }
    __syncthreads();
    for (uint64_t i = b + t; i < end; i += nt) {
        const uint32_t l = layer[i];
        if (l < n_layers) atomicAdd(&cnt[l], 1u);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (uint32_t l = 0; l < n_layers; ++l) {
            start[l] = run;
            run += cnt[l];
        }
    }
    __syncthreads();
    for (uint32_t l0 = 0; l0 < n_layers; l0 += group_layers) {
        const uint32_t gl = min(group_layers, n_layers - l0);
        uint32_t *bmin = lds, *bmax = lds + gl * nphi;
        for (uint32_t i = t; i < gl * nphi; i += nt) {
            bmin[i] = 0xFFFFFFFFu;
            bmax[i] = 0u;
        }
        __syncthreads();
        for (uint64_t i = b + t; i < end; i += nt) {
            const uint32_t l = layer[i];
            if (l >= l0 && l < l0 + gl) {
                const uint32_t ph = phi[i];
                const uint32_t bi = (l - l0) * nphi + (ph >> shift);
                atomicMin(&bmin[bi], ph);
                atomicMax(&bmax[bi], ph);
                if (cnt[l] <= scap) {
                    const uint32_t pos = atomicAdd(&fill[l], 1u);
                    lists[b + start[l] + pos] = make_uint2(ph, 0u);
                }
            }
        }
        __syncthreads();
        // one wave per layer of the group; no block barriers inside
        for (uint32_t ll = wave; ll < gl; ll += nwaves) {
            const uint32_t l = l0 + ll;
            const uint32_t n = cnt[l];
            uint2 *out = lists + b + start[l];
            uint32_t mode = kLayerEmpty, count = 0;
            if (n > 0 && n <= scap) {
                mode = kLayerSparse;
                count = n;
            } else if (n > scap) {
                mode = kLayerDense;
                const uint32_t *mn = bmin + ll * nphi, *mx = bmax + ll * nphi;
                // first non-empty bucket (a bucket is empty iff min > max);
                // one exists because the layer has hits
                uint32_t first = nphi;
                for (uint32_t base = 0; base < nphi && first == nphi; base += 64) {
                    const uint32_t i = base + lane;
                    const uint64_t bal = __ballot(i < nphi && mn[i] <= mx[i]);
                    if (bal) first = base + uint32_t(__builtin_ctzll(bal));
                }
                // chunks from the top down; carry = the lowest non-empty
                // bucket above the current chunk, or first + nphi (wrap)
                uint32_t carry = first + nphi;
                for (int base = int((nphi - 1) & ~63u); base >= 0; base -= 64) {
                    const uint32_t i = uint32_t(base) + lane;
                    const bool ne = i < nphi && mn[i] <= mx[i];
                    const uint64_t bal = __ballot(ne);
                    const uint64_t above = lane == 63 ? 0ull : (bal & ~((2ull << lane) - 1ull));
                    const uint32_t nxt = above ? uint32_t(base) + uint32_t(__builtin_ctzll(above)) : carry;
                    bool big = false;
                    uint32_t ga = 0, glen1 = 0;
                    if (ne) {
                        const bool wrap = nxt >= nphi;
                        const uint32_t j = wrap ? nxt - nphi : nxt;
                        const uint32_t a = mx[i];
                        const uint64_t bnext = uint64_t(mn[j]) + (wrap ? (uint64_t(1) << 32) : 0ull);
                        const uint64_t len = bnext - a;
                        big = len > W;
                        ga = a;
                        glen1 = uint32_t(len - 1);
                    }
                    const uint64_t bb = __ballot(big);
                    if (big) out[count + __popcll(bb & ((1ull << lane) - 1ull))] = make_uint2(ga, glen1);
                    count += __popcll(bb);
                    if (bal) carry = uint32_t(base) + uint32_t(__builtin_ctzll(bal));
                }
            }
            if (lane == 0) info[size_t(e) * n_layers + l] = make_uint4(mode, count, uint32_t(b + start[l]), 0u);
        }
        __syncthreads();
    }
}

template <int R>
__global__ void __launch_bounds__(1024)
k_vote_gaps(const uint4 *__restrict__ info, const uint2 *__restrict__ lists, const uint32_t *__restrict__ O,
            const uint8_t *__restrict__ V, uint32_t n_layers, uint32_t rows, uint32_t nphi, uint32_t log2phi,
            uint32_t shift, int all_valid, uint32_t n_tiles, uint32_t n_items, uint16_t *__restrict__ acc)
{
    constexpr uint32_t LR = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : R == 16 ? 4 : R == 32 ? 5 : 6;
    HOUGH_DYNAMIC_LDS(uint32_t, tile);               // [R][nphi / 2] packed cell pairs
    __shared__ uint32_t rmask[R];
    const uint32_t t = threadIdx.x, nt = blockDim.x;  // nt is a multiple of 64 >= R
    const uint64_t cells = uint64_t(rows) * nphi;
    const uint32_t half = nphi >> 1;
    const uint32_t rr = t & (R - 1);                  // this thread's row within a tile, fixed
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t e = item / n_tiles;
        const uint32_t r0 = (item % n_tiles) * R;
        const uint32_t nr = min(uint32_t(R), rows - r0);
        const uint4 *inf = info + size_t(e) * n_layers;
        if (t < R) {
            uint32_t m = 0;
            if (t < nr)
                for (uint32_t l = 0; l < n_layers; ++l)
                    if (inf[l].x == kLayerDense && (all_valid || V[size_t(l) * rows + r0 + t])) m |= 1u << l;
            rmask[t] = m | (m << 16);
        }
        __syncthreads();
        for (uint32_t i = t; i < nr * half; i += nt) tile[i] = rmask[i >> (log2phi - 1)];
        __syncthreads();
        const bool row_in = rr < nr;
        for (uint32_t l = 0; l < n_layers; ++l) {
            const uint4 hd = inf[l];
            const uint32_t mode = __builtin_amdgcn_readfirstlane(hd.x);
            const uint32_t count = __builtin_amdgcn_readfirstlane(hd.y);
            if (mode == kLayerEmpty || count == 0) continue;
            const uint2 *lst = lists + __builtin_amdgcn_readfirstlane(hd.z);
            const size_t ti = size_t(l) * rows + r0 + rr;
            if (!row_in || !(all_valid || V[ti])) continue;
            const uint32_t o = O[ti];
            const uint32_t bit = 1u << l;
            uint32_t *trow = tile + rr * half;
            if (mode == kLayerSparse) {
                for (uint32_t g = t >> LR; g < count; g += nt >> LR) {
                    const uint32_t p = (lst[g].x - o) >> shift;
                    atomicOr(&trow[p >> 1], bit << ((p & 1) * 16));
                }
            } else {
                for (uint32_t g = t >> LR; g < count; g += nt >> LR) {
                    const uint2 it = lst[g];
                    // bins p whose start o + p W lies in [a + 1, a + L - W]:
                    // x0 = a + 1 - o, the first such p is ceil(x0 / W), and
                    // the run continues while p W - x0 <= L - W - 1
                    const uint32_t x0 = it.x + 1u - o;
                    const uint64_t plo = (uint64_t(x0) + (uint64_t(1) << shift) - 1) >> shift;
                    const uint64_t delta = (plo << shift) - x0;
                    const uint64_t len = uint64_t(it.y) + 1 - (uint64_t(1) << shift);
                    if (delta < len) {
                        const uint32_t n_empty = uint32_t((len - 1 - delta) >> shift) + 1;
                        for (uint32_t q = 0; q < n_empty; ++q) {
                            const uint32_t p = (uint32_t(plo) + q) & (nphi - 1);
                            atomicAnd(&trow[p >> 1], ~(bit << ((p & 1) * 16)));
                        }
                    }
                }
            }
        }
        __syncthreads();
        uint32_t *dst = reinterpret_cast<uint32_t *>(acc + uint64_t(e) * cells + uint64_t(r0) * nphi);
        for (uint32_t i = t; i < nr * half; i += nt) dst[i] = tile[i];
        __syncthreads();
    }
}

namespace {

template <int R>
void launch_gaps(hough_ctx *c, uint32_t n_events, uint16_t *acc, uint32_t threads, hipStream_t s)
{
    const uint32_t n_tiles = (c->rows + R - 1) / R;
    const uint32_t n_items = n_tiles * n_events;
    const uint32_t per_cu = c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 4;
    const uint32_t grid = std::max(1u, std::min(n_items, uint32_t(c->n_cu) * per_cu));
    hipLaunchKernelGGL(k_vote_gaps<R>, dim3(grid), dim3(threads), size_t(R) * c->spec.n_phi * 2, s, c->d_gap_info,
                       c->d_gap_list, c->d_O, c->d_V, c->spec.n_layers, c->rows, c->spec.n_phi, c->log2_phi,
                       c->shift, int(c->all_valid), n_tiles, n_items, acc);
}

}  // namespace

// Rows per gap-vote tile: the tuned value, else 32, halved while the packed
// uint16 tile exceeds the LDS budget; 0 when one row does not fit.
uint32_t gap_rows(const hough_ctx *c)
{
    uint32_t r = c->tun.vote_rows ? c->tun.vote_rows : 32;
    while (r > 1 && size_t(r) * c->spec.n_phi * 2 > c->max_lds) r >>= 1;
    return size_t(r) * c->spec.n_phi * 2 <= c->max_lds ? r : 0;
}

// The scan needs the minima and maxima of one layer's n_phi buckets in LDS
// (then one packed row, and every valid tuned tile, fits as well).
bool gap_vote_usable(const hough_ctx *c)
{
    return size_t(c->spec.n_phi) * 8 <= c->max_lds;
}

hipError_t launch_vote_gaps(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s)
{
    const uint32_t E = h->n_events;
    const uint32_t group = uint32_t(std::min<size_t>(c->spec.n_layers, c->max_lds / (size_t(c->spec.n_phi) * 8)));
    KernelTimer t;
    prof_begin(c, "vote_scan", s, &t);
    hipLaunchKernelGGL(k_vote_scan, dim3(E), dim3(1024), size_t(group) * c->spec.n_phi * 8, s, h->layer, h->phi,
                       h->event_offsets, h->n_hits, c->spec.n_layers, c->spec.n_phi, c->shift, group,
                       c->d_gap_info, c->d_gap_list);
    prof_end(c, s, &t);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const uint32_t R = gap_rows(c);
    const uint32_t threads = std::max(64u, c->tun.vote_threads ? c->tun.vote_threads : 256u);
    prof_begin(c, "vote_gaps", s, &t);
    switch (R) {
    case 1: launch_gaps<1>(c, E, acc, threads, s); break;
    case 2: launch_gaps<2>(c, E, acc, threads, s); break;
    case 4: launch_gaps<4>(c, E, acc, threads, s); break;
    case 8: launch_gaps<8>(c, E, acc, threads, s); break;
    case 16: launch_gaps<16>(c, E, acc, threads, s); break;
    case 32: launch_gaps<32>(c, E, acc, threads, s); break;
    default: launch_gaps<64>(c, E, acc, threads, s); break;
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
