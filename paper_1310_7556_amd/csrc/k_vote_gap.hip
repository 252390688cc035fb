// Step 1 of the transform in its exact gap form (Section 4, first step; the
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
// k_vote_gaps (grid-stride over items of one event and a run of R-row
// tiles): the event's layer info and, when they fit, all its list entries
// are staged in LDS once per item and reused by every tile of the run.  In a
// tile every cell of a row starts with the bits of the dense layers that
// reach the row, sparse layers add their bits hit by hit, each (row, gap)
// pair of a dense layer clears that layer's bit in the bins the gap empties,
// and the tile is written once with coalesced 16-byte stores.  The result is
// bit-identical to the per-hit vote, whatever the hit order.
#include "hough_internal.h"

namespace hough {

constexpr uint32_t kLayerEmpty = 0, kLayerSparse = 1, kLayerDense = 2;

// Calls f(layer, phi) for every hit of [b, end).  With `vec` (layer 4-byte
// and phi 16-byte aligned) the aligned middle is read four hits per load.
template <bool PHI, class F>
__device__ __forceinline__ void for_event_hits(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
                                               uint64_t b, uint64_t end, uint32_t t, uint32_t nt, bool vec, F &&f)
{
    uint64_t tail = b;
    if (vec) {
        const uint64_t a = min((b + 3) & ~uint64_t(3), end);
        if (t < a - b) f(uint32_t(layer[b + t]), PHI ? phi[b + t] : 0u);
        const uint64_t nq = (end - a) >> 2;
        const uint32_t *l4 = reinterpret_cast<const uint32_t *>(layer + a);
        const uint4 *p4 = reinterpret_cast<const uint4 *>(phi + a);
        for (uint64_t q = t; q < nq; q += nt) {
            const uint32_t lw = l4[q];
            uint4 pw = make_uint4(0u, 0u, 0u, 0u);
            if (PHI) pw = p4[q];
            f(lw & 0xFFu, pw.x);
            f((lw >> 8) & 0xFFu, pw.y);
            f((lw >> 16) & 0xFFu, pw.z);
            f(lw >> 24, pw.w);
        }
        tail = a + (nq << 2);
    }
    for (uint64_t i = tail + t; i < end; i += nt) f(uint32_t(layer[i]), PHI ? phi[i] : 0u);
}

// info[e][l] = {mode, entries, first list index, 0}.  Layers are scanned in
// groups whose bucket minima and maxima fit the LDS budget; with a single
// group the hit counts come from the same pass as the minima and maxima and
// the hits are read a second time only to list the sparse layers.
__global__ void __launch_bounds__(1024)
k_vote_scan(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
            const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_layers, uint32_t nphi,
            uint32_t shift, uint32_t group_layers, int vec, uint4 *__restrict__ info, uint2 *__restrict__ lists)
{
    HOUGH_DYNAMIC_LDS(uint32_t, lds);                // bmin[gl][nphi], bmax[gl][nphi]
    __shared__ uint32_t cnt[kMaxLayers], fill[kMaxLayers], start[kMaxLayers];
    __shared__ uint32_t any_sparse;
    const uint32_t e = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    const uint32_t scap = nphi / 2;
    const uint64_t W = uint64_t(1) << shift;
    const uint64_t b = min(offs[e], n_hits);
    uint64_t end = min(offs[e + 1], n_hits);
    if (end < b) end = b;
    const bool one = group_layers >= n_layers;
    if (t < kMaxLayers) {
        cnt[t] = 0;
        fill[t] = 0;
    }
    __syncthreads();
    auto prefix = [&]() {
        if (t == 0) {
            uint32_t run = 0, sp = 0;
            for (uint32_t l = 0; l < n_layers; ++l) {
                start[l] = run;
                run += cnt[l];
                sp |= cnt[l] > 0 && cnt[l] <= scap;
            }
            any_sparse = sp;
        }
        __syncthreads();
    };
    if (!one) {
        for_event_hits<false>(layer, phi, b, end, t, nt, vec, [&](uint32_t l, uint32_t) {
            if (l < n_layers) atomicAdd(&cnt[l], 1u);
        });
        __syncthreads();
        prefix();
    }
    for (uint32_t l0 = 0; l0 < n_layers; l0 += group_layers) {
        const uint32_t gl = min(group_layers, n_layers - l0);
        uint32_t *bmin = lds, *bmax = lds + gl * nphi;
        for (uint32_t i = t; i < gl * nphi; i += nt) {
            bmin[i] = 0xFFFFFFFFu;
            bmax[i] = 0u;
        }
        __syncthreads();
        for_event_hits<true>(layer, phi, b, end, t, nt, vec, [&](uint32_t l, uint32_t ph) {
            if (l >= l0 && l < l0 + gl) {
                const uint32_t bi = (l - l0) * nphi + (ph >> shift);
                atomicMin(&bmin[bi], ph);
                atomicMax(&bmax[bi], ph);
                if (one) {
                    atomicAdd(&cnt[l], 1u);
                } else if (cnt[l] <= scap) {
                    lists[b + start[l] + atomicAdd(&fill[l], 1u)] = make_uint2(ph, 0u);
                }
            }
        });
        __syncthreads();
        if (one) {
            prefix();
            if (any_sparse) {
                for_event_hits<true>(layer, phi, b, end, t, nt, vec, [&](uint32_t l, uint32_t ph) {
                    if (l < n_layers && cnt[l] <= scap)
                        lists[b + start[l] + atomicAdd(&fill[l], 1u)] = make_uint2(ph, 0u);
                });
            }
        }
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

// Dynamic LDS of k_vote_gaps, in bytes: the packed tile, the per-(layer,
// row) offsets, then `cap` staged list entries.
__host__ __device__ inline size_t gap_tile_bytes(uint32_t R, uint32_t nphi) { return (size_t(R) * nphi * 2 + 15) & ~size_t(15); }
__host__ __device__ inline size_t gap_offs_bytes(uint32_t R, uint32_t L) { return (size_t(R) * L * 4 + 15) & ~size_t(15); }
inline size_t gap_lds_bytes(uint32_t R, uint32_t nphi, uint32_t L, uint32_t cap)
{
    return gap_tile_bytes(R, nphi) + gap_offs_bytes(R, L) + size_t(cap) * 8;
}

template <int R>
__global__ void __launch_bounds__(1024)
k_vote_gaps(const uint4 *__restrict__ info, const uint2 *__restrict__ lists, const uint32_t *__restrict__ O,
            const uint8_t *__restrict__ V, uint32_t n_layers, uint32_t rows, uint32_t nphi, uint32_t log2phi,
            uint32_t shift, int all_valid, uint32_t n_tiles, uint32_t run_tiles, uint32_t runs_per_event,
            uint32_t n_items, uint32_t cap, int vec_store, uint16_t *__restrict__ acc)
{
    constexpr uint32_t LR = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : R == 16 ? 4 : R == 32 ? 5 : 6;
    HOUGH_DYNAMIC_LDS(uint4, lds4);
    uint32_t *tile = reinterpret_cast<uint32_t *>(lds4);                    // [R][nphi / 2] cell pairs
    uint32_t *o_s = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(lds4) + gap_tile_bytes(R, nphi));
    uint2 *ent = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(o_s) + gap_offs_bytes(R, n_layers));
    __shared__ uint4 linf[kMaxLayers];
    __shared__ uint32_t pre[kMaxLayers + 1];          // flattened list start of each layer
    __shared__ uint32_t sl[kMaxLayers], sh[kMaxLayers], upre[kMaxLayers + 1];
    __shared__ uint64_t vl[kMaxLayers];               // rows of the tile that layer l reaches
    __shared__ uint32_t rmask[R];
    __shared__ uint32_t dense_s;
    const uint32_t t = threadIdx.x, nt = blockDim.x;  // nt is a multiple of 64 >= R
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    const uint64_t cells = uint64_t(rows) * nphi;
    const uint32_t half = nphi >> 1;
    const uint32_t wmask = (1u << shift) - 1u;        // W - 1

    // entries [c0, c0 + cn) of the event's flattened lists into LDS, and the
    // work units over them: runs of up to 64 entries of one layer
    auto stage = [&](uint32_t c0, uint32_t cn) {
        for (uint32_t f = t; f < cn; f += nt) {
            const uint32_t g = c0 + f;
            uint32_t l = 0;
            while (g >= pre[l + 1]) ++l;
            ent[f] = lists[linf[l].z + (g - pre[l])];
        }
        if (t == 0) {
            uint32_t u = 0;
            for (uint32_t l = 0; l < n_layers; ++l) {
                const uint32_t lo = min(max(pre[l], c0), c0 + cn) - c0;
                const uint32_t hi = min(max(pre[l + 1], c0), c0 + cn) - c0;
                sl[l] = lo;
                sh[l] = hi;
                upre[l] = u;
                u += (hi - lo + 63) >> 6;
            }
            upre[n_layers] = u;
        }
    };
    // one wave per unit: each lane takes one entry and applies it to every
    // row of the tile, with the layer's row offsets held in registers
    auto vote = [&]() {
        const uint32_t nunits = upre[n_layers];
        for (uint32_t u = wave; u < nunits; u += nwaves) {
            uint32_t l = 0;
            while (upre[l + 1] <= u) ++l;
            const uint32_t j = sl[l] + ((u - upre[l]) << 6) + lane;
            const bool act = j < sh[l];
            const uint2 it = ent[act ? j : sl[l]];
            const uint64_t rows_ok = act ? vl[l] : 0ull;
            const bool sparse = linf[l].x == kLayerSparse;
            const uint32_t bit = 1u << l;
            uint32_t ov[R];
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) ov[r] = o_s[l * R + r];
            if (sparse) {
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    if (!((rows_ok >> r) & 1ull)) continue;
                    const uint32_t p = (it.x - ov[r]) >> shift;
                    atomicOr(&tile[r * half + (p >> 1)], bit << ((p & 1) * 16));
                }
            } else {
                const uint32_t len = it.y - wmask;  // L - W (> 0)
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    if (!((rows_ok >> r) & 1ull)) continue;
                    // bins p whose start o + p W lies in [a + 1, a + L - W]
                    // (mod 2^32): with x0 = a + 1 - o, the first such p is
                    // ceil(x0 / W) mod n_phi, delta = its start - x0, and the
                    // run continues while delta + q W <= L - W - 1
                    const uint32_t x0 = it.x + 1u - ov[r];
                    const uint32_t delta = (0u - x0) & wmask;
                    if (delta < len) {
                        const uint32_t p0 = (x0 + wmask) >> shift;
                        const uint32_t n_empty = ((len - 1 - delta) >> shift) + 1;
                        for (uint32_t q = 0; q < n_empty; ++q) {
                            const uint32_t p = (p0 + q) & (nphi - 1);
                            atomicAnd(&tile[r * half + (p >> 1)], ~(bit << ((p & 1) * 16)));
                        }
                    }
                }
            }
        }
    };

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t e = item / runs_per_event;
        const uint32_t tile_lo = (item % runs_per_event) * run_tiles;
        const uint32_t tile_hi = min(n_tiles, tile_lo + run_tiles);
        if (t < n_layers) linf[t] = info[size_t(e) * n_layers + t];
        __syncthreads();
        if (t == 0) {
            uint32_t run = 0, dense = 0;
            for (uint32_t l = 0; l < n_layers; ++l) {
                pre[l] = run;
                if (linf[l].x != kLayerEmpty) run += linf[l].y;
                if (linf[l].x == kLayerDense) dense |= 1u << l;
            }
            pre[n_layers] = run;
            dense_s = dense;
        }
        __syncthreads();
        const uint32_t total = pre[n_layers];
        const uint32_t dense = dense_s;
        const bool staged = total <= cap;
        if (staged) stage(0, total);
        for (uint32_t tl = tile_lo; tl < tile_hi; ++tl) {
            const uint32_t r0 = tl * R;
            const uint32_t nr = min(uint32_t(R), rows - r0);
            for (uint32_t i = t; i < n_layers * R; i += nt) {
                const uint32_t l = i >> LR, r = i & (R - 1);
                o_s[i] = r < nr ? O[size_t(l) * rows + r0 + r] : 0u;
            }
            if (t < n_layers) {
                uint64_t m = 0;
                for (uint32_t r = 0; r < nr; ++r)
                    if (all_valid || V[size_t(t) * rows + r0 + r]) m |= 1ull << r;
                vl[t] = m;
            }
            if (t < R) {
                uint32_t m = 0;
                if (t < nr) {
#pragma unroll
                    for (uint32_t l = 0; l < kMaxLayers; ++l)
                        if (l < n_layers && ((dense >> l) & 1u) && (all_valid || V[size_t(l) * rows + r0 + t]))
                            m |= 1u << l;
                }
                rmask[t] = m | (m << 16);
            }
            __syncthreads();
            for (uint32_t i = t; i < nr * half; i += nt) tile[i] = rmask[i >> (log2phi - 1)];
            __syncthreads();
            if (staged) {
                vote();
            } else {
                for (uint32_t c0 = 0; c0 < total; c0 += cap) {
                    stage(c0, min(cap, total - c0));
                    __syncthreads();
                    vote();
                    __syncthreads();
                }
            }
            __syncthreads();
            uint16_t *dst = acc + uint64_t(e) * cells + uint64_t(r0) * nphi;
            const uint32_t nw = nr * half;
            if (vec_store) {
                const uint4 *src4 = reinterpret_cast<const uint4 *>(tile);
                uint4 *dst4 = reinterpret_cast<uint4 *>(dst);
                for (uint32_t i = t; i < (nw >> 2); i += nt) dst4[i] = src4[i];
            } else {
                uint32_t *dst1 = reinterpret_cast<uint32_t *>(dst);
                for (uint32_t i = t; i < nw; i += nt) dst1[i] = tile[i];
            }
        }
        __syncthreads();
    }
}

namespace {

template <int R>
void launch_gaps(hough_ctx *c, uint32_t n_events, uint16_t *acc, uint32_t threads, uint32_t cap, hipStream_t s)
{
    const uint32_t n_tiles = (c->rows + R - 1) / R;
    const uint32_t per_cu = c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 4;
    const uint64_t want = uint64_t(c->n_cu) * per_cu;
    // runs of tiles sharing one staging of the event's lists: as long as
    // there are still about four items per workgroup
    const uint64_t all = uint64_t(n_tiles) * n_events;
    const uint32_t run = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(n_tiles, all / (want * 4))));
    const uint32_t runs = (n_tiles + run - 1) / run;
    const uint32_t n_items = runs * n_events;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(n_items, want)));
    const int vec = c->spec.n_phi >= 8 && (reinterpret_cast<uintptr_t>(acc) & 15) == 0;
    hipLaunchKernelGGL(k_vote_gaps<R>, dim3(grid), dim3(threads), gap_lds_bytes(R, c->spec.n_phi, c->spec.n_layers, cap),
                       s, c->d_gap_info, c->d_gap_list, c->d_O, c->d_V, c->spec.n_layers, c->rows, c->spec.n_phi,
                       c->log2_phi, c->shift, int(c->all_valid), n_tiles, run, runs, n_items, cap, vec, acc);
}

// Staged list entries per workgroup: up to 1024, within the LDS budget.
uint32_t gap_stage_cap(const hough_ctx *c, uint32_t R)
{
    const size_t fixed = gap_tile_bytes(R, c->spec.n_phi) + gap_offs_bytes(R, c->spec.n_layers);
    if (fixed + 64 * 8 > c->max_lds) return 0;
    return uint32_t(std::min<size_t>(1024, (c->max_lds - fixed) / 8));
}

}  // namespace

// Rows per gap-vote tile: the tuned value, else 32, halved until the tile,
// the row offsets and a staging area of at least 64 entries fit in LDS.
uint32_t gap_rows(const hough_ctx *c)
{
    uint32_t r = c->tun.vote_rows ? c->tun.vote_rows : 32;
    while (r > 1 && !gap_stage_cap(c, r)) r >>= 1;
    return gap_stage_cap(c, r) ? r : 0;
}

// The scan needs the minima and maxima of one layer's n_phi buckets in LDS.
bool gap_vote_usable(const hough_ctx *c)
{
    return size_t(c->spec.n_phi) * 8 <= c->max_lds && gap_rows(c) > 0;
}

hipError_t launch_vote_gaps(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s)
{
    const uint32_t E = h->n_events;
    const uint32_t group = uint32_t(std::min<size_t>(c->spec.n_layers, c->max_lds / (size_t(c->spec.n_phi) * 8)));
    const int vec = (reinterpret_cast<uintptr_t>(h->layer) & 3) == 0 && (reinterpret_cast<uintptr_t>(h->phi) & 15) == 0;
    KernelTimer t;
    prof_begin(c, "vote_scan", s, &t);
    hipLaunchKernelGGL(k_vote_scan, dim3(E), dim3(1024), size_t(group) * c->spec.n_phi * 8, s, h->layer, h->phi,
                       h->event_offsets, h->n_hits, c->spec.n_layers, c->spec.n_phi, c->shift, group, vec,
                       c->d_gap_info, c->d_gap_list);
    prof_end(c, s, &t);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    uint32_t R = gap_rows(c);
    if (!c->tun.vote_rows) {
        // small batches: narrower tiles until there are enough of them
        const uint64_t want = uint64_t(c->n_cu) * (c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 4);
        while (R > 8 && uint64_t((c->rows + R - 1) / R) * E < want) R >>= 1;
    }
    const uint32_t cap = gap_stage_cap(c, R);
    const uint32_t threads = std::max(64u, c->tun.vote_threads ? c->tun.vote_threads : 256u);
    prof_begin(c, "vote_gaps", s, &t);
    switch (R) {
    case 1: launch_gaps<1>(c, E, acc, threads, cap, s); break;
    case 2: launch_gaps<2>(c, E, acc, threads, cap, s); break;
    case 4: launch_gaps<4>(c, E, acc, threads, cap, s); break;
    case 8: launch_gaps<8>(c, E, acc, threads, cap, s); break;
    case 16: launch_gaps<16>(c, E, acc, threads, cap, s); break;
    case 32: launch_gaps<32>(c, E, acc, threads, cap, s); break;
    default: launch_gaps<64>(c, E, acc, threads, cap, s); break;
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
