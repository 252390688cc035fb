// Step 1 of the transform (Section 4, first step; the Discussion's
// A[B[i]] += 1 in its layer-mask form) in a rank form that decides four
// (cell, layer) pairs with one 32-bit operation.  The default vote.
//
// Bin p of row r (offset o = J W + F, W = 2^32 / n_phi) holds a hit of layer
// l unless bucket j = J + p is empty at F: F in [lo_j, hi_j], with lo_j the
// largest fine offset of bucket j plus one (0 when the bucket is empty) and
// hi_j the smallest fine offset of bucket j + 1 (W - 1 when empty); this is
// the bucket-bounds form of k_vote_direct.hip.  Within a tile of at most 128
// consecutive rows only the order of the rows' fine offsets matters: with
// the tile's F values sorted, F_r in [lo, hi] iff rank_r in [a, b), where
// rank_r = #{F < F_r}, a = #{F < lo} and b = #{F <= hi}.  Rank, a and the
// span b - a all fit a byte (at most 128), so a word holds the (a, span) of
// four consecutive buckets, and with R = 0x80 + rank in every byte
//     x = R - a,  y = x - span
// never borrow across bytes (x in [0, 255], y >= rank); bucket byte k is
// empty iff bit 7 of x is set and bit 7 of y is clear.  Per row and layer,
// rank and J are wave-uniform scalars from a static table; a lane owns
// groups of four consecutive cells and keeps the (a, span) words of its
// buckets in registers while the row's J is unchanged (J moves by at most a
// fraction of a bin per row).  Layer bits are shifted into byte-wide masks
// and interleaved into uint16 cells with byte permutes.  Bit-identical to
// the per-hit vote; no atomics outside the bucket bounds, no divergence.
//
// Items are (event, run of 128-row tiles).  With BOUNDS an item covers a
// whole event and first finds the bucket bounds from the event's hits in
// LDS (the hits are read once, no table goes through HBM); otherwise the
// bounds come from k_vote_bounds' per-event table, for single large events
// split into many items.
#include <algorithm>
#include <vector>

#include "hough_internal.h"

namespace hough {

namespace {

// Calls f(layer, phi) for every hit of [b, end); with `vec` (layer 4-byte
// and phi 16-byte aligned) the aligned middle is read four hits per load.
template <class F>
__device__ __forceinline__ void rank_event_hits(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
                                                uint64_t b, uint64_t end, uint32_t t, uint32_t nt, bool vec, F &&f)
{
    uint64_t tail = b;
    if (vec) {
        const uint64_t a = min((b + 3) & ~uint64_t(3), end);
        if (t < a - b) f(uint32_t(layer[b + t]), phi[b + t]);
        const uint64_t nq = (end - a) >> 2;
        const uint32_t *l4 = reinterpret_cast<const uint32_t *>(layer + a);
        const uint4 *p4 = reinterpret_cast<const uint4 *>(phi + a);
        // four groups of four hits per thread per step, all loads issued
        // before any is used, so a step waits for memory once
        constexpr uint32_t U = 4;
        for (uint64_t q0 = t; q0 < nq; q0 += U * uint64_t(nt)) {
            uint32_t lw[U];
            uint4 pw[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint64_t q = q0 + u * uint64_t(nt);
                lw[u] = q < nq ? l4[q] : 0xFFFFFFFFu;       // layer 255: ignored
                pw[u] = q < nq ? p4[q] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                f(lw[u] & 0xFFu, pw[u].x);
                f((lw[u] >> 8) & 0xFFu, pw[u].y);
                f((lw[u] >> 16) & 0xFFu, pw[u].z);
                f(lw[u] >> 24, pw[u].w);
            }
        }
        tail = a + (nq << 2);
    }
    for (uint64_t i = tail + t; i < end; i += nt) f(uint32_t(layer[i]), phi[i]);
}

// #{s[k] < x} over a tile's sorted fine offsets s[0..count) and their
// index (kRankIndexAt: smallest f0, largest f1, shift sh, count, then the
// bytes ix[b] = #{s < f0 + b 2^sh}, b = 0..256): outside [f0, f1] the rank
// is 0 or count; inside, part b = (x - f0) >> sh narrows it to [ix[b],
// ix[b + 1]), searched by bisection (one or two values on average, where a
// bisection of all 128 takes eight dependent reads).
__device__ __forceinline__ uint32_t rank_below(const uint32_t *s, uint32_t x)
{
    const uint32_t f0 = s[kRankIndexAt], f1 = s[kRankIndexAt + 1], sh = s[kRankIndexAt + 2];
    const uint32_t cnt = s[kRankIndexAt + 3];
    if (cnt == 0 || x <= f0) return 0;
    if (x > f1) return cnt;
    const uint8_t *ix = reinterpret_cast<const uint8_t *>(s + kRankIndexAt + 4);
    const uint32_t b = (x - f0) >> sh;
    uint32_t lo = ix[b], hi = ix[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// #{v < x} over all rows' sorted fine offsets of a layer, with the layout
// of RankGlobLayout (header, 16-bit part counts, values): as rank_below.
__device__ __forceinline__ uint32_t rank_all(const uint32_t *s, uint32_t x)
{
    const uint32_t f0 = s[0], f1 = s[1], sh = s[2], cnt = s[3];
    if (cnt == 0 || x <= f0) return 0;
    if (x > f1) return cnt;
    const uint16_t *ix = reinterpret_cast<const uint16_t *>(s + 4);
    const uint32_t *v = s + kRankGlobAt;
    const uint32_t b = (x - f0) >> sh;
    uint32_t lo = ix[b], hi = ix[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (v[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace

// NL > 0: exactly NL layers; NL == 0: L (at most 16) at run time.  ALLV:
// every (row, layer) pair is reachable.
template <int G, int NL, bool ALLV, bool BOUNDS>
__global__ void __launch_bounds__(kRankThreads)
k_vote_rank(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi, const uint64_t *__restrict__ offs,
            uint64_t n_hits, int vec, const uint2 *__restrict__ tab, const uint32_t *__restrict__ rk_info,
            const uint32_t *__restrict__ rk_sorted, const uint32_t *__restrict__ rk_glob,
            const uint32_t *__restrict__ rk_cnt, uint32_t gstride, uint32_t cstride,
            uint32_t L, uint32_t rows, uint32_t nphi, uint32_t log2phi,
            uint32_t shift, uint32_t n_tiles, uint32_t run_tiles, uint32_t runs_per_event,
            uint16_t *__restrict__ acc)
{
    constexpr int LMAX = NL > 0 ? NL : 16;
    HOUGH_DYNAMIC_LDS(uint4, lds4);                  // 16-byte aligned: no static LDS in this kernel
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t lane = t & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6), nwaves = nt >> 6;
    const uint32_t wmask = (1u << shift) - 1u;
    const uint32_t ngrp = nphi >> 2;                 // 4-bucket groups per layer
    const uint32_t item = blockIdx.x;
    const uint32_t e = item / runs_per_event;
    const uint32_t tile_lo = (item % runs_per_event) * run_tiles;
    const uint32_t tile_hi = min(n_tiles, tile_lo + run_tiles);

    // LDS.  Tile items (!BOUNDS): the byte tables, the tile's sorted
    // offsets, the list of (layer, bucket) entries that can be empty, its
    // length.  Event items (BOUNDS), over the same bytes in turn: [bmin |
    // bmax] (N = L * nphi entries each) while the bounds are found; all
    // rows' sorted offsets per layer while each entry's interval [lo, hi]
    // is ranked against them; then those ranks, g(lo) | g(hi + 1) << 16 per
    // entry, the byte tables and the tile's counts cnt -- 8 N bytes in all
    // (40 KB for ten layers of 512 bins).
    const uint32_t N = L * nphi;
    uint32_t *bmin = lds, *bmax = lds + (BOUNDS ? N : 0);
    uint32_t *p_g = lds;                                          // BOUNDS: [N] global ranks
    uint32_t *bytes = lds + (BOUNDS ? N : 0);                     // [L][ngrp + 1] x {a word, span word}
    uint32_t *srt = bytes + L * (ngrp + 1) * 2;                   // [L][kRankSortStride] or [L][cstride]
    uint16_t *ivl = reinterpret_cast<uint16_t *>(srt + L * kRankSortStride);   // !BOUNDS: [N]
    uint32_t &n_ivl = *(srt + L * kRankSortStride + (N + 1) / 2);              // !BOUNDS: the list's length
    // BOUNDS: the entries i = t + k * kRankThreads (k < EPT) of this thread,
    // bit k set when entry i has an interval
    constexpr uint32_t EPT = (LMAX * 256 * G + kRankThreads - 1) / kRankThreads;   // n_phi = 256 G
    uint32_t has_bits = 0;

    if (BOUNDS) {
        // 16-byte stores (L * nphi is a multiple of 4; bmin is 16-byte aligned)
        uint4 *b4 = reinterpret_cast<uint4 *>(bmin);
        for (uint32_t i = t; i < L * nphi / 2; i += nt)
            b4[i] = i < L * nphi / 4 ? make_uint4(~0u, ~0u, ~0u, ~0u) : make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
        const uint64_t b = min(offs[e], n_hits);
        uint64_t end = min(offs[e + 1], n_hits);
        if (end < b) end = b;
        rank_event_hits(layer, phi, b, end, t, nt, vec != 0, [&](uint32_t l, uint32_t ph) {
            if (l < L) {
                const uint32_t i = l * nphi + (ph >> shift), f = ph & wmask;
                atomicMin(&bmin[i], f);
                atomicMax(&bmax[i], f);
            }
        });
    }

    // The interval [lo, hi] of a (layer, bucket) entry i: the fine offsets at
    // which its bin is empty; lo > hi when it never is.
    auto interval = [&](uint32_t i, uint32_t &lo, uint32_t &hi) {
        const uint32_t l = i >> log2phi, j = i & (nphi - 1);
        if (BOUNDS) {
            const uint32_t jn = l * nphi + ((j + 1) & (nphi - 1));
            const bool ne = bmin[i] <= bmax[i], ne1 = bmin[jn] <= bmax[jn];
            lo = ne ? bmax[i] + 1u : 0u;                     // may be W: never empty
            hi = ne1 ? bmin[jn] : wmask;
        } else {
            const uint2 v = tab[(size_t(e) * L + l) * nphi + j];
            lo = v.x;                                        // 0xFFFFFFFF: never empty
            hi = v.x == 0xFFFFFFFFu ? 0u : v.x + v.y;
        }
    };
    // Once per item: every byte-table entry starts at (a, span) = (0, 0),
    // never empty, and only entries with an interval (about a fifth of the
    // buckets of a dense layer) are ranked per tile.  Event items rank each
    // such interval once against all rows, g(x) = #{F < x} over the layer's
    // sorted offsets of every row, so that a tile's a = #{F in tile, F < lo}
    // is cnt[g(lo)] (the tile's share of the first g values; equal values
    // never straddle g) and b = cnt[g(hi + 1)]; tile items list the
    // entries and search each tile's own sorted offsets.
    if (BOUNDS) {
        __syncthreads();                                 // every hit's bounds update done
        uint32_t lo_r[EPT], hi_r[EPT];
#pragma unroll
        for (uint32_t k = 0; k < EPT; ++k) {
            const uint32_t i = t + k * kRankThreads;
            lo_r[k] = 1;
            hi_r[k] = 0;
            if (i < N) interval(i, lo_r[k], hi_r[k]);
        }
        __syncthreads();                                 // every bound read before any is overwritten
        {
            const uint4 *src4 = reinterpret_cast<const uint4 *>(rk_glob);   // gstride: a multiple of 4
            for (uint32_t i = t; i < L * gstride / 4; i += nt) lds4[i] = src4[i];
        }
        __syncthreads();
        uint32_t g_r[EPT];
#pragma unroll
        for (uint32_t k = 0; k < EPT; ++k) {
            const uint32_t i = t + k * kRankThreads;
            g_r[k] = 0;
            if (i < N && lo_r[k] <= hi_r[k]) {
                has_bits |= 1u << k;
                const uint32_t *gl = lds + (i >> log2phi) * gstride;
                g_r[k] = rank_all(gl, lo_r[k]) | (rank_all(gl, hi_r[k] + 1u) << 16);
            }
        }
        __syncthreads();                                 // the sorted offsets are no longer read
#pragma unroll
        for (uint32_t k = 0; k < EPT; ++k)
            if (has_bits & (1u << k)) p_g[t + k * kRankThreads] = g_r[k];
        for (uint32_t i = t; i < L * (ngrp + 1) * 2; i += nt) bytes[i] = 0u;
        __syncthreads();
    } else {
    if (t == 0) n_ivl = 0;
    for (uint32_t i = t; i < L * (ngrp + 1) * 2; i += nt) bytes[i] = 0u;
    __syncthreads();
    // eight entries per thread per step, their bounds read before any is
    // used (one memory wait per step when they come from the table)
    constexpr uint32_t UI = 8;
    for (uint32_t i0 = 0; i0 < L * nphi; i0 += UI * nt) {
        bool has[UI];
#pragma unroll
        for (uint32_t u = 0; u < UI; ++u) {
            const uint32_t i = i0 + u * nt + t;
            uint32_t lo = 1, hi = 0;
            if (i < L * nphi) interval(i, lo, hi);
            has[u] = lo <= hi;
        }
#pragma unroll
        for (uint32_t u = 0; u < UI; ++u) {
            if (i0 + u * nt >= L * nphi) break;
            const uint32_t i = i0 + u * nt + t;
            const uint64_t bal = __ballot(has[u]);
            uint32_t base = 0;
            if (lane == 0 && bal) base = atomicAdd(&n_ivl, uint32_t(__popcll(bal)));
            base = __shfl(base, 0, 64);
            if (has[u]) ivl[base + __popcll(bal & ((1ull << lane) - 1ull))] = uint16_t(i);
        }
    }
    }

    uint16_t *eacc = acc + uint64_t(e) * rows * nphi;
    // a tile's sorted offsets (event items: its counts) are loaded into
    // registers one tile ahead (the loads are in flight while the previous
    // tile is ranked and voted) and stored to LDS when that tile is done
    constexpr uint32_t kSrtRegs =
        BOUNDS ? (LMAX * (kRankEventRowsMax / 4 + 1) + kRankThreads - 1) / kRankThreads
               : (16 * kRankSortStride + kRankThreads - 1) / kRankThreads;
    const uint32_t n_srt = L * (BOUNDS ? cstride : kRankSortStride);
    uint32_t sp[kSrtRegs];
    auto srt_load = [&](uint32_t tl) {
        const uint32_t *gs = (BOUNDS ? rk_cnt : rk_sorted) + size_t(tl) * n_srt;
#pragma unroll
        for (uint32_t k = 0; k < kSrtRegs; ++k) {
            const uint32_t i = t + k * kRankThreads;
            sp[k] = i < n_srt ? gs[i] : 0u;
        }
    };
    if (tile_lo < tile_hi) srt_load(tile_lo);
    for (uint32_t tile = tile_lo; tile < tile_hi; ++tile) {
        // previous tile's rows are done with the byte tables; the list is complete
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < kSrtRegs; ++k) {
            const uint32_t i = t + k * kRankThreads;
            if (i < n_srt) srt[i] = sp[k];
        }
        __syncthreads();
        if (tile + 1 < tile_hi) srt_load(tile + 1);
        // (a, span) bytes of the entries with an interval for this tile
        auto put_entry = [&](uint32_t i, uint32_t a, uint32_t sp) {
            const uint32_t l = i >> log2phi, j = i & (nphi - 1);
            uint8_t *bl = reinterpret_cast<uint8_t *>(bytes + l * (ngrp + 1) * 2);
            const uint32_t g = j >> 2, k = j & 3;
            bl[g * 8 + k] = uint8_t(a);
            bl[g * 8 + 4 + k] = uint8_t(sp);
            if (g == 0) {                                   // wrap group: buckets n_phi .. n_phi + 3
                bl[ngrp * 8 + k] = uint8_t(a);
                bl[ngrp * 8 + 4 + k] = uint8_t(sp);
            }
        };
        if (BOUNDS) {
            // each lane walks its own entries with an interval (the wave
            // takes as many steps as its busiest lane has entries)
            for (uint32_t bits = has_bits; bits; bits &= bits - 1u) {
                const uint32_t i = t + uint32_t(__builtin_ctz(bits)) * kRankThreads;
                const uint32_t g = p_g[i];
                const uint8_t *cn = reinterpret_cast<const uint8_t *>(srt + (i >> log2phi) * cstride);
                const uint32_t a = cn[g & 0xFFFFu];
                put_entry(i, a, uint32_t(cn[g >> 16]) - a);
            }
        } else {
            const uint32_t nl_ivl = n_ivl;
            for (uint32_t q = t; q < nl_ivl; q += nt) {
                const uint32_t i = ivl[q];
                uint32_t lo, hi;
                interval(i, lo, hi);
                const uint32_t *sl = srt + (i >> log2phi) * kRankSortStride;
                const uint32_t a = rank_below(sl, lo);
                put_entry(i, a, rank_below(sl, hi + 1u) - a);
            }
        }
        __syncthreads();

        const uint32_t r0 = tile * kRankTileRows;
        const uint32_t tr = min(kRankTileRows, rows - r0);
        const uint32_t rpw = (tr + nwaves - 1) / nwaves;
        const uint32_t rb = r0 + wave * rpw, re = min(r0 + tr, rb + rpw);
        uint32_t jc[LMAX];
        uint32_t ca[LMAX][G], cs[LMAX][G];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            jc[l] = 0xFFFFFFFFu;
#pragma unroll
            for (int g = 0; g < G; ++g) ca[l][g] = cs[l][g] = 0;
        }
        // the row's words: J (| unreachable << 31) per layer, then R =
        // (0x80 + rank) in every byte per layer; the next row's are loaded
        // while this one is computed
        uint32_t jn[LMAX], rn[LMAX];
        if (rb < re) {
            const uint32_t *info = rk_info + size_t(rb) * 32;
#pragma unroll
            for (int l = 0; l < LMAX; ++l) {
                jn[l] = info[l];
                rn[l] = info[16 + l];
            }
        }
        for (uint32_t r = rb; r < re; ++r) {
            uint32_t jw[LMAX], rw[LMAX];
#pragma unroll
            for (int l = 0; l < LMAX; ++l) {
                jw[l] = jn[l];
                rw[l] = rn[l];
            }
            if (r + 1 < re) {
                const uint32_t *info = rk_info + size_t(r + 1) * 32;
#pragma unroll
                for (int l = 0; l < LMAX; ++l) {
                    jn[l] = info[l];
                    rn[l] = info[16 + l];
                }
            }
            uint32_t m1[G], m2[G];                 // layers 0..7, 8..15: bit l of each byte
#pragma unroll
            for (int g = 0; g < G; ++g) m1[g] = m2[g] = 0;
#pragma unroll
            for (int l = 0; l < LMAX; ++l) {
                if (NL > 0 || uint32_t(l) < L) {
                    const uint32_t w = jw[l];
                    if (ALLV || !(w & kRankInvalid)) {
                        const uint32_t J = w & 0xFFFFu;
                        if (J != jc[l]) {
                            jc[l] = J;
                            const uint2 *bg = reinterpret_cast<const uint2 *>(bytes + l * (ngrp + 1) * 2);
                            const uint32_t sh = J & 3u;
#pragma unroll
                            for (int g = 0; g < G; ++g) {
                                const uint32_t kk = ((J >> 2) + 64u * g + lane) & (ngrp - 1);
                                const uint2 q0 = bg[kk], q1 = bg[kk + 1];
                                ca[l][g] = __builtin_amdgcn_alignbyte(q1.x, q0.x, sh);
                                cs[l][g] = __builtin_amdgcn_alignbyte(q1.y, q0.y, sh);
                            }
                        }
                        const uint32_t kBit = 0x01010101u << (l & 7);       // l is unrolled: a constant
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            const uint32_t x = rw[l] - ca[l][g];
                            const uint32_t y = x - cs[l][g];
                            const uint32_t occ = (~x | y) >> (7 - (l & 7));   // occupied: bit l & 7
                            if (l < 8) m1[g] = (occ & kBit) | (m1[g] & ~kBit);
                            else m2[g] = (occ & kBit) | (m2[g] & ~kBit);
                        }
                    }
                }
            }
            uint16_t *dst = eacc + size_t(r) * nphi;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                uint2 out;
                out.x = __builtin_amdgcn_perm(m2[g], m1[g], 0x05010400u);
                out.y = __builtin_amdgcn_perm(m2[g], m1[g], 0x07030602u);
                // written once and read back by the peak search long after:
                // a non-temporal store (c4 vote 0.73 -> 0.72 ms)
                __builtin_nontemporal_store(uint64_t(out.x) | (uint64_t(out.y) << 32),
                                            reinterpret_cast<uint64_t *>(dst + 256u * g + 4u * lane));
            }
        }
    }
}

namespace {

template <int G, int NL, bool ALLV>
void launch_rank_g(hough_ctx *c, bool bounds, const hough_hits *h, int vec, uint32_t n_tiles, uint32_t run,
                   uint32_t runs, uint32_t n_items, size_t lds, uint16_t *acc, hipStream_t s)
{
    const hough_grid_spec &g = c->spec;
    const RankGlobLayout y = rank_glob_layout(c->rows, g.n_layers);
    const uint32_t *glob = c->d_rk_sorted + y.glob_at, *cnt = c->d_rk_sorted + y.cnt_at;
    if (bounds)
        hipLaunchKernelGGL((k_vote_rank<G, NL, ALLV, true>), dim3(n_items), dim3(kRankThreads), lds, s, h->layer,
                           h->phi, h->event_offsets, h->n_hits, vec, c->d_dir_tab, c->d_rk_info, c->d_rk_sorted,
                           glob, cnt, y.gstride, y.cstride, g.n_layers, c->rows, g.n_phi, c->log2_phi, c->shift, n_tiles, run, runs, acc);
    else
        hipLaunchKernelGGL((k_vote_rank<G, NL, ALLV, false>), dim3(n_items), dim3(kRankThreads), lds, s, h->layer,
                           h->phi, h->event_offsets, h->n_hits, vec, c->d_dir_tab, c->d_rk_info, c->d_rk_sorted,
                           glob, cnt, y.gstride, y.cstride, g.n_layers, c->rows, g.n_phi, c->log2_phi, c->shift, n_tiles, run, runs, acc);
}

template <int G>
void launch_rank(hough_ctx *c, bool bounds, const hough_hits *h, int vec, uint32_t n_tiles, uint32_t run,
                 uint32_t runs, uint32_t n_items, size_t lds, uint16_t *acc, hipStream_t s)
{
    // the ten-layer detector of every workload here gets exact-count
    // instances; other layer counts the general one
    if (c->spec.n_layers == 10 && c->all_valid)
        launch_rank_g<G, 10, true>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s);
    else if (c->spec.n_layers == 10)
        launch_rank_g<G, 10, false>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s);
    else
        launch_rank_g<G, 0, false>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s);
}

size_t rank_lds_bytes(const hough_ctx *c, bool bounds)
{
    const size_t L = c->spec.n_layers, nphi = c->spec.n_phi, N = L * nphi;
    if (bounds) {
        // the bounds; all rows' sorted offsets; the ranks, byte tables and counts
        const RankGlobLayout y = rank_glob_layout(c->rows, uint32_t(L));
        return 4 * std::max({2 * N, L * y.gstride, N + L * (nphi / 4 + 1) * 2 + L * y.cstride});
    }
    return L * (nphi / 4 + 1) * 8 + L * kRankSortStride * 4 + ((N + 1) / 2) * 4 + 4;
}

}  // namespace

bool rank_vote_usable(const hough_ctx *c, const uint16_t *acc)
{
    return c->d_rk_info != nullptr && (reinterpret_cast<uintptr_t>(acc) & 7) == 0 &&
           rank_lds_bytes(c, false) <= c->max_lds_rank;
}

hipError_t launch_vote_rank(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s)
{
    const uint32_t E = h->n_events;
    const uint32_t n_tiles = (c->rows + kRankTileRows - 1) / kRankTileRows;
    const int vec = (reinterpret_cast<uintptr_t>(h->layer) & 3) == 0 && (reinterpret_cast<uintptr_t>(h->phi) & 15) == 0;
    const uint64_t want = uint64_t(c->n_cu) * 2;
    // whole events per item (bounds found in the kernel) when there are
    // enough events to fill the device and the bounds fit in LDS; else one
    // tile per item with the bounds from k_vote_bounds' table
    const bool fits = c->rows <= kRankEventRowsMax && rank_lds_bytes(c, true) <= c->max_lds_rank;
    const bool bounds = c->tun.vote_items == 1 ? fits : c->tun.vote_items == 2 ? false : uint64_t(E) >= want && fits;
    hipError_t err;
    KernelTimer t;
    if (!bounds && (err = launch_vote_bounds(c, h, s)) != hipSuccess) return err;
    const uint32_t run = bounds ? n_tiles : 1;
    const uint32_t runs = (n_tiles + run - 1) / run;
    const uint32_t n_items = runs * E;
    const size_t lds = rank_lds_bytes(c, bounds);
    prof_begin(c, bounds ? "vote_rank_event" : "vote_rank_tile", s, &t);
    switch (c->spec.n_phi) {
    case 256: launch_rank<1>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s); break;
    case 512: launch_rank<2>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s); break;
    default: launch_rank<4>(c, bounds, h, vec, n_tiles, run, runs, n_items, lds, acc, s); break;
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
