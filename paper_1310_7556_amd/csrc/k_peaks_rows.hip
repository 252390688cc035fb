// Step 2 of the transform (Section 4, second step) in a row-window form for
// grids whose n_phi is 64 times C, C = 4, 8 or 16.  The rule is k_peaks': a
// cell is a peak iff its popcount is >= the threshold and >= the popcount
// of each neighbour in its 3x3 (q/pT, phi0) window, 3x3x3 with a d0 axis,
// phi0 periodic, q/pT and d0 not (rows and planes outside the grid count
// as 0).
//
// A wavefront owns a strip of R consecutive q/pT rows of one event (and one
// d0 plane) and walks it one row at a time, with one halo row above and one
// below (and the same rows of the planes on either side); nothing is
// staged in LDS.  Lane i holds cells C*i .. C*i + C - 1 of the row, their
// popcounts packed as 16-bit pairs.  A row is exactly the wave's 64 * C
// cells, so the neighbours of a lane's first and last cell come from the
// lanes beside it by a wave-wide rotate, which also closes the periodic phi0
// axis.  Per row and pair the lane forms
//     lr = max(left, right, threshold),   h = max(lr, self)
// and a cell of the centre row is a peak iff its popcount is >= max(h of
// the row above, h of the row below, its own lr): the threshold is folded
// into every maximum, and the test is the sign bit of a packed 16-bit
// difference.  Rows are prefetched a few ahead, so a strip waits for
// memory about once.
//
// The count pass writes one count per strip.  The write pass compacts each
// row's peaks in cell order: a wave prefix of the lanes' counts (one ballot
// per count bit), the records written to a per-wave LDS buffer at their
// positions, then stored contiguously from it, 8 bytes per lane.
#include "hough_internal.h"

namespace hough {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pmax(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

// a - b per 16-bit half, wrapping: bit 15 of a half is set iff b > a there
// (both at most 17)
__device__ __forceinline__ uint32_t psub(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}

__device__ __forceinline__ uint32_t popc_pair(uint32_t w)
{
    return uint32_t(__popc(w & 0xFFFFu)) | (uint32_t(__popc(w >> 16)) << 16);
}

// lane i receives lane i - 1's value, lane 0 lane 63's (a wave-wide rotate
// right by one lane)
__device__ __forceinline__ uint32_t from_left(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0x13C, 0xF, 0xF, false));
}

// lane i receives lane i + 1's value, lane 63 lane 0's (rotate left)
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0x134, 0xF, 0xF, false));
}

// the lane's C cells of row r (r clamped into the grid; the caller zeroes
// rows outside it)
template <int C>
__device__ __forceinline__ void load_row(const uint16_t *__restrict__ ev, int r, uint32_t n_qpt, uint32_t lane,
                                         uint32_t (&w)[C / 2])
{
    const uint32_t rr = uint32_t(min(max(r, 0), int(n_qpt) - 1));
    const uint16_t *p = ev + size_t(rr) * (64u * C) + size_t(lane) * C;
    if constexpr (C == 4) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        w[0] = v.x;
        w[1] = v.y;
    } else {
#pragma unroll
        for (int g = 0; g < C / 8; ++g) {
            const uint4 v = reinterpret_cast<const uint4 *>(p)[g];
            w[4 * g] = v.x;
            w[4 * g + 1] = v.y;
            w[4 * g + 2] = v.z;
            w[4 * g + 3] = v.w;
        }
    }
}

// popcount pairs, lr and h of one row (see the header)
template <int C>
__device__ __forceinline__ void row_maxima(const uint32_t (&raw)[C / 2], uint32_t t2, uint32_t (&pc)[C / 2],
                                           uint32_t (&lr)[C / 2], uint32_t (&h)[C / 2])
{
    constexpr int D = C / 2;
#pragma unroll
    for (int d = 0; d < D; ++d) pc[d] = popc_pair(raw[d]);
    const uint32_t lft = from_left(pc[D - 1]);     // high half: the cell before the lane's first
    const uint32_t rgt = from_right(pc[0]);        // low half: the cell after the lane's last
    // s[d] = (cell 2d - 1, cell 2d): the left neighbours of pair d and the
    // right neighbours of pair d - 1
    uint32_t s[D + 1];
    s[0] = __builtin_amdgcn_alignbit(pc[0], lft, 16);
#pragma unroll
    for (int d = 1; d < D; ++d) s[d] = __builtin_amdgcn_alignbit(pc[d], pc[d - 1], 16);
    s[D] = __builtin_amdgcn_alignbit(rgt, pc[D - 1], 16);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lr[d] = pmax(pmax(s[d], s[d + 1]), t2);
        h[d] = pmax(lr[d], pc[d]);
    }
}

// D3: grids with a d0 axis (n_d0 > 1); a strip lies in one d0 plane, and
// the matching rows of the planes before and after it enter only through
// nb(r) = max(h of plane d - 1, h of plane d + 1) at row r (a missing plane
// counts as zeros, whose h is the threshold, as for rows outside the grid).
template <int C, bool WRITE, bool D3>
__global__ void __launch_bounds__(kPeakThreads)
k_peaks_rows(const uint16_t *__restrict__ acc, uint32_t n_qpt, uint32_t n_d0, uint32_t R, uint32_t n_strips,
             uint64_t n_tiles, uint32_t thr, uint32_t *__restrict__ tile_counts,
             const uint64_t *__restrict__ tile_off, hough_peak *__restrict__ peaks, uint64_t capacity)
{
    constexpr int D = C / 2;
    constexpr int PF = D3 ? 2 : (D <= 4 ? 4 : 2);  // rows in flight (per plane)
    HOUGH_DYNAMIC_LDS(uint2, lds);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t tile = uint64_t(blockIdx.x) * (kPeakThreads / 64) + wave;
    if (tile >= n_tiles) return;                   // no workgroup barrier below
    // tiles in (event, d0 plane, strip) order: the order of the records
    const uint32_t planes = D3 ? n_d0 : 1u;
    const uint32_t e = uint32_t(tile / (uint64_t(planes) * n_strips));
    const uint32_t rem = uint32_t(tile % (uint64_t(planes) * n_strips));
    const uint32_t dp = rem / n_strips, st = rem % n_strips;
    const int r0 = int(st * R), r1 = int(min(st * R + R, n_qpt));
    const uint64_t plane = uint64_t(n_qpt) * (64u * C);
    const uint16_t *ev = acc + (uint64_t(e) * planes + dp) * plane;
    const bool has_m = D3 && dp > 0, has_p = D3 && dp + 1 < planes;
    const uint16_t *evm = has_m ? ev - plane : ev, *evp = has_p ? ev + plane : ev;
    const uint32_t t2 = min(thr, 17u) * 0x00010001u;   // popcounts are <= 16

    // halo rows and the first PF strip rows, all in flight together
    uint32_t top[D], bot[D], buf[PF][D];
    uint32_t topm[D], topp[D], botm[D], botp[D], bufm[PF][D], bufp[PF][D];
    load_row<C>(ev, r0 - 1, n_qpt, lane, top);
    load_row<C>(ev, r1, n_qpt, lane, bot);
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (r0 + i < r1) load_row<C>(ev, r0 + i, n_qpt, lane, buf[i]);
    // a neighbour plane's row (zeros where the plane or the row is missing)
    auto load_nb = [&](bool has, const uint16_t *pv, int r, uint32_t (&w)[D]) {
        if (has && r >= 0 && r < int(n_qpt)) {
            load_row<C>(pv, r, n_qpt, lane, w);
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) w[d] = 0u;
        }
    };
    if (D3) {
        load_nb(has_m, evm, r0 - 1, topm);
        load_nb(has_p, evp, r0 - 1, topp);
        load_nb(has_m, evm, r1, botm);
        load_nb(has_p, evp, r1, botp);
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            load_nb(has_m, evm, r0 + i < r1 ? r0 + i : -1, bufm[i]);
            load_nb(has_p, evp, r0 + i < r1 ? r0 + i : -1, bufp[i]);
        }
    }
    // nb of one row from the two neighbour planes' raw cells
    auto nb_of = [&](const uint32_t (&rm)[D], const uint32_t (&rp)[D], uint32_t (&nb)[D]) {
        uint32_t pcx[D], lrx[D], hm[D], hq[D];
        row_maxima<C>(rm, t2, pcx, lrx, hm);
        row_maxima<C>(rp, t2, pcx, lrx, hq);
#pragma unroll
        for (int d = 0; d < D; ++d) nb[d] = pmax(hm[d], hq[d]);
    };

    // the window: h of the row above the centre row, and the centre row's
    // popcounts, lr, h (and raw cells when writing)
    uint32_t hp[D], pcc[D], lrc[D], hc[D], rawc[D];
    uint32_t nbp[D], nbc[D];                       // D3: nb of the rows above and at the centre
    {
        uint32_t raw[D];
#pragma unroll
        for (int d = 0; d < D; ++d) raw[d] = r0 > 0 ? top[d] : 0u;
        row_maxima<C>(raw, t2, pcc, lrc, hc);
#pragma unroll
        for (int d = 0; d < D; ++d) rawc[d] = raw[d];
        if (D3) nb_of(topm, topp, nbc);
    }
    uint32_t nonpeak = 0;                          // centre cells that failed, summed over rows
    uint64_t running = WRITE ? tile_off[tile] : 0;
    uint2 *rec = lds + size_t(wave) * (64u * C);
    const uint32_t cell_row0 = lane * C;

    // with the next row's h known, the centre row (q - 1) is decided
    auto decide = [&](int q, const uint32_t (&hn)[D], const uint32_t (&nbn)[D]) {
        uint32_t neg[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            uint32_t mx = pmax(pmax(hp[d], hn[d]), lrc[d]);
            if (D3) mx = pmax(mx, pmax(pmax(nbp[d], nbc[d]), nbn[d]));
            neg[d] = psub(pcc[d], mx) & 0x80008000u;
        }
        if (!WRITE) {
#pragma unroll
            for (int d = 0; d < D; ++d) nonpeak += __popc(neg[d]);
            return;
        }
        uint32_t bits = 0;                         // bit j: cell j of the lane is a peak
#pragma unroll
        for (int d = 0; d < D; ++d)
            bits |= (((neg[d] >> 15) & 1u) | ((neg[d] >> 30) & 2u)) << (2 * d);
        bits ^= (1u << C) - 1u;
        const uint32_t cnt = __popc(bits);
        const uint64_t lt = (1ull << lane) - 1ull;
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int b = 0; (1 << b) <= C; ++b) {
            const uint64_t m = __ballot((cnt >> b) & 1u);
            before += uint32_t(__popcll(m & lt)) << b;
            total += uint32_t(__popcll(m)) << b;
        }
        const uint32_t cell0 = (dp * n_qpt + uint32_t(q - 1)) * (64u * C) + cell_row0;
        uint32_t o = before;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            if ((bits >> j) & 1u) {
                const uint32_t m = (rawc[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                const uint32_t p = (pcc[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                rec[o++] = make_uint2(cell0 + j, m | (p << 16));
            }
        }
        // the wave's records are in LDS before any lane reads them back
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint2 *out = reinterpret_cast<uint2 *>(peaks);
        for (uint32_t i = lane; i < total; i += 64) {
            const uint64_t pos = running + i;
            if (pos < capacity) out[pos] = rec[i];
        }
        running += total;
        // and read back before the next row overwrites them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto advance = [&](const uint32_t (&raw)[D], const uint32_t (&nbn)[D], int q) {
        uint32_t pcn[D], lrn[D], hn[D];
        row_maxima<C>(raw, t2, pcn, lrn, hn);
        decide(q, hn, nbn);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            hp[d] = hc[d];
            hc[d] = hn[d];
            pcc[d] = pcn[d];
            lrc[d] = lrn[d];
            rawc[d] = raw[d];
            if (D3) {
                nbp[d] = nbc[d];
                nbc[d] = nbn[d];
            }
        }
    };

    // rows r0 + 1 .. r1 - 1 each decide the row above them; row r0 is the
    // first centre row and needs no decision of its own row above
    for (int q0 = r0; q0 < r1; q0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int q = q0 + i;
            if (q >= r1) break;
            uint32_t raw[D], nbn[D];
#pragma unroll
            for (int d = 0; d < D; ++d) raw[d] = buf[i][d];
            if (D3) nb_of(bufm[i], bufp[i], nbn);
            if (q + PF < r1) {
                load_row<C>(ev, q + PF, n_qpt, lane, buf[i]);
                if (D3) {
                    load_nb(has_m, evm, q + PF, bufm[i]);
                    load_nb(has_p, evp, q + PF, bufp[i]);
                }
            }
            if (q == r0) {
                uint32_t pcn[D], lrn[D], hn[D];
                row_maxima<C>(raw, t2, pcn, lrn, hn);
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    hp[d] = hc[d];
                    hc[d] = hn[d];
                    pcc[d] = pcn[d];
                    lrc[d] = lrn[d];
                    rawc[d] = raw[d];
                    if (D3) {
                        nbp[d] = nbc[d];
                        nbc[d] = nbn[d];
                    }
                }
            } else {
                advance(raw, nbn, q);
            }
        }
    }
    {
        // the bottom halo row decides the strip's last row
        uint32_t raw[D], nbn[D];
#pragma unroll
        for (int d = 0; d < D; ++d) raw[d] = r1 < int(n_qpt) ? bot[d] : 0u;
        if (D3) nb_of(botm, botp, nbn);
        advance(raw, nbn, r1);
    }
    if (!WRITE) {
        uint32_t cnt = uint32_t(C) * uint32_t(r1 - r0) - nonpeak;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if (lane == 0) tile_counts[tile] = cnt;
    }
}

template <int C, bool D3>
void launch_rows_d(bool write, uint32_t blocks, size_t lds, hipStream_t s, const uint16_t *acc, uint32_t n_qpt,
                   uint32_t n_d0, uint32_t R, uint32_t n_strips, uint64_t n_tiles, uint32_t thr,
                   uint32_t *tile_counts, const uint64_t *tile_off, hough_peak *peaks, uint64_t capacity)
{
    if (write)
        hipLaunchKernelGGL((k_peaks_rows<C, true, D3>), dim3(blocks), dim3(kPeakThreads), lds, s, acc, n_qpt, n_d0,
                           R, n_strips, n_tiles, thr, tile_counts, tile_off, peaks, capacity);
    else
        hipLaunchKernelGGL((k_peaks_rows<C, false, D3>), dim3(blocks), dim3(kPeakThreads), 0, s, acc, n_qpt, n_d0,
                           R, n_strips, n_tiles, thr, tile_counts, tile_off, peaks, capacity);
}

template <int C>
void launch_rows(bool write, uint32_t blocks, size_t lds, hipStream_t s, const uint16_t *acc, uint32_t n_qpt,
                 uint32_t n_d0, uint32_t R, uint32_t n_strips, uint64_t n_tiles, uint32_t thr, uint32_t *tile_counts,
                 const uint64_t *tile_off, hough_peak *peaks, uint64_t capacity)
{
    if (n_d0 > 1)
        launch_rows_d<C, true>(write, blocks, lds, s, acc, n_qpt, n_d0, R, n_strips, n_tiles, thr, tile_counts,
                               tile_off, peaks, capacity);
    else
        launch_rows_d<C, false>(write, blocks, lds, s, acc, n_qpt, 1, R, n_strips, n_tiles, thr, tile_counts,
                                tile_off, peaks, capacity);
}

}  // namespace

uint32_t peak_rows_strip(const hough_ctx *c)
{
    return std::min(c->tun.peak_rows ? c->tun.peak_rows : 16u, c->spec.n_qpt);
}

uint32_t peak_rows_cells_per_lane(const hough_ctx *c, const uint16_t *acc, uint32_t n_events)
{
    if (c->tun.peak_algo == 1) return 0;
    const uint32_t C = c->spec.n_phi / 64;
    if (c->spec.n_phi % 64 != 0 || (C != 4 && C != 8 && C != 16)) return 0;
    const uintptr_t align = C == 4 ? 8 : 16;
    if (reinterpret_cast<uintptr_t>(acc) % align != 0) return 0;
    if (size_t(kPeakThreads / 64) * 64 * C * 8 > c->max_lds) return 0;
    // by default only when the strips (one wave each) fill the chip about
    // twice: a single event has few strips, and the tile form's many small
    // workgroups then finish sooner
    if (c->tun.peak_algo == 0) {
        const uint32_t R = peak_rows_strip(c);
        const uint64_t strips = uint64_t(n_events) * c->spec.n_d0 * ((c->spec.n_qpt + R - 1) / R);
        if (strips < uint64_t(c->n_cu) * 8) return 0;
    }
    return C;
}

hipError_t launch_peaks_rows_pass(hough_ctx *c, bool write, const uint16_t *acc, uint32_t n_events,
                                  hough_peak *peaks, uint64_t capacity, const PeakScratch &ps, hipStream_t s)
{
    const uint32_t C = peak_rows_cells_per_lane(c, acc, n_events);
    const uint32_t R = peak_rows_strip(c);
    const uint32_t n_strips = (c->spec.n_qpt + R - 1) / R;
    const uint64_t n_tiles = uint64_t(n_events) * c->spec.n_d0 * n_strips;
    const uint64_t blocks = (n_tiles + kPeakThreads / 64 - 1) / (kPeakThreads / 64);
    if (blocks > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    const size_t lds = size_t(kPeakThreads / 64) * 64 * C * 8;
    const uint32_t thr = c->spec.threshold;
    if (C == 4)
        launch_rows<4>(write, uint32_t(blocks), lds, s, acc, c->spec.n_qpt, c->spec.n_d0, R, n_strips, n_tiles, thr,
                       ps.tile_counts, ps.tile_off, peaks, capacity);
    else if (C == 8)
        launch_rows<8>(write, uint32_t(blocks), lds, s, acc, c->spec.n_qpt, c->spec.n_d0, R, n_strips, n_tiles, thr,
                       ps.tile_counts, ps.tile_off, peaks, capacity);
    else if (C == 16)
        launch_rows<16>(write, uint32_t(blocks), lds, s, acc, c->spec.n_qpt, c->spec.n_d0, R, n_strips, n_tiles, thr,
                        ps.tile_counts, ps.tile_off, peaks, capacity);
    else
        return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

}  // namespace hough
