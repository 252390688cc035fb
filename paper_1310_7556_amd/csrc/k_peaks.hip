// Step 2 of the transform: local maxima of the accumulator (Section 4, second
// step; Section 8 notes this search is regular in memory but reduction-heavy).
//
// A cell is a peak iff popcount >= threshold and >= the popcount of each
// neighbour in its 3x3 (q/pT, phi0) window, 3x3x3 with a d0 axis; phi0 is
// periodic, q/pT and d0 are not.  Tile = (event, d0 plane, RP rows of q/pT).
// The tile plus a one-row halo (and the adjacent d0 planes in 3D) is staged
// in LDS as popcount bytes.  Compaction keeps cell order: a count pass, one
// exclusive scan over tiles in (event, d0, row) order, and a write pass that
// places each 64-wide wavefront's peaks with ballot + mbcnt prefixes and
// each workgroup's waves with an LDS prefix.
#include <mutex>

#include "hough_internal.h"

// Scratch of hough_peaks_noalloc, for callers that cannot allocate device
// memory: one file-scope array, of which each GPU holds its own copy until
// the process ends.  In host code its name is only a stand-in for the
// device symbol; its address on a device comes from hipGetSymbolAddress,
// looked up once per device (noalloc_scratch_init) and then used for every
// kernel argument.  Concurrent noalloc calls on one GPU share it and race.
static __device__ __align__(256) unsigned char scratch[size_t(8) << 20];

namespace hough {

const size_t kNoAllocScratchBytes = size_t(8) << 20;

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = p;
    return e;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

size_t peak_scratch_bytes(uint64_t n_tiles)
{
    const uint64_t nb = scan_blocks(n_tiles);
    return align256(4 * n_tiles) + align256(8 * (n_tiles + 1)) + align256(8 * nb) + align256(8 * (nb + 1));
}

PeakScratch carve_peak_scratch(void *base, uint64_t n_tiles)
{
    const uint64_t nb = scan_blocks(n_tiles);
    char *p = static_cast<char *>(base);
    PeakScratch ps;
    ps.tile_counts = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * n_tiles);
    ps.tile_off = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * (n_tiles + 1));
    ps.scan_part = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * nb);
    ps.scan_off = reinterpret_cast<uint64_t *>(p);
    ps.scan_blocks_max = nb;
    return ps;
}

template <bool WRITE>
__global__ void __launch_bounds__(256)
k_peaks(const uint16_t *__restrict__ acc, uint32_t n_d0, uint32_t n_qpt, uint32_t nphi,
        uint32_t log2phi, uint32_t rp, uint32_t n_kt, uint32_t thr, uint32_t *__restrict__ tile_counts,
        const uint64_t *__restrict__ tile_off, hough_peak *__restrict__ peaks, uint64_t capacity)
{
    HOUGH_DYNAMIC_LDS(uint8_t, pc);
    __shared__ uint32_t wave_cnt[4];
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t item = blockIdx.x;
    const uint32_t per_event = n_d0 * n_kt;
    const uint32_t e = item / per_event;
    const uint32_t d = (item % per_event) / n_kt;
    const uint32_t k0 = (item % n_kt) * rp;
    const uint32_t nr = min(rp, n_qpt - k0);
    const uint32_t planes = n_d0 > 1 ? 3 : 1;
    const uint32_t prow = nr + 2;                       // rows staged per plane
    const uint64_t cells = uint64_t(n_d0) * n_qpt * nphi;
    const uint16_t *ev = acc + uint64_t(e) * cells;

    // stage popcounts of planes d-1..d+1 (or d), rows k0-1 .. k0+nr; absent -> 0
    const uint32_t staged = planes * prow * nphi;
    for (uint32_t i = t; i < staged; i += nt) {
        const uint32_t p = i & (nphi - 1);
        const uint32_t rr = (i >> log2phi) % prow;
        const uint32_t pl = (i >> log2phi) / prow;
        const int dd = planes == 3 ? int(d) + int(pl) - 1 : int(d);
        const int kk = int(k0) + int(rr) - 1;
        uint8_t v = 0;
        if (dd >= 0 && dd < int(n_d0) && kk >= 0 && kk < int(n_qpt))
            v = uint8_t(__popc(ev[(uint64_t(dd) * n_qpt + kk) * nphi + p]));
        pc[i] = v;
    }
    __syncthreads();

    const uint32_t cp = planes == 3 ? 1 : 0;           // centre plane in LDS
    const uint32_t ncell = nr * nphi;
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    uint32_t count = 0;
    uint64_t running = WRITE ? tile_off[item] : 0;
    for (uint32_t base = 0; base < ncell; base += nt) {
        const uint32_t cidx = base + t;
        bool is_peak = false;
        uint32_t rr = 0, p = 0;
        if (cidx < ncell) {
            rr = cidx >> log2phi;
            p = cidx & (nphi - 1);
            const uint32_t pm = (p - 1) & (nphi - 1), pp = (p + 1) & (nphi - 1);
            const uint8_t *c0 = pc + (cp * prow + rr + 1) * nphi;
            const uint32_t v = c0[p];
            if (v >= thr) {
                bool ok = true;
                for (uint32_t pl = 0; pl < planes && ok; ++pl) {
                    for (uint32_t dr = 0; dr < 3; ++dr) {
                        const uint8_t *row = pc + (pl * prow + rr + dr) * nphi;
                        const bool centre_row = pl == cp && dr == 1;
                        ok &= row[pm] <= v && row[pp] <= v && (centre_row || row[p] <= v);
                    }
                }
                is_peak = ok;
            }
        }
        if (!WRITE) {
            count += is_peak;
            continue;
        }
        const uint64_t bal = __ballot(is_peak);
        const uint32_t before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wave] = __popcll(bal);
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < nwaves; ++w) {
            const uint32_t x = wave_cnt[w];
            woff += w < wave ? x : 0;
            total += x;
        }
        if (is_peak) {
            const uint64_t pos = running + woff + before;
            if (pos < capacity) {
                const uint32_t cell = uint32_t((uint64_t(d) * n_qpt + k0 + rr) * nphi + p);
                const uint16_t m = ev[cell];
                uint2 rec;
                rec.x = cell;
                rec.y = uint32_t(m) | (uint32_t(__popc(m)) << 16);
                reinterpret_cast<uint2 *>(peaks)[pos] = rec;
            }
        }
        running += total;
        __syncthreads();
    }
    if (!WRITE) {
        // block sum of per-thread counts
        for (uint32_t off = 32; off > 0; off >>= 1) count += __shfl_down(count, off, 64);
        if (lane == 0) wave_cnt[wave] = count;
        __syncthreads();
        if (t == 0) {
            uint32_t s = 0;
            for (uint32_t w = 0; w < nwaves; ++w) s += wave_cnt[w];
            tile_counts[item] = s;
        }
    }
}

// Two 16-bit lanes per 32-bit word: max of each half.  On the GPU one
// packed-integer instruction (v_pk_max_u16); the expression in the other
// branch is the same arithmetic for host compilation.
__device__ __forceinline__ uint32_t pk_max_u16(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
#else
    return max(a & 0xFFFFu, b & 0xFFFFu) | (max(a >> 16, b >> 16) << 16);
#endif
}

// (hi:lo) >> 16: the pair of cells one position to the right of `lo`
__device__ __forceinline__ uint32_t shift_pair(uint32_t hi, uint32_t lo)
{
    return (lo >> 16) | (hi << 16);
}

__device__ __forceinline__ uint32_t popc2(uint32_t a)
{
    // popcounts of the two uint16 halves of a, one per half
    return uint32_t(__popc(a & 0xFFFFu)) | (uint32_t(__popc(a >> 16)) << 16);
}

// Vector form of k_peaks for n_phi >= 8 and a 16-byte aligned accumulator.
// Staging reads 8 cells per 16-byte load and keeps their popcounts as
// 16-bit pairs; each thread tests 4 consecutive cells, two per word, with
// packed 16-bit maxima of the shifted neighbour pairs; with WRITE, a
// chunk's peaks are compacted into LDS in cell order and stored with
// consecutive 8-byte writes.
template <bool WRITE>
__global__ void __launch_bounds__(256)
k_peaks_vec(const uint16_t *__restrict__ acc, uint32_t n_d0, uint32_t n_qpt, uint32_t nphi,
            uint32_t log2phi, uint32_t rp, uint32_t n_kt, uint32_t thr, uint32_t *__restrict__ tile_counts,
            const uint64_t *__restrict__ tile_off, hough_peak *__restrict__ peaks, uint64_t capacity)
{
    HOUGH_DYNAMIC_LDS(uint4, lds4);
    __shared__ uint32_t wave_cnt[4];
    const uint32_t t = threadIdx.x, nt = blockDim.x;    // nt == 256
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    const uint32_t item = blockIdx.x;
    const uint32_t per_event = n_d0 * n_kt;
    const uint32_t e = item / per_event;
    const uint32_t d = (item % per_event) / n_kt;
    const uint32_t k0 = (item % n_kt) * rp;
    const uint32_t nr = min(rp, n_qpt - k0);
    const uint32_t planes = n_d0 > 1 ? 3 : 1;
    const uint32_t prow = nr + 2;
    const uint64_t cells = uint64_t(n_d0) * n_qpt * nphi;
    const uint16_t *ev = acc + uint64_t(e) * cells;
    // LDS: popcounts [planes][prow][nphi] as uint16, then (WRITE) the raw
    // centre rows [nr][nphi] uint16 and the chunk's records [nt * 4] uint2
    uint16_t *pc = reinterpret_cast<uint16_t *>(lds4);
    const size_t pc_bytes = (size_t(planes) * prow * nphi * 2 + 15) & ~size_t(15);
    uint16_t *raw = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lds4) + pc_bytes);
    uint2 *rec = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(raw) + size_t(nr) * nphi * 2);

    const uint32_t vpr = nphi >> 3;                     // 8-cell vectors per row
    const uint32_t lv = log2phi - 3;
    const uint32_t nvec = planes * prow * vpr;
    const uint32_t cp = planes == 3 ? 1 : 0;
    // staging, four vectors per thread per step: all four loads are issued
    // before any is used, so a tile pays the memory latency once per step
    constexpr uint32_t kStageU = 4;
    for (uint32_t i0 = t; i0 < nvec; i0 += kStageU * nt) {
        uint4 v[kStageU];
        bool ok[kStageU];
#pragma unroll
        for (uint32_t u = 0; u < kStageU; ++u) {
            const uint32_t i = i0 + u * nt;
            const uint32_t ri = i >> lv, col = i & (vpr - 1);
            const uint32_t pl = planes == 1 ? 0 : (ri >= 2 * prow ? 2 : ri >= prow ? 1 : 0);
            const uint32_t rr = ri - pl * prow;
            const int dd = planes == 3 ? int(d) + int(pl) - 1 : int(d);
            const int kk = int(k0) + int(rr) - 1;
            ok[u] = i < nvec && dd >= 0 && dd < int(n_d0) && kk >= 0 && kk < int(n_qpt);
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            if (ok[u]) v[u] = *reinterpret_cast<const uint4 *>(ev + (uint64_t(dd) * n_qpt + kk) * nphi + col * 8);
        }
#pragma unroll
        for (uint32_t u = 0; u < kStageU; ++u) {
            const uint32_t i = i0 + u * nt;
            if (i >= nvec) break;
            const uint32_t ri = i >> lv, col = i & (vpr - 1);
            const uint32_t pl = planes == 1 ? 0 : (ri >= 2 * prow ? 2 : ri >= prow ? 1 : 0);
            const uint32_t rr = ri - pl * prow;
            uint4 packed = make_uint4(0u, 0u, 0u, 0u);
            if (ok[u]) {
                packed = make_uint4(popc2(v[u].x), popc2(v[u].y), popc2(v[u].z), popc2(v[u].w));
                if (WRITE && pl == cp && rr >= 1 && rr <= nr)
                    *reinterpret_cast<uint4 *>(raw + (rr - 1) * nphi + col * 8) = v[u];
            }
            *reinterpret_cast<uint4 *>(pc + size_t(ri) * nphi + col * 8) = packed;
        }
    }
    __syncthreads();

    const uint32_t t2 = min(thr, 17u) * 0x00010001u;    // popcounts are <= 16
    const uint32_t nquad = (nr * nphi) >> 2;
    uint32_t count = 0;
    uint64_t running = WRITE ? tile_off[item] : 0;
    for (uint32_t base = 0; base < nquad; base += nt) {
        const uint32_t q = base + t;
        uint32_t bits = 0;                              // peak flags of 4 cells
        if (q < nquad) {
            const uint32_t rr = (q << 2) >> log2phi;
            const uint32_t p0 = (q << 2) & (nphi - 1);
            const uint32_t pm = (p0 - 2) & (nphi - 1), pn = (p0 + 4) & (nphi - 1);
            const uint2 vv = *reinterpret_cast<const uint2 *>(pc + (cp * prow + rr + 1) * nphi + p0);
            uint32_t m0 = t2, m1 = t2;                  // neighbour maxima, threshold folded in
            for (uint32_t pl = 0; pl < planes; ++pl) {
#pragma unroll
                for (uint32_t dr = 0; dr < 3; ++dr) {
                    const uint16_t *row = pc + (pl * prow + rr + dr) * nphi;
                    const uint2 w = *reinterpret_cast<const uint2 *>(row + p0);       // cells p0..p0+3
                    const uint32_t wl = *reinterpret_cast<const uint32_t *>(row + pm);  // p0-2, p0-1
                    const uint32_t wr = *reinterpret_cast<const uint32_t *>(row + pn);  // p0+4, p0+5
                    const uint32_t mid = shift_pair(w.y, w.x);                          // p0+1, p0+2
                    m0 = pk_max_u16(m0, pk_max_u16(shift_pair(w.x, wl), mid));          // p0-1.. / p0+1..
                    m1 = pk_max_u16(m1, pk_max_u16(mid, shift_pair(wr, w.y)));
                    if (!(pl == cp && dr == 1)) {
                        m0 = pk_max_u16(m0, w.x);
                        m1 = pk_max_u16(m1, w.y);
                    }
                }
            }
            // a cell is a peak iff its popcount is >= every neighbour and >= thr:
            // max(m, v) == v in its half
            const uint32_t x0 = pk_max_u16(m0, vv.x) ^ vv.x, x1 = pk_max_u16(m1, vv.y) ^ vv.y;
            bits = ((x0 & 0xFFFFu) == 0 ? 1u : 0u) | ((x0 >> 16) == 0 ? 2u : 0u) |
                   ((x1 & 0xFFFFu) == 0 ? 4u : 0u) | ((x1 >> 16) == 0 ? 8u : 0u);
        }
        const uint32_t c = __popc(bits);
        if (!WRITE) {
            count += c;
            continue;
        }
        const uint64_t b0 = __ballot(c & 1u), b1 = __ballot(c & 2u), b2 = __ballot(c & 4u);
        const uint64_t lt = (1ull << lane) - 1ull;
        const uint32_t before = __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
        if (lane == 0) wave_cnt[wave] = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < nwaves; ++w) {
            const uint32_t x = wave_cnt[w];
            woff += w < wave ? x : 0;
            total += x;
        }
        if (bits) {
            const uint32_t rr = (q << 2) >> log2phi;
            const uint32_t p0 = (q << 2) & (nphi - 1);
            const uint32_t cell0 = uint32_t((uint64_t(d) * n_qpt + k0 + rr) * nphi + p0);
            uint32_t o = woff + before;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                if ((bits >> j) & 1u) {
                    const uint32_t mk = raw[rr * nphi + p0 + j];
                    rec[o++] = make_uint2(cell0 + j, mk | (uint32_t(__popc(mk)) << 16));
                }
            }
        }
        __syncthreads();
        uint2 *out = reinterpret_cast<uint2 *>(peaks);
        for (uint32_t i = t; i < total; i += nt) {
            const uint64_t pos = running + i;
            if (pos < capacity) out[pos] = rec[i];
        }
        running += total;
        __syncthreads();
    }
    if (!WRITE) {
        for (uint32_t off = 32; off > 0; off >>= 1) count += __shfl_down(count, off, 64);
        if (lane == 0) wave_cnt[wave] = count;
        __syncthreads();
        if (t == 0) {
            uint32_t s = 0;
            for (uint32_t w = 0; w < nwaves; ++w) s += wave_cnt[w];
            tile_counts[item] = s;
        }
    }
}

// Local maxima of the counting accumulator (the paper's A[B[i]] += 1 form):
// the rule of k_peaks with the uint32 vote count of a cell in place of its
// popcount.  Same tiles, halo and ordered compaction; the staged values are
// the counts themselves; records are {cell, count}.
template <bool WRITE>
__global__ void __launch_bounds__(256)
k_peaks_count(const uint32_t *__restrict__ cnt, uint32_t n_d0, uint32_t n_qpt, uint32_t nphi,
              uint32_t log2phi, uint32_t rp, uint32_t n_kt, uint32_t thr, uint32_t *__restrict__ tile_counts,
              const uint64_t *__restrict__ tile_off, uint2 *__restrict__ peaks, uint64_t capacity)
{
    HOUGH_DYNAMIC_LDS(uint32_t, val);
    __shared__ uint32_t wave_cnt[4];
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t item = blockIdx.x;
    const uint32_t per_event = n_d0 * n_kt;
    const uint32_t e = item / per_event;
    const uint32_t d = (item % per_event) / n_kt;
    const uint32_t k0 = (item % n_kt) * rp;
    const uint32_t nr = min(rp, n_qpt - k0);
    const uint32_t planes = n_d0 > 1 ? 3 : 1;
    const uint32_t prow = nr + 2;
    const uint64_t cells = uint64_t(n_d0) * n_qpt * nphi;
    const uint32_t *ev = cnt + uint64_t(e) * cells;
    // absent neighbours stage as 0, which never exceeds a cell's count
    const uint32_t staged = planes * prow * nphi;
    for (uint32_t i = t; i < staged; i += nt) {
        const uint32_t p = i & (nphi - 1);
        const uint32_t row = i >> log2phi;
        const uint32_t pl = planes == 1 ? 0 : row / prow;
        const uint32_t rr = row - pl * prow;
        const int dd = planes == 3 ? int(d) + int(pl) - 1 : int(d);
        const int kk = int(k0) + int(rr) - 1;
        uint32_t v = 0;
        if (dd >= 0 && dd < int(n_d0) && kk >= 0 && kk < int(n_qpt)) v = ev[(uint64_t(dd) * n_qpt + kk) * nphi + p];
        val[i] = v;
    }
    __syncthreads();

    const uint32_t cp = planes == 3 ? 1 : 0;
    const uint32_t ncell = nr * nphi;
    const uint32_t lane = t & 63, wave = t >> 6, nwaves = nt >> 6;
    uint32_t count = 0;
    uint64_t running = WRITE ? tile_off[item] : 0;
    for (uint32_t base = 0; base < ncell; base += nt) {
        const uint32_t cidx = base + t;
        bool is_peak = false;
        uint32_t rr = 0, p = 0, v = 0;
        if (cidx < ncell) {
            rr = cidx >> log2phi;
            p = cidx & (nphi - 1);
            const uint32_t pm = (p - 1) & (nphi - 1), pp = (p + 1) & (nphi - 1);
            v = val[(cp * prow + rr + 1) * nphi + p];
            if (v >= thr) {
                bool ok = true;
                for (uint32_t pl = 0; pl < planes && ok; ++pl) {
                    for (uint32_t dr = 0; dr < 3; ++dr) {
                        const uint32_t *row = val + (pl * prow + rr + dr) * nphi;
                        const bool centre_row = pl == cp && dr == 1;
                        ok &= row[pm] <= v && row[pp] <= v && (centre_row || row[p] <= v);
                    }
                }
                is_peak = ok;
            }
        }
        if (!WRITE) {
            count += is_peak;
            continue;
        }
        const uint64_t bal = __ballot(is_peak);
        const uint32_t before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wave] = __popcll(bal);
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < nwaves; ++w) {
            const uint32_t x = wave_cnt[w];
            woff += w < wave ? x : 0;
            total += x;
        }
        if (is_peak) {
            const uint64_t pos = running + woff + before;
            if (pos < capacity)
                peaks[pos] = make_uint2(uint32_t((uint64_t(d) * n_qpt + k0 + rr) * nphi + p), v);
        }
        running += total;
        __syncthreads();
    }
    if (!WRITE) {
        for (uint32_t off = 32; off > 0; off >>= 1) count += __shfl_down(count, off, 64);
        if (lane == 0) wave_cnt[wave] = count;
        __syncthreads();
        if (t == 0) {
            uint32_t s = 0;
            for (uint32_t w = 0; w < nwaves; ++w) s += wave_cnt[w];
            tile_counts[item] = s;
        }
    }
}

namespace {


// LDS of one peak tile of rp rows: popcounts of the staged rows (bytes in
// the scalar kernel, uint16 in the vector one, which with WRITE adds the raw
// centre rows and a chunk of records).
size_t peaks_lds_bytes(const hough_ctx *c, uint32_t rp, bool vec, bool write = true)
{
    const uint32_t planes = c->spec.n_d0 > 1 ? 3 : 1;
    const size_t pc = size_t(planes) * (rp + 2) * c->spec.n_phi;
    if (!vec) return pc;
    const size_t pc16 = (2 * pc + 15) & ~size_t(15);
    if (!write) return pc16;
    return pc16 + size_t(rp) * c->spec.n_phi * 2 + size_t(kPeakThreads) * 4 * 8;
}

// Rows per peak tile: the tuned or default value, reduced until the staged
// popcount bytes fit in the LDS budget; 0 if a single row does not fit.
uint32_t fit_rows(const hough_ctx *c, bool vec)
{
    uint32_t rp = std::min(peak_rows(c), c->spec.n_qpt);
    while (rp > 0 && peaks_lds_bytes(c, rp, vec) > c->max_lds) --rp;
    return rp;
}

}  // namespace

uint64_t peak_items(const hough_ctx *c, uint32_t n_events, const uint16_t *acc)
{
    if (peak_rows_cells_per_lane(c, acc, n_events)) {
        const uint32_t R = peak_rows_strip(c);
        return uint64_t(n_events) * c->spec.n_d0 * ((c->spec.n_qpt + R - 1) / R);
    }
    const bool vec = c->spec.n_phi >= 8 && (reinterpret_cast<uintptr_t>(acc) & 15) == 0 &&
                     fit_rows(c, true) > 0;
    const uint32_t rp = fit_rows(c, vec);
    if (rp == 0) return 0;
    const uint32_t n_kt = (c->spec.n_qpt + rp - 1) / rp;
    return uint64_t(n_events) * c->spec.n_d0 * n_kt;
}

PeakScratch ctx_peak_scratch(hough_ctx *c)
{
    return PeakScratch{c->d_tile_counts, c->d_tile_off, c->d_scan_part, c->d_scan_off, c->scan_blocks_max};
}

hipError_t launch_peaks(hough_ctx *c, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                        uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s, const PeakScratch &ps,
                        bool timed)
{
    hipError_t err;
    KernelTimer t;
    t.name = nullptr;
    if (peak_rows_cells_per_lane(c, acc, n_events)) {
        const uint32_t R = peak_rows_strip(c);
        const uint32_t n_strips = (c->spec.n_qpt + R - 1) / R;
        if (n_events == 0)
            return launch_scan_counts(c, ps.tile_counts, 0, ps.tile_off, 1, event_peak_offsets, s, ps.scan_part,
                                      ps.scan_off, ps.scan_blocks_max, timed);
        if (timed) prof_begin(c, "peaks_count", s, &t);
        err = launch_peaks_rows_pass(c, false, acc, n_events, peaks, capacity, ps, s);
        if (timed) prof_end(c, s, &t);
        if (err != hipSuccess) return err;
        if ((err = launch_scan_counts(c, ps.tile_counts, uint64_t(n_events) * c->spec.n_d0 * n_strips, ps.tile_off,
                                      uint64_t(c->spec.n_d0) * n_strips,
                                      event_peak_offsets, s, ps.scan_part, ps.scan_off, ps.scan_blocks_max,
                                      timed)) != hipSuccess)
            return err;
        if (timed) prof_begin(c, "peaks_write", s, &t);
        err = launch_peaks_rows_pass(c, true, acc, n_events, peaks, capacity, ps, s);
        if (timed) prof_end(c, s, &t);
        return err;
    }
    const bool vec = c->spec.n_phi >= 8 && (reinterpret_cast<uintptr_t>(acc) & 15) == 0 &&
                     fit_rows(c, true) > 0;
    const uint32_t rp = fit_rows(c, vec);
    if (rp == 0) return hipErrorInvalidConfiguration;
    const uint32_t n_kt = (c->spec.n_qpt + rp - 1) / rp;
    const uint64_t n_items = uint64_t(n_events) * c->spec.n_d0 * n_kt;
    if (n_events == 0) {
        return launch_scan_counts(c, ps.tile_counts, 0, ps.tile_off, 1, event_peak_offsets, s, ps.scan_part,
                                  ps.scan_off, ps.scan_blocks_max, timed);
    }
    const size_t lds = peaks_lds_bytes(c, rp, vec);
    if (timed) prof_begin(c, "peaks_count", s, &t);
    if (vec)
        hipLaunchKernelGGL(k_peaks_vec<false>, dim3(uint32_t(n_items)), dim3(kPeakThreads),
                           peaks_lds_bytes(c, rp, true, false),
                           s, acc, c->spec.n_d0, c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt,
                           c->spec.threshold, ps.tile_counts, ps.tile_off, peaks, capacity);
    else
        hipLaunchKernelGGL(k_peaks<false>, dim3(uint32_t(n_items)), dim3(kPeakThreads), lds, s, acc, c->spec.n_d0,
                           c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt, c->spec.threshold,
                           ps.tile_counts, ps.tile_off, peaks, capacity);
    if (timed) prof_end(c, s, &t);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_scan_counts(c, ps.tile_counts, n_items, ps.tile_off, uint64_t(c->spec.n_d0) * n_kt,
                                  event_peak_offsets, s, ps.scan_part, ps.scan_off, ps.scan_blocks_max,
                                  timed)) != hipSuccess)
        return err;
    if (timed) prof_begin(c, "peaks_write", s, &t);
    if (vec)
        hipLaunchKernelGGL(k_peaks_vec<true>, dim3(uint32_t(n_items)), dim3(kPeakThreads), lds, s, acc, c->spec.n_d0,
                           c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt, c->spec.threshold,
                           ps.tile_counts, ps.tile_off, peaks, capacity);
    else
        hipLaunchKernelGGL(k_peaks<true>, dim3(uint32_t(n_items)), dim3(kPeakThreads), lds, s, acc, c->spec.n_d0,
                           c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt, c->spec.threshold,
                           ps.tile_counts, ps.tile_off, peaks, capacity);
    if (timed) prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_peaks(hough_ctx *c, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                        uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s)
{
    return launch_peaks(c, acc, n_events, peaks, capacity, event_peak_offsets, s, ctx_peak_scratch(c), true);
}

hipError_t launch_peaks_count(hough_ctx *c, const uint32_t *counts, uint32_t n_events, uint2 *peaks,
                              uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s)
{
    hipError_t err;
    const uint32_t planes = c->spec.n_d0 > 1 ? 3 : 1;
    uint32_t rp = std::min(peak_rows(c), c->spec.n_qpt);
    while (rp > 0 && size_t(planes) * (rp + 2) * c->spec.n_phi * 4 > c->max_lds) --rp;
    if (rp == 0) return hipErrorInvalidConfiguration;
    const uint32_t n_kt = (c->spec.n_qpt + rp - 1) / rp;
    const uint64_t n_items = uint64_t(n_events) * c->spec.n_d0 * n_kt;
    if (n_events == 0) return launch_scan_counts(c, c->d_tile_counts, 0, c->d_tile_off, 1, event_peak_offsets, s);
    const size_t lds = size_t(planes) * (rp + 2) * c->spec.n_phi * 4;
    KernelTimer t;
    prof_begin(c, "peaks_count_form", s, &t);
    hipLaunchKernelGGL(k_peaks_count<false>, dim3(uint32_t(n_items)), dim3(kPeakThreads), lds, s, counts,
                       c->spec.n_d0, c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt, c->spec.threshold,
                       c->d_tile_counts, c->d_tile_off, peaks, capacity);
    prof_end(c, s, &t);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_scan_counts(c, c->d_tile_counts, n_items, c->d_tile_off, uint64_t(c->spec.n_d0) * n_kt,
                                  event_peak_offsets, s)) != hipSuccess)
        return err;
    prof_begin(c, "peaks_write_count_form", s, &t);
    hipLaunchKernelGGL(k_peaks_count<true>, dim3(uint32_t(n_items)), dim3(kPeakThreads), lds, s, counts,
                       c->spec.n_d0, c->spec.n_qpt, c->spec.n_phi, c->log2_phi, rp, n_kt, c->spec.threshold,
                       c->d_tile_counts, c->d_tile_off, peaks, capacity);
    prof_end(c, s, &t);
    return hipGetLastError();
}

uint64_t max_peak_tiles(const hough_ctx *c)
{
    // the smallest tile is one row, so at most every row of every event
    return uint64_t(c->lim.max_events) * c->rows;
}

}  // namespace hough
