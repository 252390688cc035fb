// Step 1 of the transform in its direct bin-occupancy form (Section 4, first
// step; the Discussion's A[B[i]] += 1 in layer-mask form), the default vote
// algorithm.
//
// Split a row's offset as o = J W + f (J = o >> s, f = o mod W, W = 2^s) and
// the azimuth circle into W-wide buckets aligned at 0.  Bin p of the row is
// [o + p W, o + (p+1) W): the part of bucket j = J + p at or above fine
// offset f, and the part of bucket j + 1 below f (indices mod n_phi).  So
// the bin holds a hit of the layer unless
//     max fine offset of bucket j < f   and   min fine offset of bucket j+1 >= f,
// i.e. unless lo_j <= f <= hi_j with lo_j = (max fine of bucket j) + 1 (0 when
// the bucket is empty) and hi_j = min fine of bucket j+1 (W - 1 when empty).
// Per (event, layer, bucket) the table holds {lo_j, hi_j - lo_j}, or
// {2^32 - 1, 0} when lo_j > hi_j (the bin is never empty); then the bin is
// occupied iff (f - lo_j) mod 2^32 > span_j, one subtract and one compare.
// The result is bit-identical to the per-hit vote.
//
// k_vote_bounds (one workgroup per event): bucket minima and maxima with LDS
// atomics, then the table.  k_vote_direct (grid-stride over items of one
// event and a run of R-row tiles): the event's table is staged in LDS once
// per item; in a tile every lane owns one cell column and walks the R rows,
// building each row's layer mask in a register; the bucket a lane reads for
// a layer changes only when a row's J changes, so table reads are rare;
// masks go straight to HBM.
#include "hough_internal.h"

namespace hough {

namespace {

// Calls f(layer, phi) for every hit of [b, end); with `vec` (layer 4-byte
// and phi 16-byte aligned) the aligned middle is read four hits per load.
template <class F>
__device__ __forceinline__ void event_hits(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
                                           uint64_t b, uint64_t end, uint32_t t, uint32_t nt, bool vec, F &&f)
{
    uint64_t tail = b;
    if (vec) {
        const uint64_t a = min((b + 3) & ~uint64_t(3), end);
        if (t < a - b) f(uint32_t(layer[b + t]), phi[b + t]);
        const uint64_t nq = (end - a) >> 2;
        const uint32_t *l4 = reinterpret_cast<const uint32_t *>(layer + a);
        const uint4 *p4 = reinterpret_cast<const uint4 *>(phi + a);
        for (uint64_t q = t; q < nq; q += nt) {
            const uint32_t lw = l4[q];
            const uint4 pw = p4[q];
            f(lw & 0xFFu, pw.x);
            f((lw >> 8) & 0xFFu, pw.y);
            f((lw >> 16) & 0xFFu, pw.z);
            f(lw >> 24, pw.w);
        }
        tail = a + (nq << 2);
    }
    for (uint64_t i = tail + t; i < end; i += nt) f(uint32_t(layer[i]), phi[i]);
}

// m[k] = 2 m[k] + [(f - lo[k]) mod 2^32 > span[k]] for four cells, f
// wave-uniform.  On the GPU: per cell a subtract, a subtract whose borrow
// out (into its own scalar register pair) is exactly the comparison, and an
// add with that borrow as carry in; the four chains are interleaved so no
// carry is read right after it is written.  The expression in the other
// branch is the same arithmetic for host compilation.
__device__ __forceinline__ void shift_in_occupied4(uint32_t (&m)[4], uint32_t f, const uint32_t (&lo)[4],
                                                   const uint32_t (&span)[4])
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t d0, d1, d2, d3;
    uint64_t c0, c1, c2, c3;
    asm("v_sub_u32 %4, %12, %13\n\t"
        "v_sub_u32 %5, %12, %14\n\t"
        "v_sub_u32 %6, %12, %15\n\t"
        "v_sub_u32 %7, %12, %16\n\t"
        "v_sub_co_u32 %4, %8, %17, %4\n\t"
        "v_sub_co_u32 %5, %9, %18, %5\n\t"
        "v_sub_co_u32 %6, %10, %19, %6\n\t"
        "v_sub_co_u32 %7, %11, %20, %7\n\t"
        "v_addc_co_u32 %0, %8, %0, %0, %8\n\t"
        "v_addc_co_u32 %1, %9, %1, %1, %9\n\t"
        "v_addc_co_u32 %2, %10, %2, %2, %10\n\t"
        "v_addc_co_u32 %3, %11, %3, %3, %11"
        : "+v"(m[0]), "+v"(m[1]), "+v"(m[2]), "+v"(m[3]), "=&v"(d0), "=&v"(d1), "=&v"(d2), "=&v"(d3),
          "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
        : "s"(f), "v"(lo[0]), "v"(lo[1]), "v"(lo[2]), "v"(lo[3]), "v"(span[0]), "v"(span[1]), "v"(span[2]),
          "v"(span[3]));
#else
    for (int k = 0; k < 4; ++k) m[k] = 2 * m[k] + (f - lo[k] > span[k] ? 1u : 0u);
#endif
}

}  // namespace

// tab[e][l][j] = {lo_j, span_j} as defined above.  Layers are processed in
// groups whose bucket minima and maxima fit the LDS budget.
__global__ void __launch_bounds__(1024)
k_vote_bounds(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
              const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_layers, uint32_t nphi,
              uint32_t log2phi, uint32_t shift, uint32_t group_layers, int vec, uint2 *__restrict__ tab)
{
    HOUGH_DYNAMIC_LDS(uint32_t, lds);                // bmin[gl][nphi], bmax[gl][nphi]
    const uint32_t e = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    const uint32_t wmask = (1u << shift) - 1u;
    const uint64_t b = min(offs[e], n_hits);
    uint64_t end = min(offs[e + 1], n_hits);
    if (end < b) end = b;
    for (uint32_t l0 = 0; l0 < n_layers; l0 += group_layers) {
        const uint32_t gl = min(group_layers, n_layers - l0);
        uint32_t *bmin = lds, *bmax = lds + gl * nphi;
        for (uint32_t i = t; i < gl * nphi; i += nt) {
            bmin[i] = 0xFFFFFFFFu;
            bmax[i] = 0u;
        }
        __syncthreads();
        event_hits(layer, phi, b, end, t, nt, vec, [&](uint32_t l, uint32_t ph) {
            if (l >= l0 && l < l0 + gl) {
                const uint32_t bi = (l - l0) * nphi + (ph >> shift);
                atomicMin(&bmin[bi], ph);
                atomicMax(&bmax[bi], ph);
            }
        });
        __syncthreads();
        uint2 *out = tab + (size_t(e) * n_layers + l0) * nphi;
        for (uint32_t i = t; i < gl * nphi; i += nt) {
            const uint32_t ll = i >> log2phi, j = i & (nphi - 1);
            const uint32_t jn = ll * nphi + ((j + 1) & (nphi - 1));
            const bool ne = bmin[i] <= bmax[i], ne1 = bmin[jn] <= bmax[jn];
            const uint32_t lo = ne ? (bmax[i] & wmask) + 1u : 0u;    // may equal W: never empty
            const uint32_t hi = ne1 ? (bmin[jn] & wmask) : wmask;
            out[i] = hi >= lo ? make_uint2(lo, hi - lo) : make_uint2(0xFFFFFFFFu, 0u);
        }
        __syncthreads();
    }
}

// Split form of k_vote_bounds for batches of few events: the table is first
// filled with {min, max} = {0xFFFFFFFF, 0}; each of an event's K parts (a
// workgroup over a K-th of its hits) finds its own minima and maxima in LDS
// and merges the non-empty ones into the table with global atomic min/max;
// then one workgroup per (event, layer) turns the row's {min, max} into
// {lo, span} exactly as k_vote_bounds does.
__global__ void k_bounds_init(uint2 *__restrict__ tab, uint64_t n)
{
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        tab[i] = make_uint2(0xFFFFFFFFu, 0u);
}

__global__ void __launch_bounds__(256)
k_bounds_part(const uint8_t *__restrict__ layer, const uint32_t *__restrict__ phi,
              const uint64_t *__restrict__ offs, uint64_t n_hits, uint32_t n_layers, uint32_t nphi, uint32_t shift,
              uint32_t group_layers, uint32_t K, uint2 *__restrict__ tab)
{
    HOUGH_DYNAMIC_LDS(uint32_t, lds);                // bmin[gl][nphi], bmax[gl][nphi]
    const uint32_t e = blockIdx.x / K, k = blockIdx.x % K, t = threadIdx.x, nt = blockDim.x;
    const uint64_t b0 = min(offs[e], n_hits);
    uint64_t end0 = min(offs[e + 1], n_hits);
    if (end0 < b0) end0 = b0;
    const uint64_t len = end0 - b0;
    const uint64_t b = b0 + len * k / K, end = b0 + len * (k + 1) / K;
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
            }
        }
        __syncthreads();
        uint2 *out = tab + (size_t(e) * n_layers + l0) * nphi;
        for (uint32_t i = t; i < gl * nphi; i += nt) {
            if (bmin[i] <= bmax[i]) {
                atomicMin(&out[i].x, bmin[i]);
                atomicMax(&out[i].y, bmax[i]);
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
k_bounds_final(uint32_t nphi, uint32_t shift, uint2 *__restrict__ tab)
{
    HOUGH_DYNAMIC_LDS(uint2, row);                   // [nphi] {min, max}
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t wmask = (1u << shift) - 1u;
    uint2 *r = tab + size_t(blockIdx.x) * nphi;      // one (event, layer) row
    for (uint32_t j = t; j < nphi; j += nt) row[j] = r[j];
    __syncthreads();
    for (uint32_t j = t; j < nphi; j += nt) {
        const uint2 a = row[j], n = row[(j + 1) & (nphi - 1)];
        const bool ne = a.x <= a.y, ne1 = n.x <= n.y;
        const uint32_t lo = ne ? (a.y & wmask) + 1u : 0u;        // may equal W: never empty
        const uint32_t hi = ne1 ? (n.x & wmask) : wmask;
        r[j] = hi >= lo ? make_uint2(lo, hi - lo) : make_uint2(0xFFFFFFFFu, 0u);
    }
}

// One workgroup of nt threads (a multiple of 64) per item.  Work unit = (tile,
// group of CPW 64-cell column chunks); waves take units round-robin.  For
// each layer, from the highest down, a lane walks the R rows of the tile
// (unrolled, masks in registers, mask = 2 mask + occupied) for its CPW cells
// and keeps their table entries, re-read only when a row's J changes; the
// row offsets are wave-uniform scalars shared by the CPW cells.
// The event's table is staged in LDS with LDS_TAB, else read from `tab`.
template <int R, int CPW, bool ALLV, bool LDS_TAB>
__global__ void __launch_bounds__(256)
k_vote_direct(const uint2 *__restrict__ tab, const uint32_t *__restrict__ O, const uint8_t *__restrict__ V,
              uint32_t n_layers, uint32_t rows, uint32_t nphi, uint32_t shift, uint32_t n_tiles,
              uint32_t run_tiles, uint32_t runs_per_event, uint32_t n_items, uint16_t *__restrict__ acc)
{
    HOUGH_DYNAMIC_LDS(uint2, tab_s);                 // [L][nphi] with LDS_TAB
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    const uint32_t lane = t & 63, nwaves = nt >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);   // uniform: row offsets are scalar loads
    const uint64_t cells = uint64_t(rows) * nphi;
    const uint32_t wmask = (1u << shift) - 1u;
    const uint32_t nchunks = (nphi + 63) >> 6;
    const uint32_t ngroups = (nchunks + CPW - 1) / CPW;
    const uint32_t tab_words = n_layers * nphi;

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t e = item / runs_per_event;
        const uint32_t tile_lo = (item % runs_per_event) * run_tiles;
        const uint32_t tile_hi = min(n_tiles, tile_lo + run_tiles);
        const uint2 *etab = tab + size_t(e) * tab_words;
        if (LDS_TAB) {
            for (uint32_t i = t; i < tab_words; i += nt) tab_s[i] = etab[i];
            __syncthreads();
        }
        const uint32_t units = (tile_hi - tile_lo) * ngroups;
        for (uint32_t u = wave; u < units; u += nwaves) {
            const uint32_t r0 = (tile_lo + u / ngroups) * R;
            const uint32_t nr = min(uint32_t(R), rows - r0);
            const uint32_t pbase = (u % ngroups) * CPW * 64 + lane;
            uint32_t mask[CPW][R];
#pragma unroll
            for (uint32_t k = 0; k < CPW; ++k)
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) mask[k][r] = 0;
            for (uint32_t l = n_layers; l-- > 0;) {
                const uint32_t *Ol = O + size_t(l) * rows + r0;   // padded: R entries readable
                uint32_t okm = 0xFFFFFFFFu;
                if (!ALLV) {
                    okm = 0;
                    for (uint32_t r = 0; r < nr; ++r)
                        if (V[size_t(l) * rows + r0 + r]) okm |= 1u << r;
                }
                uint32_t ov[R];                          // scalar loads, issued together
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) ov[r] = Ol[r];
                uint32_t jcur = 0xFFFFFFFFu, lo[CPW], span[CPW];
#pragma unroll
                for (uint32_t k = 0; k < CPW; ++k) lo[k] = span[k] = 0;
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    const uint32_t o = ov[r];
                    const uint32_t J = o >> shift, f = o & wmask;
                    if (J != jcur) {
                        jcur = J;
#pragma unroll
                        for (uint32_t k = 0; k < CPW; ++k) {
                            const uint32_t j = l * nphi + ((J + pbase + 64 * k) & (nphi - 1));
                            const uint2 v = LDS_TAB ? tab_s[j] : etab[j];
                            lo[k] = v.x;
                            span[k] = v.y;
                        }
                    }
                    if (ALLV || ((okm >> r) & 1u)) {
                        uint32_t mr[CPW];
#pragma unroll
                        for (uint32_t k = 0; k < CPW; ++k) mr[k] = mask[k][r];
                        shift_in_occupied4(mr, f, lo, span);
#pragma unroll
                        for (uint32_t k = 0; k < CPW; ++k) mask[k][r] = mr[k];
                    } else {
#pragma unroll
                        for (uint32_t k = 0; k < CPW; ++k) mask[k][r] *= 2;
                    }
                }
            }
            uint16_t *dst = acc + uint64_t(e) * cells + uint64_t(r0) * nphi;
#pragma unroll
            for (uint32_t k = 0; k < CPW; ++k) {
                const uint32_t p = pbase + 64 * k;
                if (p < nphi) {
#pragma unroll
                    for (uint32_t r = 0; r < R; ++r)
                        if (r < nr) dst[uint64_t(r) * nphi + p] = uint16_t(mask[k][r]);
                }
            }
        }
        if (LDS_TAB) __syncthreads();
    }
}

namespace {

constexpr int kDirectCpw = 4;   // cells per lane: shift_in_occupied4

template <int R, bool ALLV, bool LDS_TAB>
void launch_direct_v(hough_ctx *c, uint32_t grid, uint32_t threads, size_t lds, hipStream_t s, uint32_t n_tiles,
                     uint32_t run, uint32_t runs, uint32_t n_items, uint16_t *acc)
{
    hipLaunchKernelGGL((k_vote_direct<R, kDirectCpw, ALLV, LDS_TAB>), dim3(grid), dim3(threads), lds, s, c->d_dir_tab, c->d_O,
                       c->d_V, c->spec.n_layers, c->rows, c->spec.n_phi, c->shift, n_tiles, run, runs, n_items, acc);
}

template <int R>
void launch_direct(hough_ctx *c, uint32_t n_events, uint16_t *acc, uint32_t threads, bool lds_tab, hipStream_t s)
{
    const uint32_t n_tiles = (c->rows + R - 1) / R;
    const uint32_t per_cu = c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 8;
    const uint64_t want = uint64_t(c->n_cu) * per_cu;
    // runs of tiles sharing one staging of the event's table, while there
    // are still about four items per workgroup
    const uint64_t all = uint64_t(n_tiles) * n_events;
    const uint32_t run = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(n_tiles, all / (want * 4))));
    const uint32_t runs = (n_tiles + run - 1) / run;
    const uint32_t n_items = runs * n_events;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(n_items, want)));
    const size_t lds = lds_tab ? size_t(c->spec.n_layers) * c->spec.n_phi * 8 : 0;
    if (c->all_valid && lds_tab)
        launch_direct_v<R, true, true>(c, grid, threads, lds, s, n_tiles, run, runs, n_items, acc);
    else if (c->all_valid)
        launch_direct_v<R, true, false>(c, grid, threads, lds, s, n_tiles, run, runs, n_items, acc);
    else if (lds_tab)
        launch_direct_v<R, false, true>(c, grid, threads, lds, s, n_tiles, run, runs, n_items, acc);
    else
        launch_direct_v<R, false, false>(c, grid, threads, lds, s, n_tiles, run, runs, n_items, acc);
}

}  // namespace

// Rows per direct-vote tile (a register per row, cell and lane; at most
// 16): the tuned value, else 16.
uint32_t direct_rows(const hough_ctx *c)
{
    return std::min(16u, c->tun.vote_rows ? c->tun.vote_rows : 16u);
}

bool direct_vote_usable(const hough_ctx *c)
{
    return c->d_dir_tab != nullptr && size_t(c->spec.n_phi) * 8 <= c->max_lds;
}

hipError_t launch_vote_bounds(hough_ctx *c, const hough_hits *h, hipStream_t s)
{
    const uint32_t E = h->n_events;
    const uint32_t group = uint32_t(std::min<size_t>(c->spec.n_layers, c->max_lds / (size_t(c->spec.n_phi) * 8)));
    const int vec = (reinterpret_cast<uintptr_t>(h->layer) & 3) == 0 && (reinterpret_cast<uintptr_t>(h->phi) & 15) == 0;
    KernelTimer t;
    prof_begin(c, "vote_bounds", s, &t);
    // split only events with many hits per table entry (at least 16): the
    // split form costs two more launches, and each part initialises and
    // merges its event's whole (layer, bucket) table (the 198k-hit displaced
    // event: 42 us in one workgroup, 22 us in 64 parts; the 20k-hit event on
    // 10 x 1024 entries: 13 us in one, 18 us in 64 parts)
    const uint64_t entries = uint64_t(c->spec.n_layers) * c->spec.n_phi;
    const uint64_t per_event = E ? h->n_hits / E : 0;
    const uint32_t K = per_event >= 16 * entries ? split_parts(c, E) : 0;
    if (K >= 2) {
        const uint64_t n = uint64_t(E) * entries;
        hipLaunchKernelGGL(k_bounds_init, dim3(uint32_t(std::min<uint64_t>((n + 255) / 256, 4096))), dim3(256), 0, s,
                           c->d_dir_tab, n);
        hipLaunchKernelGGL(k_bounds_part, dim3(E * K), dim3(256), size_t(group) * c->spec.n_phi * 8, s, h->layer,
                           h->phi, h->event_offsets, h->n_hits, c->spec.n_layers, c->spec.n_phi, c->shift, group, K,
                           c->d_dir_tab);
        hipLaunchKernelGGL(k_bounds_final, dim3(E * c->spec.n_layers), dim3(256), size_t(c->spec.n_phi) * 8, s,
                           c->spec.n_phi, c->shift, c->d_dir_tab);
    } else {
        hipLaunchKernelGGL(k_vote_bounds, dim3(E), dim3(1024), size_t(group) * c->spec.n_phi * 8, s, h->layer,
                           h->phi, h->event_offsets, h->n_hits, c->spec.n_layers, c->spec.n_phi, c->log2_phi,
                           c->shift, group, vec, c->d_dir_tab);
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

hipError_t launch_vote_direct(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s)
{
    const uint32_t E = h->n_events;
    KernelTimer t;
    hipError_t err = launch_vote_bounds(c, h, s);
    if (err != hipSuccess) return err;
    uint32_t R = direct_rows(c);
    if (!c->tun.vote_rows) {
        // small batches: shorter tiles until there are enough of them
        const uint64_t want = uint64_t(c->n_cu) * (c->tun.vote_wgs_per_cu ? c->tun.vote_wgs_per_cu : 8);
        while (R > 8 && uint64_t((c->rows + R - 1) / R) * E < want) R >>= 1;
    }
    const bool lds_tab = size_t(c->spec.n_layers) * c->spec.n_phi * 8 <= c->max_lds_direct;
    const uint32_t threads = std::min(256u, std::max(64u, c->tun.vote_threads ? c->tun.vote_threads : 256u));
    prof_begin(c, "vote_direct", s, &t);
    switch (R) {
    case 1: launch_direct<1>(c, E, acc, threads, lds_tab, s); break;
    case 2: launch_direct<2>(c, E, acc, threads, lds_tab, s); break;
    case 4: launch_direct<4>(c, E, acc, threads, lds_tab, s); break;
    case 8: launch_direct<8>(c, E, acc, threads, lds_tab, s); break;
    default: launch_direct<16>(c, E, acc, threads, lds_tab, s); break;
    }
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
