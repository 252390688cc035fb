// rz refinement of candidate cells: the "more expensive computations to
// confirm" that Section 3 leaves to follow the local-maximum search.
//
// Candidates of an event are its peaks (in list order), or the first
// rz_max_candidates of them by (popcount desc, cell asc).  For a candidate
// (k, p) the members are the hits that voted into that exact cell; they sit
// in a few coarse azimuth buckets of each layer named in the cell's mask.
// Each member votes once per cot(theta) bin j at z0 bin
//   b = floor((z - Z[k][l][j] - z0_lo) * n_z0 / (z0_hi - z0_lo)),
// and the record is the argmax over (j, b), ties to the smallest j then b.
//
// One 64-wide wavefront per candidate, persistent over a work counter.  A
// lane owns cot bins j = lane, lane + 64, ... and a private uint16 z0
// histogram column in LDS (hist[b * 64 + lane]): its running maximum is
// exact because counts only grow, and the touched bins are cleared after
// each cot bin.  A candidate with more than 65535 members (or a z0 grid too
// large for LDS) takes a slower path through a uint32 histogram in global
// scratch, one cot bin at a time.
#include "fastdiv.h"
#include "hough_internal.h"

namespace hough {

struct RzParams {
    const uint32_t *phi;          // hits grouped by (layer, bucket)
    const int32_t *z;
    const uint64_t *offs;
    uint64_t n_hits;
    const uint32_t *bucket_off;   // [E][L][NB + 1]
    const uint32_t *O;            // [L][rows]
    const uint8_t *V;
    const int32_t *Z;             // [K][L][C]
    const uint2 *peaks;
    uint64_t peak_capacity;
    const uint64_t *poff;         // [E + 1]
    const uint64_t *roff;         // [E + 1]
    const uint32_t *cand;         // selected local peak indices (cap > 0)
    uint2 *out4;                  // hough_rz records as 4 x uint32 (2 x uint2)
    uint64_t out_capacity;
    uint32_t *counter;
    uint32_t *gscratch;           // [blocks][n_z0] zeroed uint32, slow path
    uint32_t n_events, n_layers, n_qpt, rows, nphi, log2phi, shift, bucket_bits;
    uint32_t n_z0, n_cot, cap;
    int64_t z0_lo;
    uint64_t span;                // z0_hi - z0_lo
    int use32;                    // span * n_z0 < 2^32: fast 32-bit division
    FastDiv32 fd;
    int lds_ok;                   // the uint16 histogram fits in LDS
};

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return uint64_t(uni(uint32_t(v))) | (uint64_t(uni(uint32_t(v >> 32))) << 32);
}

// z0 bin of a member, or -1 when outside [z0_lo, z0_hi).
__device__ __forceinline__ int32_t z0_bin(const RzParams &P, int32_t z, int64_t zl)
{
    const int64_t x = int64_t(z) - zl;
    if (x < 0 || uint64_t(x) >= P.span) return -1;
    if (P.use32) return int32_t(fastdiv32(uint32_t(x) * P.n_z0, P.fd));
    const double q = double(uint64_t(x) * P.n_z0) / double(P.span);
    return int32_t(q);
}

// Visits the member hits of candidate (k, p): fn(hit index relative to the
// event, layer).  All lanes see every hit (uniform loop).
template <typename Fn>
__device__ __forceinline__ void for_members(const RzParams &P, uint64_t eb, const uint32_t *bo,
                                            uint32_t k, uint32_t p, uint32_t mask, Fn &&fn)
{
    const uint32_t nb = 1u << P.bucket_bits, bs = 32 - P.bucket_bits;
    const uint64_t W = uint64_t(1) << P.shift, BW = uint64_t(1) << bs;
    for (uint32_t l = 0; l < P.n_layers; ++l) {
        if (!((mask >> l) & 1u)) continue;
        const size_t ti = size_t(l) * P.rows + k;
        if (!P.V[ti]) continue;
        const uint32_t o = P.O[ti];
        const uint32_t start = o + (p << P.shift);
        const uint32_t b0 = start >> bs;
        const uint32_t nbk = uint32_t(((uint64_t(start) & (BW - 1)) + W - 1) / BW + 1);
        const uint32_t *bl = bo + size_t(l) * (nb + 1);
        for (uint32_t i = 0; i < nbk && i < nb; ++i) {
            const uint32_t bk = (b0 + i) & (nb - 1);
            const uint32_t hs = bl[bk], he = bl[bk + 1];
            for (uint32_t h = hs; h < he; ++h) {
                const uint32_t ph = P.phi[eb + h];
                if (((ph - o) >> P.shift) == p) fn(h, l);
            }
        }
    }
}

__global__ void __launch_bounds__(64) k_rz_vote(RzParams P)
{
    HOUGH_DYNAMIC_LDS(uint16_t, hist);       // [n_z0][64] when lds_ok
    const uint32_t lane = threadIdx.x;
    const uint64_t total = min(P.roff[P.n_events], P.out_capacity);
    if (P.lds_ok)
        for (uint32_t i = lane; i < P.n_z0 * 64; i += 64) hist[i] = 0;
    __syncthreads();
    uint32_t *g = P.gscratch + size_t(blockIdx.x) * P.n_z0;
    const uint32_t nb = 1u << P.bucket_bits;
    for (;;) {
        // Work fetch without lane-divergent control flow: every lane executes
        // the atomic (only lane 0 adds 1) and lane 0's ticket is broadcast by
        // readfirstlane.  A fetch guarded by "if (lane == 0)" followed by a
        // cross-lane read assumes the wave reconverges at the loop head, which
        // the compiler does not guarantee (it may keep lanes 1..63 cycling in
        // an inner loop that never re-reads the counter).
        const uint64_t c = uni(atomicAdd(P.counter, lane == 0 ? 1u : 0u));
        if (c >= total) break;
        // event of candidate c: largest e with roff[e] <= c
        uint32_t lo = 0, hi = P.n_events;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (P.roff[mid] <= c) lo = mid; else hi = mid;
        }
        const uint32_t e = uni(lo);
        const uint32_t local = uni(uint32_t(c - P.roff[e]));
        const uint32_t pk = P.cap ? uni(P.cand[c]) : local;
        const uint64_t gp = uni64(P.poff[e] + pk);
        const uint2 rec = P.peaks[gp];
        const uint32_t cell = uni(rec.x), mask = uni(rec.y & 0xFFFFu);
        const uint32_t k = (cell >> P.log2phi) % P.n_qpt, p = cell & (P.nphi - 1);
        const uint64_t eb = uni64(min(P.offs[e], P.n_hits));
        const uint32_t *bo = P.bucket_off + size_t(e) * P.n_layers * (nb + 1);

        uint32_t nm = 0;
        for_members(P, eb, bo, k, p, mask, [&](uint32_t, uint32_t) { ++nm; });

        uint32_t best_c = 0, best_j = lane, best_b = 0;     // lane's best over its cot bins
        if (P.lds_ok && nm <= 65535u) {
            for (uint32_t j0 = 0; j0 < P.n_cot; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool jv = j < P.n_cot;
                uint32_t bc = 0, bb = 0;
                for_members(P, eb, bo, k, p, mask, [&](uint32_t h, uint32_t l) {
                    if (!jv) return;
                    const int64_t zl = int64_t(P.Z[(size_t(k) * P.n_layers + l) * P.n_cot + j]) + P.z0_lo;
                    const int32_t b = z0_bin(P, P.z[eb + h], zl);
                    if (b < 0) return;
                    const uint32_t idx = uint32_t(b) * 64 + lane;
                    const uint32_t cnt = uint32_t(hist[idx]) + 1;
                    hist[idx] = uint16_t(cnt);
                    if (cnt > bc || (cnt == bc && uint32_t(b) < bb)) { bc = cnt; bb = uint32_t(b); }
                });
                for_members(P, eb, bo, k, p, mask, [&](uint32_t h, uint32_t l) {
                    if (!jv) return;
                    const int64_t zl = int64_t(P.Z[(size_t(k) * P.n_layers + l) * P.n_cot + j]) + P.z0_lo;
                    const int32_t b = z0_bin(P, P.z[eb + h], zl);
                    if (b >= 0) hist[uint32_t(b) * 64 + lane] = 0;
                });
                if (jv && bc > best_c) { best_c = bc; best_j = j; best_b = bb; }
            }
        } else {
            // slow path: one cot bin at a time, lanes stride over the members
            for (uint32_t j = 0; j < P.n_cot; ++j) {
                for (int pass = 0; pass < 3; ++pass) {
                    uint32_t seen = 0, bc = 0, bb = 0;
                    for_members(P, eb, bo, k, p, mask, [&](uint32_t h, uint32_t l) {
                        if ((seen++ & 63u) != lane) return;
                        const int64_t zl = int64_t(P.Z[(size_t(k) * P.n_layers + l) * P.n_cot + j]) + P.z0_lo;
                        const int32_t b = z0_bin(P, P.z[eb + h], zl);
                        if (b < 0) return;
                        if (pass == 0) {
                            atomicAdd(&g[b], 1u);
                        } else if (pass == 1) {
                            const uint32_t cnt = __atomic_load_n(&g[b], __ATOMIC_RELAXED);
                            if (cnt > bc || (cnt == bc && uint32_t(b) < bb)) { bc = cnt; bb = uint32_t(b); }
                        } else {
                            g[b] = 0;
                        }
                    });
                    // every lane's updates of this pass are complete and
                    // visible before any lane starts the next pass
                    __threadfence();
                    __syncthreads();
                    if (pass == 1) {
                        // wave argmax of (count desc, bin asc) for this cot bin
                        uint64_t key = (uint64_t(bc) << 32) | (0xFFFFFFFFu - bb);
                        for (int off = 32; off > 0; off >>= 1) {
                            const uint64_t o = __shfl_xor(key, off, 64);
                            key = o > key ? o : key;
                        }
                        const uint32_t cc = uint32_t(key >> 32), b = 0xFFFFFFFFu - uint32_t(key);
                        if (cc > best_c) { best_c = cc; best_j = j; best_b = cc ? b : 0; }
                    }
                }
            }
            if (lane != 0) { best_c = 0; best_j = 0xFFFFu; best_b = 0; }
            else if (best_c == 0) { best_j = 0; best_b = 0; }
        }
        // wave argmax of (count desc, cot asc, z0 asc)
        uint64_t key = (uint64_t(best_c) << 32) | (uint64_t(0xFFFFu - (best_j & 0xFFFFu)) << 16) |
                       (0xFFFFu - (best_b & 0xFFFFu));
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(key, off, 64);
            key = o > key ? o : key;
        }
        // key is wave-uniform after the butterfly: every lane stores the same
        // record to the same address (no divergent branch at the loop tail)
        {
            const uint32_t cnt = uint32_t(key >> 32);
            const uint32_t jj = 0xFFFFu - uint32_t((key >> 16) & 0xFFFFu);
            const uint32_t bb = 0xFFFFu - uint32_t(key & 0xFFFFu);
            uint2 a, b;
            a.x = pk;
            a.y = (cnt ? jj : 0u) | ((cnt ? bb : 0u) << 16);
            b.x = cnt;
            b.y = nm;
            P.out4[2 * c] = a;
            P.out4[2 * c + 1] = b;
        }
    }
}

// Per-event candidate counts: every available peak, or at most cap of them.
__global__ void k_rz_counts(const uint64_t *__restrict__ poff, uint64_t peak_capacity,
                            uint32_t n_events, uint32_t cap, uint32_t *__restrict__ counts)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_events) return;
    const uint64_t lo = min(poff[e], peak_capacity), hi = min(max(poff[e + 1], poff[e]), peak_capacity);
    const uint64_t n = hi - lo;
    counts[e] = uint32_t(cap ? min(n, uint64_t(cap)) : n);
}

// Candidate selection with a cap: the first cap peaks of the event ordered
// by (popcount desc, cell asc), i.e. a stable partition by popcount.  One
// workgroup of 256 threads per event.
__global__ void __launch_bounds__(256)
k_rz_select(const uint2 *__restrict__ peaks, uint64_t peak_capacity, const uint64_t *__restrict__ poff,
            const uint64_t *__restrict__ roff, uint32_t cap, uint32_t *__restrict__ cand)
{
    __shared__ uint32_t hist[17];
    __shared__ uint32_t wave_cnt[4];
    __shared__ uint32_t vstar_s, take_s;
    const uint32_t e = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint64_t lo = min(poff[e], peak_capacity), hi = min(max(poff[e + 1], poff[e]), peak_capacity);
    const uint64_t n = hi - lo;
    const uint32_t need = uint32_t(min(n, uint64_t(cap)));
    if (need == 0) return;
    if (t < 17) hist[t] = 0;
    __syncthreads();
    for (uint64_t i = lo + t; i < hi; i += blockDim.x) atomicAdd(&hist[min(peaks[i].y >> 16, 16u)], 1u);
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        vstar_s = 0;
        take_s = need;
        for (int v = 16; v >= 0; --v) {
            if (acc + hist[v] >= need) { vstar_s = uint32_t(v); take_s = need - acc; break; }
            acc += hist[v];
        }
    }
    __syncthreads();
    const uint32_t vstar = vstar_s, take = take_s;
    uint64_t pos = roff[e];
    for (int v = 16; v >= int(vstar); --v) {
        const uint32_t limit = uint32_t(v) == vstar ? take : hist[v];
        uint32_t taken = 0;
        for (uint64_t base = lo; base < hi && taken < limit; base += blockDim.x) {
            const uint64_t i = base + t;
            const bool sel = i < hi && min(peaks[i].y >> 16, 16u) == uint32_t(v);
            const uint64_t bal = __ballot(sel);
            const uint32_t before = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wave_cnt[wave] = __popcll(bal);
            __syncthreads();
            uint32_t woff = 0, tot = 0;
            for (uint32_t w = 0; w < 4; ++w) {
                woff += w < wave ? wave_cnt[w] : 0;
                tot += wave_cnt[w];
            }
            const uint32_t rank = taken + woff + before;
            if (sel && rank < limit) cand[pos + rank] = uint32_t(i - lo);
            taken += tot;
            __syncthreads();
        }
        pos += limit;
    }
}

__global__ void k_copy_u64(const uint64_t *__restrict__ a, uint64_t *__restrict__ b, uint64_t n)
{
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}

uint32_t rz_blocks(const hough_ctx *c)
{
    const uint32_t w = c->tun.rz_waves_per_cu ? c->tun.rz_waves_per_cu : 4;
    return uint32_t(c->n_cu) * w;
}

hipError_t launch_rz(hough_ctx *c, const hough_hits *h, const hough_peak *peaks, uint64_t peak_capacity,
                     const uint64_t *poff, hough_rz *out, uint64_t capacity, uint64_t *roff, hipStream_t s)
{
    hipError_t err;
    const hough_grid_spec &g = c->spec;
    const uint32_t E = h->n_events;
    if ((err = launch_bucket_layers(c, h, true, s)) != hipSuccess) return err;
    if ((err = launch_bucket_phi(c, h, s)) != hipSuccess) return err;
    KernelTimer t;
    prof_begin(c, "rz_counts", s, &t);
    hipLaunchKernelGGL(k_rz_counts, dim3((E + 255) / 256), dim3(256), 0, s, poff, peak_capacity, E,
                       g.rz_max_candidates, c->d_cand_counts);
    prof_end(c, s, &t);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_scan_counts(c, c->d_cand_counts, E, c->d_tile_off, 1, roff, s)) != hipSuccess)
        return err;
    if (g.rz_max_candidates) {
        prof_begin(c, "rz_select", s, &t);
        hipLaunchKernelGGL(k_rz_select, dim3(E), dim3(256), 0, s,
                           reinterpret_cast<const uint2 *>(peaks), peak_capacity, poff, roff,
                           g.rz_max_candidates, c->d_cand);
        prof_end(c, s, &t);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if ((err = launch_fill_u32(c, c->d_counters + 1, 0, 1, s)) != hipSuccess) return err;

    RzParams P;
    P.phi = c->d_phi_b;
    P.z = c->d_z_b;
    P.offs = h->event_offsets;
    P.n_hits = h->n_hits;
    P.bucket_off = c->d_bucket_off;
    P.O = c->d_O;
    P.V = c->d_V;
    P.Z = c->d_Z;
    P.peaks = reinterpret_cast<const uint2 *>(peaks);
    P.peak_capacity = peak_capacity;
    P.poff = poff;
    P.roff = roff;
    P.cand = c->d_cand;
    P.out4 = reinterpret_cast<uint2 *>(out);
    P.out_capacity = capacity;
    P.counter = c->d_counters + 1;
    P.gscratch = c->d_rz_hist;
    P.n_events = E;
    P.n_layers = g.n_layers;
    P.n_qpt = g.n_qpt;
    P.rows = c->rows;
    P.nphi = g.n_phi;
    P.log2phi = c->log2_phi;
    P.shift = c->shift;
    P.bucket_bits = c->bucket_bits;
    P.n_z0 = g.n_z0;
    P.n_cot = g.n_cot;
    P.cap = g.rz_max_candidates;
    P.z0_lo = g.z0_lo_um;
    P.span = uint64_t(int64_t(g.z0_hi_um) - int64_t(g.z0_lo_um));
    P.use32 = P.span * g.n_z0 < (uint64_t(1) << 32);
    P.fd = make_fastdiv32(P.use32 ? uint32_t(P.span) : 1u);
    const size_t lds = size_t(g.n_z0) * 64 * sizeof(uint16_t);
    P.lds_ok = lds <= c->max_lds && !c->tun.rz_slow_path;
    prof_begin(c, "rz_vote", s, &t);
    hipLaunchKernelGGL(k_rz_vote, dim3(rz_blocks(c)), dim3(64), P.lds_ok ? lds : 0, s, P);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
