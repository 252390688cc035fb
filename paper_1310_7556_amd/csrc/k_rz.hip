// rz refinement of candidate cells: the "more expensive computations to
// confirm" that Section 4 leaves to follow the local-maximum search.
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
// lane owns cot bins j = lane, lane + 64, ... and a private column of z0
// counters in LDS; its running maximum is exact because counts only grow.
//
// k_rz_vote_fast (used when the spec allows exact 32-bit arithmetic):
//   1. lanes 0..L-1 each find their layer's window of azimuth buckets; a
//      wave prefix over window lengths flattens all layers' scanned hits,
//      and one ballot-compacted pass copies the members' z (grouped by layer)
//      into LDS;
//   2. per pass of 64 cot bins (one per lane), the members that can vote in
//      range are compacted again; per member: u = z - (Z + z0_lo) in
//      uint32, bin by one multiply-high (BinMagic, no shift where that is
//      exact), which maps every u >= span past the last bin into a trash
//      counter, and an LDS atomic add on a lane-private packed counter (4-,
//      8- or 16-bit) whose return value gives the running count without a
//      read-modify-write chain;
//   3. the counters are cleared wholesale with 16-byte stores.  A pass with
//      at most 12 members skips 2 and 3: each lane sorts its bins in
//      registers with a sorting network and takes the longest run.
// A candidate with more members than the LDS list holds, or whose 4- or
// 8-bit counter overflowed, is marked in its record and recomputed by
// k_rz_redo on the exact slow path: a uint32 histogram in global scratch,
// one cot bin at a time.  k_rz_vote is the general kernel (64-bit
// arithmetic) for specs outside the fast path's range conditions.
#include <type_traits>

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
    const int32_t *Zl;            // [K][C][16] = Z + z0_lo, 0 past n_layers (fast path)
    const uint2 *peaks;
    uint64_t peak_capacity;
    const uint64_t *poff;         // [E + 1]
    const uint64_t *roff;         // [E + 1]
    const uint32_t *cand;         // selected local peak indices (cap > 0)
    uint2 *out4;                  // hough_rz records as 4 x uint32 (2 x uint2)
    uint64_t out_capacity;
    uint32_t *counter;            // the work counter (general kernel); queue q's at counter[q * kRzQueueStride] (fast)
    uint32_t n_queues;            // fast kernel: work queues, 1 .. kRzQueues
    uint32_t *redo_count;         // records marked for the exact path
    uint64_t *redo_list;          // their indices, the first redo_cap of them
    uint32_t redo_cap;
    uint32_t *gscratch;           // [blocks][n_z0] zeroed uint32, slow path
    uint32_t n_events, n_layers, n_qpt, rows, nphi, log2phi, shift, bucket_bits;
    uint32_t n_z0, n_cot, cap;
    int64_t z0_lo;
    uint64_t span;                // z0_hi - z0_lo
    int use32;                    // span * n_z0 < 2^32: fast 32-bit division
    FastDiv32 fd;
    int lds_ok;                   // general kernel: the uint16 histogram fits in LDS
    uint32_t bm, bs;              // fast path: bin = mulhi(u, bm) >> bs
    uint32_t span24;              // MUL == 2: span (< 2^24, with bm < 2^24 and bs == 0)
    uint32_t redo_lds;            // k_rz_redo has LDS for kRedoMembers members and an n_z0 histogram
    uint32_t hw;                  // fast path: counter dwords per lane
    uint32_t mcap;                // fast path: member list capacity
};

// The fast kernel's work queues: the candidates are split into kRzQueues
// contiguous ranges, one per XCD, each with its own counter (kRzQueueStride
// dwords apart, in different cache lines); a wave starts on the queue of
// the XCD it runs on (read from the hardware, as the XCD a workgroup lands
// on depends on what else runs), so that an XCD's waves share a range:
// neighbouring cells, whose members and tables are the same cache lines in
// that XCD's L2.  A wave takes kRzChunk consecutive candidates per ticket
// and, when its queue is empty, moves on to the next queue (each empty
// queue costs the wave one ticket, so short record lists -- a micro-batch --
// use one queue).  (1000-track event: 0.96 ms with 8 queues of 8-candidate tickets;
// 1.00 ms with one queue, 0.99 and 0.98 ms with tickets of 4 and 16, 1.04
// and 1.17 ms with 32 and 64 queues.)
constexpr uint32_t kRzQueues = 8;
constexpr uint32_t kRzQueueStride = 32;
constexpr uint32_t kRzChunk = 8;
// Passes with at most kRzSortMax members are counted by sorting each lane's
// bins with a sorting network, 8 or 12 inputs: 19 and 39 comparators (both
// minimal in size; each checked on every 0-1 input, which by the 0-1
// principle shows that it sorts every input; so are their restrictions to
// fewer inputs, the rest held above every value).  Where most passes have 12
// members or fewer (the 1000-track event: 76%, a third 8 or fewer) this
// replaces most counter atomics and clears: rz 0.95 -> 0.89 ms (0.92 with
// 8-input sorts only; 0.91 with a 16-input network added for up to 16).
constexpr uint32_t kRzSortMax = 12;
constexpr int kSortNet8Size = 19;
constexpr int kSortNet12Size = 39;
__device__ constexpr uint8_t kSortNet8[19][2] = {
    {0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
    {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
__device__ constexpr uint8_t kSortNet12[39][2] = {
    {0, 8}, {1, 7}, {2, 6}, {3, 11}, {4, 10}, {5, 9}, {0, 1}, {2, 5}, {3, 4}, {6, 9},
    {7, 8}, {10, 11}, {0, 2}, {1, 6}, {5, 10}, {9, 11}, {0, 3}, {1, 2}, {4, 6}, {5, 7},
    {8, 11}, {9, 10}, {1, 4}, {3, 5}, {6, 8}, {7, 10}, {1, 3}, {2, 5}, {6, 9}, {8, 10},
    {2, 3}, {4, 5}, {6, 7}, {8, 9}, {4, 6}, {5, 7}, {3, 4}, {5, 6}, {7, 8}};
// the rz counters in the context's counter array: from dword kRzCounterBase,
// the queues' counters, then the marked-record count
constexpr uint32_t kRzCounterBase = 32;
constexpr uint32_t kRzRedoCountAt = kRzQueues * kRzQueueStride;
constexpr uint32_t kRzCounterDwords = kRzRedoCountAt + 1;
static_assert(kRzCounterBase + kRzCounterDwords <= kCounterDwords, "rz counters fit the counter array");

// count field of a record that k_rz_vote_fast leaves to k_rz_redo
constexpr uint32_t kRzRedo = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The XCD (accelerator complex die) the wave runs on: the hardware register
// XCC_ID, bits 0..3.
__device__ __forceinline__ uint32_t xcd_id()
{
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
}

// a dword in LDS, addressed by its 32-bit LDS address
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// floor(a * b / 2^32) of the low 24 bits of a and b, one full-rate
// instruction.  Written as an instruction of its own so that the compiler
// keeps the product's high word and derives the counter address from it,
// instead of recomputing the address from a second, low-word multiply.
__device__ __forceinline__ uint32_t mulhi_u24(uint32_t a_uniform, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(r) : "s"(a_uniform), "v"(b));
    return r;
#else
    return uint32_t((uint64_t(a_uniform & 0xFFFFFFu) * (b & 0xFFFFFFu)) >> 32);
#endif
}

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

// Slow path for one candidate: one cot bin at a time, lanes stride over the
// members, counts in a zeroed uint32 histogram g[n_z0] in global scratch
// (left zeroed on return).  Results are wave-uniform.
__device__ void rz_slow(const RzParams &P, uint64_t eb, const uint32_t *bo, uint32_t k, uint32_t p,
                        uint32_t mask, uint32_t *g, uint32_t lane, uint32_t &best_c, uint32_t &best_j,
                        uint32_t &best_b)
{
    best_c = 0;
    best_j = 0;
    best_b = 0;
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
            // every lane's updates of this pass are complete and visible
            // before any lane starts the next pass
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
}

// Wave argmax of (count desc, cot asc, z0 asc) over the lanes' bests, then
// every lane stores the (uniform) record of candidate c.
// Maximum of x over the wave's 64 lanes (all active), uniform: DPP swaps
// within quads, rotates within rows of 16, then the last lane of each row
// broadcast into the next rows.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x)
{
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0xB1, 0xF, 0xF, false)));   // quad_perm 1,0,3,2
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x4E, 0xF, 0xF, false)));   // quad_perm 2,3,0,1
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x124, 0xF, 0xF, false)));  // row_ror:4
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x128, 0xF, 0xF, false)));  // row_ror:8
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x142, 0xA, 0xF, false)));  // row_bcast:15
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(int(x), int(x), 0x143, 0xC, 0xF, false)));  // row_bcast:31
    return uint32_t(__builtin_amdgcn_readlane(int(x), 63));
}

__device__ __forceinline__ void rz_finish(const RzParams &P, uint64_t c, uint32_t pk, uint32_t nm,
                                          uint32_t best_c, uint32_t best_j, uint32_t best_b)
{
    // the largest count, then among the lanes holding it the smallest cot
    // bin and then the smallest z0 bin (as one 32-bit key)
    const uint32_t cnt = wave_max_u32(best_c);
    const uint32_t key = best_c == cnt ? ((0xFFFFu - (best_j & 0xFFFFu)) << 16) | (0xFFFFu - (best_b & 0xFFFFu)) : 0u;
    const uint32_t kmax = wave_max_u32(key);
    const uint32_t jj = 0xFFFFu - (kmax >> 16);
    const uint32_t bb = 0xFFFFu - (kmax & 0xFFFFu);
    uint2 a, b;
    a.x = pk;
    a.y = (cnt ? jj : 0u) | ((cnt ? bb : 0u) << 16);
    b.x = cnt;
    b.y = nm;
    P.out4[2 * c] = a;
    P.out4[2 * c + 1] = b;
}

// Decoded candidate c: its event, local peak index, cell and event base.
struct RzCand {
    uint32_t e, pk, mask, k, p;
    uint64_t eb;
    const uint32_t *bo;
};

// Peak record of candidate c (event search, candidate index, record load).
__device__ __forceinline__ uint2 rz_record(const RzParams &P, uint64_t c)
{
    uint32_t lo = 0, hi = P.n_events;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (P.roff[mid] <= c) lo = mid; else hi = mid;
    }
    const uint32_t e = uni(lo);
    const uint32_t pk = P.cap ? uni(P.cand[c]) : uni(uint32_t(c - P.roff[e]));
    return P.peaks[uni64(P.poff[e] + pk)];
}

// rz_decode with the peak record already fetched.
__device__ __forceinline__ RzCand rz_decode_rec(const RzParams &P, uint64_t c, uint2 rec)
{
    RzCand r;
    const uint32_t nb = 1u << P.bucket_bits;
    uint32_t lo = 0, hi = P.n_events;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (P.roff[mid] <= c) lo = mid; else hi = mid;
    }
    r.e = uni(lo);
    const uint32_t local = uni(uint32_t(c - P.roff[r.e]));
    r.pk = P.cap ? uni(P.cand[c]) : local;
    const uint32_t cell = uni(rec.x);
    r.mask = uni(rec.y & 0xFFFFu);
    r.k = (cell >> P.log2phi) % P.n_qpt;
    r.p = cell & (P.nphi - 1);
    r.eb = uni64(min(P.offs[r.e], P.n_hits));
    r.bo = P.bucket_off + size_t(r.e) * P.n_layers * (nb + 1);
    return r;
}

__device__ __forceinline__ RzCand rz_decode(const RzParams &P, uint64_t c)
{
    RzCand r;
    const uint32_t nb = 1u << P.bucket_bits;
    // event of candidate c: largest e with roff[e] <= c
    uint32_t lo = 0, hi = P.n_events;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (P.roff[mid] <= c) lo = mid; else hi = mid;
    }
    r.e = uni(lo);
    const uint32_t local = uni(uint32_t(c - P.roff[r.e]));
    r.pk = P.cap ? uni(P.cand[c]) : local;
    const uint64_t gp = uni64(P.poff[r.e] + r.pk);
    const uint2 rec = P.peaks[gp];
    const uint32_t cell = uni(rec.x);
    r.mask = uni(rec.y & 0xFFFFu);
    r.k = (cell >> P.log2phi) % P.n_qpt;
    r.p = cell & (P.nphi - 1);
    r.eb = uni64(min(P.offs[r.e], P.n_hits));
    r.bo = P.bucket_off + size_t(r.e) * P.n_layers * (nb + 1);
    return r;
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
    for (;;) {
        // Work fetch without lane-divergent control flow: every lane executes
        // the atomic (only lane 0 adds 1) and lane 0's ticket is broadcast by
        // readfirstlane.  A fetch guarded by "if (lane == 0)" followed by a
        // cross-lane read assumes the wave reconverges at the loop head, which
        // the compiler does not guarantee (it may keep lanes 1..63 cycling in
        // an inner loop that never re-reads the counter).
        const uint64_t c = uni(atomicAdd(P.counter, lane == 0 ? 1u : 0u));
        if (c >= total) break;
        const RzCand r = rz_decode(P, c);
        const uint32_t k = r.k, p = r.p, mask = r.mask;

        uint32_t nm = 0;
        for_members(P, r.eb, r.bo, k, p, mask, [&](uint32_t, uint32_t) { ++nm; });

        uint32_t best_c = 0, best_j = lane, best_b = 0;     // lane's best over its cot bins
        if (P.lds_ok && nm <= 65535u) {
            for (uint32_t j0 = 0; j0 < P.n_cot; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool jv = j < P.n_cot;
                uint32_t bc = 0, bb = 0;
                for_members(P, r.eb, r.bo, k, p, mask, [&](uint32_t h, uint32_t l) {
                    if (!jv) return;
                    const int64_t zl = int64_t(P.Z[(size_t(k) * P.n_layers + l) * P.n_cot + j]) + P.z0_lo;
                    const int32_t b = z0_bin(P, P.z[r.eb + h], zl);
                    if (b < 0) return;
                    const uint32_t idx = uint32_t(b) * 64 + lane;
                    const uint32_t cnt = uint32_t(hist[idx]) + 1;
                    hist[idx] = uint16_t(cnt);
                    if (cnt > bc || (cnt == bc && uint32_t(b) < bb)) { bc = cnt; bb = uint32_t(b); }
                });
                for_members(P, r.eb, r.bo, k, p, mask, [&](uint32_t h, uint32_t l) {
                    if (!jv) return;
                    const int64_t zl = int64_t(P.Z[(size_t(k) * P.n_layers + l) * P.n_cot + j]) + P.z0_lo;
                    const int32_t b = z0_bin(P, P.z[r.eb + h], zl);
                    if (b >= 0) hist[uint32_t(b) * 64 + lane] = 0;
                });
                if (jv && bc > best_c) { best_c = bc; best_j = j; best_b = bb; }
            }
        } else {
            rz_slow(P, r.eb, r.bo, k, p, mask, g, lane, best_c, best_j, best_b);
            if (lane != 0) { best_c = 0; best_j = 0xFFFFu; best_b = 0; }
        }
        rz_finish(P, c, r.pk, nm, best_c, best_j, best_b);
    }
}

// LDS layout of the fast kernel, in dwords: counters, the layer windows,
// the pass boundary table, then two member lists (all members of the
// candidate; those of the current pass), each z values then layer bytes for
// mcap members and 8 spare slots, 16-byte aligned.
__host__ __device__ inline uint32_t rz_list_z_dwords(uint32_t mcap) { return (mcap + 8 + 3) & ~3u; }
__host__ __device__ inline uint32_t rz_list_dwords(uint32_t mcap)
{
    return rz_list_z_dwords(mcap) + ((((mcap + 8 + 3) / 4) + 3) & ~3u);
}
__host__ __device__ inline uint32_t rz_fast_lds_dwords(uint32_t hw, uint32_t mcap)
{
    return hw * 64 + 96 + 32 + 2 * rz_list_dwords(mcap);
}

// MUL: how the bin is found from u = z - (Z + z0_lo): 0 = min(mulhi(u, bm),
// n_z0); 1 = the same with the extra right shift bs; 2 = mulhi24(min(u,
// span), bm), two full-rate operations where the 32-bit multiply-high is
// quarter rate: when span and bm are below 2^24 (and bs == 0) the 24-bit
// multiply-high is exact, min(u, span) keeps every in-range u and maps the
// others to span, and floor(span * bm / 2^32) is exactly n_z0 (bm =
// ceil(n_z0 2^32 / span) and span < 2^32), the trash bin.
template <int BITS, int MUL>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))   // <= 128 VGPRs
k_rz_vote_fast(RzParams P)
{
    constexpr uint32_t PACK = 32 / BITS;           // counters per dword
    constexpr uint32_t PSH = BITS == 4 ? 3 : BITS == 8 ? 2 : 1;    // log2(PACK)
    constexpr uint32_t BSH = BITS == 4 ? 2 : BITS == 8 ? 3 : 4;    // log2(BITS)
    constexpr uint32_t FIELD = (1u << BITS) - 1u;
    static_assert(PACK == (1u << PSH) && BITS == (1u << BSH), "counter layout");
    HOUGH_DYNAMIC_LDS(uint32_t, lds);
    const uint32_t lane = threadIdx.x;
    uint32_t *hist = lds;                            // [hw][64] lane-private packed counters
    uint32_t *lay = hist + P.hw * 64;                // [5][16] per-layer windows
    int32_t *tb = reinterpret_cast<int32_t *>(lay + 96);     // [2][16] pass boundaries per layer
    int32_t *mz = tb + 32;                                   // [mcap] member z
    uint8_t *ml = reinterpret_cast<uint8_t *>(mz + rz_list_z_dwords(P.mcap));   // member layer
    int32_t *mzc = mz + rz_list_dwords(P.mcap);              // this pass's members: z
    uint8_t *mlc = reinterpret_cast<uint8_t *>(mzc + rz_list_z_dwords(P.mcap));  // and layer
    // 16-bit counters cannot overflow below FIELD members; 4- and 8-bit
    // counters detect an overflow instead and send the candidate to the
    // exact slow path
    const uint32_t lim = BITS <= 8 ? P.mcap : min(P.mcap, FIELD);
    const uint32_t nb = 1u << P.bucket_bits, bsh = 32 - P.bucket_bits;
    const uint32_t nl = P.n_layers;
    const uint64_t total = min(P.roff[P.n_events], P.out_capacity);
    for (uint32_t i = lane; i < P.hw * 64; i += 64) hist[i] = 0;
    __syncthreads();
    const uint32_t nq = P.n_queues, q0 = xcd_id();
    for (uint32_t qi = 0; qi < nq; ++qi) {
      const uint32_t q = (q0 + qi) % nq;
      const uint64_t qb = total * q / nq, qe = total * (q + 1) / nq;
      uint32_t *qc = P.counter + q * kRzQueueStride;
      for (;;) {
        const uint64_t c0 = qb + uni(atomicAdd(qc, lane == 0 ? kRzChunk : 0u));
        if (c0 >= qe) break;
        const uint64_t c1 = min(c0 + kRzChunk, qe);
        // the next candidate's peak record is fetched while the current one
        // is processed, so its latency overlaps the current loads
        uint2 nrec = rz_record(P, c0);
      for (uint64_t c = c0; c < c1; ++c) {
        const uint2 rec = nrec;
        if (c + 1 < c1) nrec = rz_record(P, c + 1);
        const RzCand r = rz_decode_rec(P, c, rec);
        const uint32_t k = r.k, p = r.p;
        // all layers' (Z + z0_lo) for this lane's first cot bin, issued now
        // so that they arrive with the member search's loads: the table is
        // [k][cot][16 layers], so they are 64 contiguous bytes (4 loads; a
        // lane past the last cot bin reads the last one).  Layers >=
        // n_layers hold 0.
        const int32_t *zrow = P.Zl + size_t(k) * P.n_cot * kMaxLayers;
        uint32_t zr[kMaxLayers], zn[kMaxLayers];
        auto load_rows = [&](uint32_t jj, uint32_t (&zz)[kMaxLayers]) {
            const uint4 *q = reinterpret_cast<const uint4 *>(zrow + size_t(min(jj, P.n_cot - 1)) * kMaxLayers);
#pragma unroll
            for (uint32_t g = 0; g < kMaxLayers / 4; ++g) {
                const uint4 v = q[g];
                zz[4 * g] = v.x;
                zz[4 * g + 1] = v.y;
                zz[4 * g + 2] = v.z;
                zz[4 * g + 3] = v.w;
            }
        };
        load_rows(lane, zr);
        // the first pass's boundary values: lanes 0..15 read layer `lane` at
        // its first cot bin, lanes 16..31 layer `lane - 16` at its last
        auto boundary = [&](uint32_t jp) {
            const uint32_t jb = lane < 16 ? jp : jp + 63u;
            return zrow[size_t(min(jb, P.n_cot - 1)) * kMaxLayers + (lane & 15u)];
        };
        int32_t tbv = boundary(0);

        // 1a. lane l < L: the azimuth-bucket window of layer l (one or two
        // ranges of the (layer, bucket)-sorted hits, two when it wraps)
        uint32_t len1 = 0, len2 = 0, hs1 = 0, hs2 = 0, o = 0;
        if (lane < nl && ((r.mask >> lane) & 1u)) {
            const size_t ti = size_t(lane) * P.rows + k;
            if (P.V[ti]) {
                o = P.O[ti];
                const uint32_t start = o + (p << P.shift);
                const uint32_t b0 = start >> bsh;
                const uint64_t W = uint64_t(1) << P.shift, BW = uint64_t(1) << bsh;
                const uint32_t nbk = min(uint32_t(((uint64_t(start) & (BW - 1)) + W - 1) / BW + 1), nb);
                const uint32_t *bl = r.bo + size_t(lane) * (nb + 1);
                const uint32_t e1 = b0 + nbk;
                hs1 = bl[b0];
                if (e1 <= nb) {
                    len1 = bl[e1] - hs1;
                } else {
                    len1 = bl[nb] - hs1;
                    hs2 = bl[0];
                    len2 = bl[e1 - nb] - hs2;
                }
            }
        }
        // 1b. exclusive prefix of window lengths across the layer lanes:
        // they are lanes 0..15 (L <= 15 here; the other lanes hold 0), one
        // DPP row, scanned with row shifts by 1, 2, 4 and 8 lanes (a lane
        // shifted in from before the row start reads 0)
        const uint32_t len = len1 + len2;
        uint32_t incl = len;
        incl += uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x111, 0xF, 0xF, false));   // row_shr:1
        incl += uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x112, 0xF, 0xF, false));   // row_shr:2
        incl += uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x114, 0xF, 0xF, false));   // row_shr:4
        incl += uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x118, 0xF, 0xF, false));   // row_shr:8
        const uint32_t T = uint32_t(__builtin_amdgcn_readlane(int(incl), 15));
        if (lane < 16) {
            lay[lane] = incl - len;
            lay[16 + lane] = len1;
            lay[32 + lane] = hs1;
            lay[48 + lane] = hs2;
            lay[64 + lane] = o;
        }
        __syncthreads();
        // 1c. one pass over all scanned hits, ballot-compacting the members
        // (their order is layer, then hit, so each layer's members are a run)
        uint32_t nm = 0;
        for (uint32_t g0 = 0; g0 < T; g0 += 64) {
            const uint32_t gi = g0 + lane;
            bool is_m = false;
            int32_t zv = 0;
            uint32_t ls = 0;
            if (gi < T) {
                // the hit's layer: the last window starting at or before gi
                // (starts are non-decreasing; lanes nl..15 hold T)
#pragma unroll
                for (uint32_t s = 8; s > 0; s >>= 1) ls += lay[ls + s] <= gi ? s : 0u;
                const uint32_t local = gi - lay[ls];
                const uint32_t l1 = lay[16 + ls];
                const uint32_t h = local < l1 ? lay[32 + ls] + local : lay[48 + ls] + (local - l1);
                // z is loaded with phi (not after the test) to save a round trip
                const uint32_t ph = P.phi[r.eb + h];
                const int32_t zh = P.z[r.eb + h];
                is_m = ((ph - lay[64 + ls]) >> P.shift) == p;
                zv = is_m ? zh : 0;
            }
            const uint64_t bal = __ballot(is_m);
            const uint32_t pos = nm + __popcll(bal & ((1ull << lane) - 1ull));
            if (is_m && pos < lim) {
                mz[pos] = zv;
                ml[pos] = uint8_t(ls);
            }
            nm += __popcll(bal);
        }
        __syncthreads();

        uint32_t best_c = 0, best_j = lane, best_b = 0;
        bool ovf = false;                  // a 4- or 8-bit counter of a real bin overflowed
        if (nm <= lim) {
            // One 64-cot pass: zc holds this pass's (Z + z0_lo) rows and zx
            // receives the next pass's, loaded while this one counts (one
            // memory latency per candidate, not per pass); consecutive passes
            // swap the two sets instead of copying.
            auto pass = [&](uint32_t j0, uint32_t (&zc)[kMaxLayers], uint32_t (&zx)[kMaxLayers]) {
                const uint32_t j = j0 + lane;
                const bool jv = j < P.n_cot;
                // Members of this pass.  (Z + z0_lo) is monotone in the cot
                // bin (cot_j is linear in j, the arc length is positive and
                // rounding keeps the order), so over the pass's cot bins
                // [ja, jb] it lies between its values at ja and jb, and a
                // member can vote in range only if min <= z and z - max <
                // span; every vote of the others would go to the trash
                // counter, so they are left out of the pass (the result is
                // unchanged).
                if (lane < 32) tb[lane] = tbv;
                __syncthreads();
                tbv = boundary(j0 + 64);             // next pass's, in flight meanwhile
                uint32_t nq = 0;
                for (uint32_t c0 = 0; c0 < nm; c0 += 64) {
                    const uint32_t m = c0 + lane;
                    bool act = false;
                    int32_t zm = 0;
                    uint32_t lm = 0;
                    if (m < nm) {
                        zm = mz[m];
                        lm = ml[m];
                        const int32_t za = tb[lm], zb = tb[16 + lm];
                        const int32_t mx = max(za, zb);
                        // z - max < span as integers: true when z < max, else
                        // the 32-bit difference is exact
                        act = zm >= min(za, zb) && (zm < mx || uint64_t(uint32_t(zm - mx)) < P.span);
                    }
                    const uint64_t bal = __ballot(act);
                    const uint32_t pos = nq + __popcll(bal & ((1ull << lane) - 1ull));
                    if (act) {
                        mzc[pos] = zm;
                        mlc[pos] = uint8_t(lm);
                    }
                    nq += __popcll(bal);
                }
                __syncthreads();
                // next pass's rows (after the last pass they are loaded and
                // not used: the index is clamped, so the loads stay in bounds)
                load_rows(j + 64, zx);
                // The members in one flat loop, eight per step, then steps of
                // four, two and one for the rest: 16-byte LDS reads give four
                // z each, 4-byte reads their layers (so (Z + z0_lo) is a
                // register-indexed move).  Per member: the bin b of u = z -
                // (Z + z0_lo) from the multiply-high -- every u >= span (out
                // of range, or a lane past the last cot bin whose result is
                // dropped) maps to n_z0 or above, so those votes land in a
                // trash counter past the last bin -- then the lane-private
                // packed counter atomic and the running maximum of the signed
                // key (count - 1) * 2^16 - b over in-range votes (largest
                // count wins, ties to the smallest bin)
                const uint4 *mz4 = reinterpret_cast<const uint4 *>(mzc);
                const uint32_t *ml4 = reinterpret_cast<const uint32_t *>(mlc);
                // this lane's counter column (row stride 64 dwords): the LDS
                // address of counter dword (b >> PSH) is colb + (b >> PSH) *
                // 256, a bit-field extract and a shift-add (written out, as
                // the compiler otherwise takes three instructions)
                const uint32_t colb = uint32_t(reinterpret_cast<uintptr_t>((lds_u32 *)(hist + lane)));
                auto counter_at = [&](uint32_t bq) {
                    uint32_t a;
#if defined(__HIP_DEVICE_COMPILE__)
                    asm("v_bfe_u32 %0, %1, %2, %3\n\tv_lshl_add_u32 %0, %0, 8, %4"
                        : "=&v"(a) : "v"(bq), "i"(PSH), "i"(32 - PSH), "v"(colb));
#else
                    a = colb + ((bq >> PSH) << 8);
#endif
                    return reinterpret_cast<lds_u32 *>(uintptr_t(a));
                };
                int32_t run = INT32_MIN;
                // Q members per step, starting at member m (a multiple of Q)
                auto step = [&](auto qc, uint32_t m) {
                    constexpr int Q = decltype(qc)::value;
                    uint32_t zm[Q], lq[Q];
                    if constexpr (Q >= 4) {
#pragma unroll
                        for (int g = 0; g < Q / 4; ++g) {
                            const uint4 z4 = mz4[(m >> 2) + g];
                            zm[4 * g] = z4.x;
                            zm[4 * g + 1] = z4.y;
                            zm[4 * g + 2] = z4.z;
                            zm[4 * g + 3] = z4.w;
                            const uint32_t lw = uni(ml4[(m >> 2) + g]);
#pragma unroll
                            for (int i = 0; i < 4; ++i) lq[4 * g + i] = (lw >> (8 * i)) & 0xFFu;
                        }
                    } else if constexpr (Q == 2) {
                        const uint2 z2 = reinterpret_cast<const uint2 *>(mzc)[m >> 1];
                        zm[0] = z2.x;
                        zm[1] = z2.y;
                        const uint32_t lw = uni(ml4[m >> 2]) >> (8 * (m & 3u));
                        lq[0] = lw & 0xFFu;
                        lq[1] = (lw >> 8) & 0xFFu;
                    } else {
                        zm[0] = uint32_t(mzc[m]);
                        lq[0] = uni(uint32_t(mlc[m]));
                    }
                    uint32_t b[Q], sh[Q], old[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const uint32_t u = zm[q] - zc[lq[q]];
                        if (MUL == 2) {
                            // both factors below 2^24: the 24-bit multiply-high
                            b[q] = mulhi_u24(P.bm, min(u, P.span24));
                        } else {
                            uint32_t t = __umulhi(u, P.bm);
                            if (MUL == 1) t >>= P.bs;
                            b[q] = min(t, P.n_z0);
                        }
                        sh[q] = b[q] << BSH;   // field offset, taken mod 32
                    }
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        // counter dword (b >> PSH) of this lane's column
                        old[q] = __hip_atomic_fetch_add(counter_at(b[q]), 1u << (sh[q] & 31u), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const uint32_t field = __builtin_amdgcn_ubfe(old[q], sh[q], BITS);
                        const int32_t key = int32_t(field << 16) - int32_t(b[q]);
                        run = b[q] < P.n_z0 ? max(run, key) : run;
                    }
                };
                // Passes of at most kRzSortMax members: the lane's bins are
                // sorted in registers (the members past nq go to the trash
                // bin, which sorts last) and the longest run of an in-range
                // bin found in one sweep -- the first in bin order among the
                // longest, as the counters give -- so the counters are
                // neither touched nor cleared.
                uint32_t bc = 0, bb = 0;
                // M (= nq, a constant of the instance) members: the inputs
                // past M are constants above every bin, so the compiler
                // drops the comparators and sweep steps they would take part
                // in (the 8- or 12-input network restricted to M inputs:
                // 5, 9, 12, 16, 19, 26, 30, 35, 39 comparators for M = 4..12)
                auto sorted_pass = [&](auto mc) {
                    constexpr int M = decltype(mc)::value;
                    constexpr int N = M <= 8 ? 8 : 12;
                    uint32_t v[N];
#pragma unroll
                    for (int q = M; q < N; ++q) v[q] = 0xFFFFFFFFu;
#pragma unroll
                    for (int g = 0; g < (M + 3) / 4; ++g) {
                        const uint4 z4 = mz4[g];
                        const uint32_t lw = uni(ml4[g]);
                        const uint32_t zq[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
                        for (int i = 0; i < 4 && 4 * g + i < M; ++i) {
                            const uint32_t u = zq[i] - zc[(lw >> (8 * i)) & 0xFFu];
                            if (MUL == 2) {
                                v[4 * g + i] = mulhi_u24(P.bm, min(u, P.span24));
                            } else {
                                uint32_t t = __umulhi(u, P.bm);
                                if (MUL == 1) t >>= P.bs;
                                v[4 * g + i] = min(t, P.n_z0);
                            }
                        }
                    }
                    // the sorting network, ascending
                    const auto &net = N == 8 ? kSortNet8 : kSortNet12;
                    constexpr int NC = N == 8 ? kSortNet8Size : kSortNet12Size;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const uint32_t a = v[net[c][0]], b2 = v[net[c][1]];
                        v[net[c][0]] = min(a, b2);
                        v[net[c][1]] = max(a, b2);
                    }
                    uint32_t cnt = 1;
                    if (v[0] < P.n_z0) {
                        bc = 1;
                        bb = v[0];
                    }
#pragma unroll
                    for (int i = 1; i < M; ++i) {
                        cnt = v[i] == v[i - 1] ? cnt + 1 : 1u;
                        if (v[i] < P.n_z0 && cnt > bc) {
                            bc = cnt;
                            bb = v[i];
                        }
                    }
                };
                const bool sorted = nq <= kRzSortMax;
                if (sorted) {
                    using std::integral_constant;
                    switch (nq) {
                    case 0: break;
                    case 1: sorted_pass(integral_constant<int, 1>{}); break;
                    case 2: sorted_pass(integral_constant<int, 2>{}); break;
                    case 3: sorted_pass(integral_constant<int, 3>{}); break;
                    case 4: sorted_pass(integral_constant<int, 4>{}); break;
                    case 5: sorted_pass(integral_constant<int, 5>{}); break;
                    case 6: sorted_pass(integral_constant<int, 6>{}); break;
                    case 7: sorted_pass(integral_constant<int, 7>{}); break;
                    case 8: sorted_pass(integral_constant<int, 8>{}); break;
                    case 9: sorted_pass(integral_constant<int, 9>{}); break;
                    case 10: sorted_pass(integral_constant<int, 10>{}); break;
                    case 11: sorted_pass(integral_constant<int, 11>{}); break;
                    default: sorted_pass(integral_constant<int, 12>{}); break;
                    }
                } else {
                    uint32_t m = 0;
                    for (; m + 8 <= nq; m += 8) step(std::integral_constant<int, 8>{}, m);
                    if (m + 4 <= nq) {
                        step(std::integral_constant<int, 4>{}, m);
                        m += 4;
                    }
                    if (m + 2 <= nq) {
                        step(std::integral_constant<int, 2>{}, m);
                        m += 2;
                    }
                    if (m < nq) step(std::integral_constant<int, 1>{}, m);
                    const int32_t fld = (run + 0xFFFF) >> 16;
                    bc = run == INT32_MIN ? 0u : uint32_t(fld) + 1u;
                    bb = uint32_t((fld << 16) - run);
                    // a count of FIELD + 1 can only come from a vote that
                    // found its field full: the counter overflowed
                    if (BITS <= 8) ovf = ovf || bc > FIELD;
                }
                // clear the counters, 16 bytes per lane per store; a store
                // covers other lanes' columns, so every lane's counting must
                // be finished first and the clear finished before the next
                // cot bins are counted (nothing to clear after an empty pass).
                // The clear bounds the kernel (8 KB per pass through the LDS,
                // 0.15 ms of the 1000-track event's 0.96 ms), so a trash bin
                // alone in the last counter dword is left as it is: its count
                // is never read.  (Zeroing just the dwords the votes went to,
                // the members' bins recomputed, costs more: 1.01 ms.)
                if (!sorted) {
                    __syncthreads();
                    // full rounds of 64 16-byte stores at fixed offsets from
                    // one address, then the partial last round
                    uint4 *h4 = reinterpret_cast<uint4 *>(hist) + lane;
                    const uint32_t n4 = (P.hw - (P.n_z0 % PACK == 0 ? 1u : 0u)) * 16, full = n4 >> 6;
#pragma unroll 8
                    for (uint32_t k = 0; k < full; ++k) h4[k * 64] = make_uint4(0u, 0u, 0u, 0u);
                    if (lane < (n4 & 63u)) h4[full * 64] = make_uint4(0u, 0u, 0u, 0u);
                }
                __syncthreads();
                if (jv && bc > best_c) { best_c = bc; best_j = j; best_b = bb; }
            };
            for (uint32_t j0 = 0; j0 < P.n_cot; j0 += 128) {
                pass(j0, zr, zn);
                if (j0 + 64 < P.n_cot) pass(j0 + 64, zn, zr);
            }
        }
        // an overflowed count makes every result of this candidate suspect
        // (a carry reaches the next bin), and a candidate with more members
        // than the list holds was not counted: its record is marked and
        // k_rz_redo recomputes it exactly
        if (nm > lim || (BITS <= 8 && __ballot(ovf) != 0)) {
            P.out4[2 * c] = make_uint2(r.pk, 0u);
            P.out4[2 * c + 1] = make_uint2(kRzRedo, nm);
            if (lane == 0) {
                const uint32_t i = atomicAdd(P.redo_count, 1u);
                if (i < P.redo_cap) P.redo_list[i] = c;
            }
        } else {
            rz_finish(P, c, r.pk, nm, best_c, best_j, best_b);
        }
      }
      }
    }
}

// The exact path for the records k_rz_vote_fast marked (count == kRzRedo):
// the wave takes every gridDim-th entry of the list of marked records the
// fast kernel appended (when they all fit it; otherwise it scans every
// record, in groups of 8, so that marked candidates that are neighbours in
// the record list, a dense event's, spread over many waves).  With
// redo_lds and at most kRedoMembers members, the members are gathered into
// LDS once and counted per cot bin in an LDS histogram of the n_z0 bins,
// every lane taking every 64th member; otherwise rz_slow with the global
// histogram of the wave's workgroup.
constexpr uint32_t kRedoMembers = 8192;
constexpr uint32_t kRedoGroup = 8;

__device__ void rz_exact_lds(const RzParams &P, const RzCand &r, int32_t *mz, uint8_t *ml, uint32_t *hist,
                             uint32_t lane, uint32_t &best_c, uint32_t &best_j, uint32_t &best_b)
{
    // members in walk order; member i is written by lane i % 64
    uint32_t seen = 0;
    for_members(P, r.eb, r.bo, r.k, r.p, r.mask, [&](uint32_t h, uint32_t l) {
        if ((seen & 63u) == lane) {
            mz[seen] = P.z[r.eb + h];
            ml[seen] = uint8_t(l);
        }
        ++seen;
    });
    const uint32_t nm = uni(seen);
    best_c = 0;
    best_j = 0;
    best_b = 0;
    for (uint32_t j = 0; j < P.n_cot; ++j) {
        for (uint32_t i = lane; i < P.n_z0; i += 64) hist[i] = 0;
        __syncthreads();
        for (uint32_t m = lane; m < nm; m += 64) {
            const int64_t zl = int64_t(P.Z[(size_t(r.k) * P.n_layers + ml[m]) * P.n_cot + j]) + P.z0_lo;
            const int32_t b = z0_bin(P, mz[m], zl);
            if (b >= 0) atomicAdd(&hist[b], 1u);
        }
        __syncthreads();
        // the largest count of the cot bin, then its smallest z0 bin
        uint32_t cnt = 0, bin = 0;
        for (uint32_t i = lane; i < P.n_z0; i += 64) {
            const uint32_t v = hist[i];
            if (v > cnt) { cnt = v; bin = i; }
        }
        const uint32_t cmax = wave_max_u32(cnt);
        const uint32_t bkey = wave_max_u32(cmax != 0 && cnt == cmax ? 0xFFFFu - bin : 0u);
        if (cmax > best_c) { best_c = cmax; best_j = j; best_b = 0xFFFFu - bkey; }
        __syncthreads();                              // histogram read before the next clear
    }
}

__global__ void __launch_bounds__(64) k_rz_redo(RzParams P)
{
    HOUGH_DYNAMIC_LDS(uint32_t, rl);                  // with redo_lds: z [kRedoMembers], layers, histogram
    int32_t *mz = reinterpret_cast<int32_t *>(rl);
    uint8_t *ml = reinterpret_cast<uint8_t *>(rl + kRedoMembers);
    uint32_t *hist = rl + kRedoMembers + kRedoMembers / 4;
    const uint32_t lane = threadIdx.x;
    const uint64_t total = min(P.roff[P.n_events], P.out_capacity);
    uint32_t *g = P.gscratch + size_t(blockIdx.x) * P.n_z0;
    auto redo = [&](uint64_t cc) {
        const RzCand r = rz_decode(P, cc);
        const uint32_t nm = uni(P.out4[2 * cc + 1].y);     // the fast kernel's member count
        uint32_t best_c = 0, best_j = 0, best_b = 0;
        if (P.redo_lds && nm <= kRedoMembers)
            rz_exact_lds(P, r, mz, ml, hist, lane, best_c, best_j, best_b);
        else
            rz_slow(P, r.eb, r.bo, r.k, r.p, r.mask, g, lane, best_c, best_j, best_b);
        if (lane != 0) { best_c = 0; best_j = 0xFFFFu; best_b = 0; }
        rz_finish(P, cc, r.pk, nm, best_c, best_j, best_b);
    };
    const uint32_t n = uni(*P.redo_count);
    if (n <= P.redo_cap) {
        for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) redo(uni64(P.redo_list[i]));
        return;
    }
    for (uint64_t c0 = uint64_t(blockIdx.x) * kRedoGroup; c0 < total; c0 += uint64_t(gridDim.x) * kRedoGroup) {
        const uint64_t c = c0 + lane;
        uint64_t bal = __ballot(lane < kRedoGroup && c < total && P.out4[2 * c + 1].x == kRzRedo);
        while (bal) {
            const uint32_t b = __ffsll(static_cast<unsigned long long>(bal)) - 1;
            bal &= bal - 1;
            redo(c0 + b);
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

// For batches of up to kRzOffsetsMaxEvents events, in one workgroup: the
// candidate count of every event (as k_rz_counts), their exclusive prefix
// into roff[0..E] and the reset of the work counters and the marked-record
// count (counter[0 .. kRzCounterDwords)) -- one launch where the general
// path takes three.
constexpr uint32_t kRzOffsetsMaxEvents = 1024 * 8;

__global__ void __launch_bounds__(1024)
k_rz_offsets(const uint64_t *__restrict__ poff, uint64_t peak_capacity, uint32_t n_events, uint32_t cap,
             uint64_t *__restrict__ roff, uint32_t *__restrict__ counter)
{
    __shared__ uint64_t part[1024];
    const uint32_t t = threadIdx.x, nt = blockDim.x;
    auto count = [&](uint32_t e) {
        const uint64_t lo = min(poff[e], peak_capacity), hi = min(max(poff[e + 1], poff[e]), peak_capacity);
        const uint64_t n = hi - lo;
        return cap ? min(n, uint64_t(cap)) : n;
    };
    const uint32_t per = (n_events + nt - 1) / nt;
    const uint32_t b = min(t * per, n_events), end = min(b + per, n_events);
    uint64_t s = 0;
    for (uint32_t e = b; e < end; ++e) s += count(e);
    part[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < nt; off <<= 1) {
        const uint64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint64_t run = t ? part[t - 1] : 0;
    for (uint32_t e = b; e < end; ++e) {
        roff[e] = run;
        run += count(e);
    }
    if (t == nt - 1) roff[n_events] = part[nt - 1];
    for (uint32_t i = t; i < kRzCounterDwords; i += nt) counter[i] = 0;
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

// Split form of the candidate selection for batches of few events: an
// event's stored peaks are cut into K parts of consecutive peaks (256
// threads each).  A peak's bin is 16 - min(popcount, 16), so ascending bins
// are descending popcounts.  k_sel_count counts a part's peaks per bin (one
// ballot per bin per 64 peaks); the split plan gives every bin's start and
// each part's first position per bin, i.e. each peak's position in the
// (popcount desc, cell asc) order; k_sel_write stores the peaks whose
// position is below the event's cap, in that order.
constexpr uint32_t kSelThreads = 256;

__device__ __forceinline__ void sel_part(const uint64_t *poff, uint64_t peak_capacity, uint32_t e, uint32_t k,
                                         uint32_t K, uint64_t &lo, uint64_t &hi, uint64_t &pb, uint64_t &pe)
{
    lo = min(poff[e], peak_capacity);
    hi = min(max(poff[e + 1], poff[e]), peak_capacity);
    const uint64_t n = hi - lo;
    pb = lo + n * k / K;
    pe = lo + n * (k + 1) / K;
}

__global__ void __launch_bounds__(kSelThreads)
k_sel_count(const uint2 *__restrict__ peaks, uint64_t peak_capacity, const uint64_t *__restrict__ poff, uint32_t K,
            uint32_t *__restrict__ part_cnt)
{
    __shared__ uint32_t wc[kSelThreads / 64][kSplitBins];
    const uint32_t t = threadIdx.x, lane = t & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
    uint64_t lo, hi, pb, pe;
    sel_part(poff, peak_capacity, blockIdx.x / K, blockIdx.x % K, K, lo, hi, pb, pe);
    uint32_t cnt[kSplitBins];
#pragma unroll
    for (uint32_t q = 0; q < kSplitBins; ++q) cnt[q] = 0;
    for (uint64_t i0 = pb + wave * 64; i0 < pe; i0 += kSelThreads) {
        const uint64_t i = i0 + lane;
        const uint32_t bin = i < pe ? 16u - min(peaks[i].y >> 16, 16u) : 0xFFu;
#pragma unroll
        for (uint32_t q = 0; q < kSplitBins; ++q) cnt[q] += uint32_t(__popcll(__ballot(bin == q)));
    }
    if (lane == 0) {
#pragma unroll
        for (uint32_t q = 0; q < kSplitBins; ++q) wc[wave][q] = cnt[q];
    }
    __syncthreads();
    if (t < kSplitBins) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < kSelThreads / 64; ++w) s += wc[w][t];
        part_cnt[size_t(blockIdx.x) * kSplitBins + t] = s;
    }
}

__global__ void __launch_bounds__(kSelThreads)
k_sel_write(const uint2 *__restrict__ peaks, uint64_t peak_capacity, const uint64_t *__restrict__ poff,
            const uint64_t *__restrict__ roff, uint32_t cap, uint32_t K, const uint32_t *__restrict__ part_base,
            uint32_t *__restrict__ cand)
{
    __shared__ uint32_t wc[kSelThreads / 64][kSplitBins];
    __shared__ uint32_t base[kSplitBins];
    const uint32_t t = threadIdx.x, lane = t & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t e = blockIdx.x / K;
    uint64_t lo, hi, pb, pe;
    sel_part(poff, peak_capacity, e, blockIdx.x % K, K, lo, hi, pb, pe);
    const uint32_t need = uint32_t(min(hi - lo, uint64_t(cap)));
    if (t < kSplitBins) base[t] = part_base[size_t(blockIdx.x) * kSplitBins + t];
    __syncthreads();
    // nothing of this part is taken once every bin's next position is past the cap
    uint32_t lowest = 0xFFFFFFFFu;
    for (uint32_t q = 0; q < kSplitBins; ++q) lowest = min(lowest, base[q]);
    if (lowest >= need) return;                     // uniform over the workgroup
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t *out = cand + roff[e];
    for (uint64_t r0 = pb; r0 < pe; r0 += kSelThreads) {
        const uint64_t i = r0 + t;
        const uint32_t bin = i < pe ? 16u - min(peaks[i].y >> 16, 16u) : 0xFFu;
        uint32_t rank = 0;
#pragma unroll
        for (uint32_t q = 0; q < kSplitBins; ++q) {
            const uint64_t m = __ballot(bin == q);
            if (lane == 0) wc[wave][q] = uint32_t(__popcll(m));
            if (bin == q) rank = uint32_t(__popcll(m & lt));
        }
        __syncthreads();
        if (bin < kSplitBins) {
            uint32_t pos = base[bin] + rank;
            for (uint32_t w = 0; w < wave; ++w) pos += wc[w][bin];
            if (pos < need) out[pos] = uint32_t(i - lo);
        }
        __syncthreads();
        if (t < kSplitBins) {
            uint32_t s = 0;
            for (uint32_t w = 0; w < kSelThreads / 64; ++w) s += wc[w][t];
            base[t] += s;
        }
        __syncthreads();
    }
}

uint32_t rz_blocks(const hough_ctx *c)
{
    const uint32_t w = c->tun.rz_waves_per_cu ? c->tun.rz_waves_per_cu : 8;
    return uint32_t(c->n_cu) * w;
}

namespace {

template <int BITS>
void launch_fast(int mul, uint32_t blocks, size_t lds, hipStream_t s, const RzParams &P)
{
    if (mul == 2)
        hipLaunchKernelGGL((k_rz_vote_fast<BITS, 2>), dim3(blocks), dim3(64), lds, s, P);
    else if (mul == 1)
        hipLaunchKernelGGL((k_rz_vote_fast<BITS, 1>), dim3(blocks), dim3(64), lds, s, P);
    else
        hipLaunchKernelGGL((k_rz_vote_fast<BITS, 0>), dim3(blocks), dim3(64), lds, s, P);
}

// An upper bound of the rz records of a call (the kernels read the true
// count on the device): the capacity, and no more than the candidates.
uint64_t rz_records_bound(const hough_ctx *c, const hough_hits *h, uint64_t peak_capacity, uint64_t capacity)
{
    const uint32_t cap = c->spec.rz_max_candidates;
    return std::min<uint64_t>(capacity, cap ? uint64_t(h->n_events) * cap : peak_capacity);
}

}  // namespace

hipError_t launch_rz(hough_ctx *c, const hough_hits *h, const hough_peak *peaks, uint64_t peak_capacity,
                     const uint64_t *poff, hough_rz *out, uint64_t capacity, uint64_t *roff, hipStream_t s)
{
    hipError_t err;
    const hough_grid_spec &g = c->spec;
    const uint32_t E = h->n_events;
    if ((err = launch_bucket_layers(c, h, true, s)) != hipSuccess) return err;
    if ((err = launch_bucket_phi(c, h, s)) != hipSuccess) return err;
    KernelTimer t;
    const bool fused = E <= kRzOffsetsMaxEvents;
    prof_begin(c, "rz_counts", s, &t);
    if (fused)
        hipLaunchKernelGGL(k_rz_offsets, dim3(1), dim3(1024), 0, s, poff, peak_capacity, E, g.rz_max_candidates,
                           roff, c->d_counters + kRzCounterBase);
    else
        hipLaunchKernelGGL(k_rz_counts, dim3((E + 255) / 256), dim3(256), 0, s, poff, peak_capacity, E,
                           g.rz_max_candidates, c->d_cand_counts);
    prof_end(c, s, &t);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (!fused && (err = launch_scan_counts(c, c->d_cand_counts, E, c->d_tile_off, 1, roff, s)) != hipSuccess)
        return err;
    if (g.rz_max_candidates) {
        prof_begin(c, "rz_select", s, &t);
        if (const uint32_t K = split_parts(c, E)) {
            const uint2 *pk = reinterpret_cast<const uint2 *>(peaks);
            hipLaunchKernelGGL(k_sel_count, dim3(E * K), dim3(kSelThreads), 0, s, pk, peak_capacity, poff, K,
                               c->d_part_cnt);
            if ((err = launch_split_plan(E, kSplitBins, K, c->d_part_cnt, c->d_part_base, nullptr, s)) !=
                hipSuccess)
                return err;
            hipLaunchKernelGGL(k_sel_write, dim3(E * K), dim3(kSelThreads), 0, s, pk, peak_capacity, poff, roff,
                               g.rz_max_candidates, K, c->d_part_base, c->d_cand);
        } else {
            hipLaunchKernelGGL(k_rz_select, dim3(E), dim3(256), 0, s,
                               reinterpret_cast<const uint2 *>(peaks), peak_capacity, poff, roff,
                               g.rz_max_candidates, c->d_cand);
        }
        prof_end(c, s, &t);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if (!fused && (err = launch_fill_u32(c, c->d_counters + kRzCounterBase, 0, kRzCounterDwords, s)) != hipSuccess)
        return err;

    RzParams P;
    P.phi = c->d_phi_b;
    P.z = c->d_z_b;
    P.offs = h->event_offsets;
    P.n_hits = h->n_hits;
    P.bucket_off = c->d_bucket_off;
    P.O = c->d_O;
    P.V = c->d_V;
    P.Z = c->d_Z;
    P.Zl = c->d_Zl;
    P.peaks = reinterpret_cast<const uint2 *>(peaks);
    P.peak_capacity = peak_capacity;
    P.poff = poff;
    P.roff = roff;
    P.cand = c->d_cand;
    P.out4 = reinterpret_cast<uint2 *>(out);
    P.out_capacity = capacity;
    P.counter = c->d_counters + kRzCounterBase;
    P.redo_count = c->d_counters + kRzCounterBase + kRzRedoCountAt;
    P.redo_list = c->d_redo_list;
    P.redo_cap = c->tun.rz_redo_list ? c->tun.rz_redo_list : kRedoListCap;
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
    P.bm = c->rz_magic_m;
    P.bs = c->rz_magic_s;
    // counter width (4- and 8-bit counters detect an overflow and then take
    // the slow path): 4 bits when a cell's members (about hits / n_phi per
    // event) are few, so that counts above 15 are rare and 16 waves fit a
    // CU's LDS; 8 bits for dense events; 16 bits only when tuned so
    const double per_cell = double(h->n_hits) / double(std::max<uint32_t>(E, 1)) / double(g.n_phi);
    uint32_t bits = c->tun.rz_counter_bits ? c->tun.rz_counter_bits : (per_cell < 48.0 ? 4u : 8u);
    const uint32_t blocks = c->tun.rz_waves_per_cu ? rz_blocks(c) : uint32_t(c->n_cu) * (bits == 4 ? 16u : 8u);
    // counter dwords per lane: bins 0 .. n_z0 - 1 plus the trash bin n_z0
    const uint32_t hw = g.n_z0 / (32 / bits) + 1;
    // member lists: 112 with 4-bit counters (16 waves of counters and two
    // lists fit 160 KB); otherwise 2048 (tunable), reduced until it fits the
    // LDS budget: a candidate with more members goes to k_rz_redo, whose
    // exact path is far slower per candidate, so dense events need a list
    // that holds their cells; a 4096-member list only costs occupancy
    // (16-event c5 micro-batches: rz 1.40 ms with 4096, 0.87 ms with 2048,
    // and 0.87 ms plus 40 ms of exact path with 1024)
    uint32_t mcap = bits == 4 ? 112 : 256;
    if (bits != 4 || c->tun.rz_member_cap) {
        mcap = c->tun.rz_member_cap ? c->tun.rz_member_cap : 2048;
        while (mcap > 256 && size_t(rz_fast_lds_dwords(hw, mcap)) * 4 > c->max_lds) mcap >>= 1;
    }
    const size_t fast_lds = size_t(rz_fast_lds_dwords(hw, mcap)) * 4;
    // the fast kernel pads member lists with a spare layer (n_layers < 16)
    if (c->rz_fast && !c->tun.rz_slow_path && fast_lds <= c->max_lds && g.n_layers < kMaxLayers) {
        P.hw = hw;
        P.mcap = mcap;
        // one queue per XCD where the records can give every wave several
        // tickets; one queue for short lists (a micro-batch), whose waves
        // would spend more on empty tickets than the queues save (16-event
        // c5 micro-batches served at 17k events/s with 8 queues, 19.7k with
        // one)
        P.n_queues = rz_records_bound(c, h, peak_capacity, capacity) >= uint64_t(4) * blocks * kRzChunk ? kRzQueues : 1u;
        P.lds_ok = 0;
        prof_begin(c, "rz_vote", s, &t);
        const int mul = P.bs != 0 ? 1 : (P.span < (1u << 24) && P.bm < (1u << 24)) ? 2 : 0;
        P.span24 = uint32_t(P.span);
        if (bits == 4)
            launch_fast<4>(mul, blocks, fast_lds, s, P);
        else if (bits == 8)
            launch_fast<8>(mul, blocks, fast_lds, s, P);
        else
            launch_fast<16>(mul, blocks, fast_lds, s, P);
        prof_end(c, s, &t);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        // candidates the fast kernel marked (grid-stride over the list of
        // them, or over every record group); at most the slow path's
        // histograms
        const uint64_t groups =
            std::max<uint64_t>(1, (rz_records_bound(c, h, peak_capacity, capacity) + kRedoGroup - 1) / kRedoGroup);
        const size_t redo_lds = (size_t(kRedoMembers) * 5 + size_t(g.n_z0) * 4 + 15) & ~size_t(15);
        P.redo_lds = redo_lds <= c->max_lds ? 1u : 0u;
        // as many workgroups as are resident at once with the LDS path's
        // allocation (they mostly find the list empty and exit)
        const uint64_t resident = uint64_t(c->n_cu) * std::max<size_t>(1, P.redo_lds ? c->max_lds / redo_lds : 16);
        const uint64_t grid = std::min<uint64_t>(std::min<uint64_t>(groups, resident), rz_blocks_max(c));
        prof_begin(c, "rz_redo", s, &t);
        hipLaunchKernelGGL(k_rz_redo, dim3(uint32_t(grid)), dim3(64), P.redo_lds ? redo_lds : 0, s, P);
        prof_end(c, s, &t);
        return hipGetLastError();
    }
    const size_t lds = size_t(g.n_z0) * 64 * sizeof(uint16_t);
    P.lds_ok = lds <= c->max_lds && !c->tun.rz_slow_path;
    P.hw = 0;
    P.mcap = 0;
    prof_begin(c, "rz_vote", s, &t);
    hipLaunchKernelGGL(k_rz_vote, dim3(blocks), dim3(64), P.lds_ok ? lds : 0, s, P);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
