// Candidate confirmation, first part: plateau clusters of the peak list.
//
// The non-strict local-maximum rule keeps every cell of a flat-topped ridge,
// so one track yields several adjacent peaks (Section 4 leaves the
// confirmation of candidates to later, more expensive computations).  Two
// peaks of one event are adjacent when their cells are neighbours in the
// local-maximum neighbourhood (3x3, 3x3x3 with a d0 axis; phi0 periodic);
// a cluster is a connected component of that relation.
//
// GPU form: lock-free union-find over peak-list indices.
//   init  -- parent[i] = i;
//   link  -- every peak looks up its half neighbourhood (the neighbours
//            after it in (d, k, p) order, so each adjacent pair is seen
//            once) in its event's sorted cell list by a bounded binary
//            search, and unites the two trees; a root is always hooked
//            under a smaller index, so parent[i] <= i, a tree's root is its
//            smallest member, and no cycle can form;
//   flat  -- parent[i] = root(i), found by a walk that writes nothing else;
//            per block of 4096 peaks, the root count;
//   scan  -- exclusive prefix of the block counts;
//   rank  -- roots get their global rank (= cluster index, ordered by first
//            peak) and initialise their cluster record;
//   acc   -- every peak replaces parent[i] by its cluster's index within
//            the event and adds its offsets to the cluster's sums (integer
//            atomics, so the result does not depend on their order).
// The parent array is the caller's per-peak label output; the ranks live in
// the context (max_peaks entries).
#include "hough_internal.h"

namespace hough {
namespace {

constexpr uint32_t kClThreads = 256, kClPer = 16, kClBlock = kClThreads * kClPer;

struct ClParams {
    const uint2 *pk;         // peak records: x = cell, y = mask | popcount << 16
    const uint64_t *poff;    // [E + 1] event peak offsets
    uint32_t E;
    uint64_t cap;            // peak capacity
    uint32_t *par;           // [cap] parent, finally the label
    uint32_t *rank;          // [cap] cluster index of each root
    uint32_t *part;          // [nb] roots per block
    const uint64_t *part_off;// [nb + 1] their exclusive prefix
    uint64_t nb;
    hough_cluster *cl;
    uint64_t cl_cap;
    uint64_t *coff;          // [E + 1] event cluster offsets
    uint32_t n_phi, log2_phi, n_qpt, n_d0;
};

__device__ __forceinline__ uint64_t n_stored(const ClParams &P)
{
    return min(P.poff[P.E], P.cap);
}

// Largest event e with start(e) <= i (offsets ascending, as hough_peaks
// writes them).
__device__ __forceinline__ uint32_t event_of(const ClParams &P, uint64_t n, uint64_t i)
{
    uint32_t lo = 0, hi = P.E;
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (min(P.poff[m], n) <= i) lo = m;
        else hi = m;
    }
    return lo;
}

__device__ __forceinline__ uint32_t ld_par(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_par(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  Every parent is <= its child and a root is
// its own parent, so the walk strictly descends and ends.
__device__ uint32_t cl_find(uint32_t *par, uint32_t x)
{
    uint32_t next = ld_par(par + x);
    while (next != x) {
        const uint32_t nn = ld_par(par + next);
        if (nn != next) st_par(par + x, nn);
        x = next;
        next = nn;
    }
    return x;
}

// Root of x without writing.  The flattening pass uses this walk: a halving
// store from another thread could otherwise overwrite parent[x] after x's
// own thread has set it to the root, leaving an ancestor that is no root.
__device__ uint32_t cl_root(const uint32_t *par, uint32_t x)
{
    uint32_t next = ld_par(par + x);
    while (next != x) {
        x = next;
        next = ld_par(par + x);
    }
    return x;
}

// Unite the trees of a and b, hooking the larger root under the smaller.  A
// failed CAS means another thread hooked b meanwhile; every hook removes one
// of at most n roots, so the retries are bounded and the loop ends.
__device__ void cl_unite(uint32_t *par, uint32_t a, uint32_t b)
{
    for (;;) {
        a = cl_find(par, a);
        b = cl_find(par, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        uint32_t expect = b;
        if (__hip_atomic_compare_exchange_strong(par + b, &expect, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        b = expect;
    }
}

__global__ void __launch_bounds__(256) k_cl_init(ClParams P)
{
    const uint64_t n = n_stored(P);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        P.par[i] = uint32_t(i);
}

__global__ void __launch_bounds__(256) k_cl_link(ClParams P)
{
    const uint64_t n = n_stored(P);
    const uint32_t pmask = P.n_phi - 1;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t e = event_of(P, n, i);
        const uint64_t lo = min(P.poff[e], n);
        const uint64_t hi = max(min(P.poff[e + 1], n), lo);
        const uint32_t c = P.pk[i].x;
        const uint32_t p = c & pmask, row = c >> P.log2_phi;
        const uint32_t k = row % P.n_qpt, d = row / P.n_qpt;
        // first index in [b, t) whose cell is >= key (cells ascend)
        auto lower = [&](uint64_t b, uint64_t t, uint32_t key) {
            while (b < t) {
                const uint64_t m = (b + t) >> 1;
                if (P.pk[m].x < key) b = m + 1;
                else t = m;
            }
            return b;
        };
        // one neighbour cell c2, wherever it is: after i when larger (at
        // most c2 - c places on), before i when smaller (phi0 wrap)
        auto try_cell = [&](uint32_t c2) {
            uint64_t b, t;
            if (c2 > c) {
                b = i + 1;
                t = min(hi, i + 1 + uint64_t(c2 - c));
            } else if (c2 < c) {
                const uint64_t back = uint64_t(c - c2);
                b = i - lo > back ? i - back : lo;
                t = i;
            } else {
                return;
            }
            if (b >= t) return;
            const uint64_t j = lower(b, t, c2);
            if (j < t && P.pk[j].x == c2) cl_unite(P.par, uint32_t(i), uint32_t(j));
        };
        // three consecutive cells ca .. ca + 2 of a later row (no wrap inside):
        // one search, then at most three list entries
        auto try_triple = [&](uint32_t ca) {
            const uint64_t t = min(hi, i + 1 + uint64_t(ca + 2 - c));
            if (i + 1 >= t) return;
            for (uint64_t q = lower(i + 1, t, ca); q < t; ++q) {
                if (P.pk[q].x > ca + 2) break;
                cl_unite(P.par, uint32_t(i), uint32_t(q));
            }
        };
        auto try_row = [&](uint32_t rbase) {
            if (p != 0 && p != pmask) {
                try_triple(rbase | (p - 1));
            } else {
                try_cell(rbase | ((p - 1) & pmask));
                try_cell(rbase | p);
                try_cell(rbase | ((p + 1) & pmask));
            }
        };
        if (p != pmask) {
            if (i + 1 < hi && P.pk[i + 1].x == c + 1) cl_unite(P.par, uint32_t(i), uint32_t(i + 1));
        } else {
            try_cell(row << P.log2_phi);                // (k, 0) across the wrap
        }
        if (k + 1 < P.n_qpt) try_row((row + 1) << P.log2_phi);
        if (d + 1 < P.n_d0) {
            for (int dk = -1; dk <= 1; ++dk) {
                const int k2 = int(k) + dk;
                if (k2 < 0 || k2 >= int(P.n_qpt)) continue;
                try_row(((d + 1) * P.n_qpt + uint32_t(k2)) << P.log2_phi);
            }
        }
    }
}

// Roots per block of kClBlock list entries, parents flattened.
__global__ void __launch_bounds__(kClThreads) k_cl_flat(ClParams P)
{
    __shared__ uint32_t wsum[kClThreads / 64];
    const uint64_t n = n_stored(P);
    const uint64_t base = uint64_t(blockIdx.x) * kClBlock;
    uint32_t roots = 0;
    if (base < n) {
#pragma unroll 4
        for (uint32_t j = 0; j < kClPer; ++j) {
            const uint64_t i = base + uint64_t(j) * kClThreads + threadIdx.x;
            if (i < n) {
                const uint32_t r = cl_root(P.par, uint32_t(i));
                st_par(P.par + i, r);
                roots += r == uint32_t(i);
            }
        }
    }
    for (uint32_t off = 32; off > 0; off >>= 1) roots += __shfl_down(roots, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = roots;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < kClThreads / 64; ++w) s += wsum[w];
        P.part[blockIdx.x] = s;
    }
}

// Global rank of every root (in list order) and its cluster record.
__global__ void __launch_bounds__(kClThreads) k_cl_rank(ClParams P)
{
    __shared__ uint32_t wsum[kClThreads / 64];
    const uint64_t n = n_stored(P);
    const uint64_t base = uint64_t(blockIdx.x) * kClBlock;
    if (base >= n) return;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t run = P.part_off[blockIdx.x];
    for (uint32_t j = 0; j < kClPer; ++j) {
        const uint64_t i = base + uint64_t(j) * kClThreads + threadIdx.x;
        const bool root = i < n && P.par[i] == uint32_t(i);
        const uint64_t bal = __ballot(root);
        if (lane == 0) wsum[wave] = uint32_t(__popcll(bal));
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t w = 0; w < kClThreads / 64; ++w) {
            before += w < wave ? wsum[w] : 0u;
            total += wsum[w];
        }
        __syncthreads();
        if (root) {
            const uint64_t r = run + before + uint32_t(__popcll(bal & ((uint64_t(1) << lane) - 1)));
            P.rank[i] = uint32_t(r);
            if (r < P.cl_cap) {
                const uint32_t e = event_of(P, n, i);
                const uint2 rec = P.pk[i];
                hough_cluster h;
                h.first = uint32_t(i - min(P.poff[e], n));
                h.popcount = uint16_t(rec.y >> 16);
                h.mask_or = uint16_t(rec.y);
                h.n_peaks = 1;
                h.sum_dk = 0;
                h.sum_dp = 0;
                h.sum_dd = 0;
                P.cl[r] = h;
            }
        }
        run += total;
        if (base + uint64_t(j + 1) * kClThreads >= n) break;
    }
}

// Labels (cluster index within the event), member sums, event offsets.
// Whole waves step through the list together: runs of adjacent lanes in one
// cluster (a flat plateau along phi0 is a run of consecutive list entries)
// are summed by segmented shuffles first, and the run's last lane issues the
// atomics once for the run.
__global__ void __launch_bounds__(256) k_cl_acc(ClParams P)
{
    const uint64_t n = n_stored(P);
    const uint64_t total = P.part_off[P.nb];
    const uint64_t g0 = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x, gs = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t e = g0; e <= P.E; e += gs) {
        const uint64_t s = min(P.poff[e], n);
        P.coff[e] = s < n ? P.rank[s] : total;
    }
    const uint32_t pmask = P.n_phi - 1, lane = threadIdx.x & 63;
    const int32_t half = int32_t(P.n_phi >> 1);
    const uint64_t lanes_below = lane == 63 ? ~uint64_t(0) : (uint64_t(2) << lane) - 1;
    for (uint64_t base = g0 - lane; base < n; base += gs) {
        const uint64_t i = base + lane;
        uint32_t key = 0xFFFFFFFFu, cnt = 0, m = 0, r = 0;
        int32_t dk = 0, dp = 0, dd = 0;
        if (i < n) {
            const uint32_t e = event_of(P, n, i);
            const uint64_t lo = min(P.poff[e], i);
            r = P.par[i];
            const uint32_t cid = P.rank[r];
            P.par[i] = cid - P.rank[lo];
            if (r != uint32_t(i) && cid < P.cl_cap) {
                const uint32_t c = P.pk[i].x, cr = P.pk[r].x;
                const uint32_t row = c >> P.log2_phi, rowr = cr >> P.log2_phi;
                key = cid;
                cnt = 1;
                dk = int32_t(row % P.n_qpt) - int32_t(rowr % P.n_qpt);
                dd = int32_t(row / P.n_qpt) - int32_t(rowr / P.n_qpt);
                dp = int32_t((c - cr) & pmask);
                if (dp >= half) dp -= int32_t(P.n_phi);
                m = P.pk[i].y & 0xFFFFu;
            }
        }
        // segmented inclusive sums over runs of equal keys
        const uint32_t prev = __shfl_up(key, 1, 64);
        const uint64_t heads = __ballot(lane == 0 || prev != key);
        const uint32_t start = 63u - uint32_t(__clzll(heads & lanes_below));
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t c2 = __shfl_up(cnt, d, 64), m2 = __shfl_up(m, d, 64);
            const int32_t k2 = __shfl_up(dk, d, 64), p2 = __shfl_up(dp, d, 64), d2 = __shfl_up(dd, d, 64);
            if (lane >= start + d) {
                cnt += c2;
                m |= m2;
                dk += k2;
                dp += p2;
                dd += d2;
            }
        }
        const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1u);
        if (tail && key != 0xFFFFFFFFu) {
            hough_cluster *h = P.cl + key;
            // n_peaks (low word, never carries) and sum_dk (high word) in one add
            atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_peaks),
                      (static_cast<unsigned long long>(uint32_t(dk)) << 32) | cnt);
            if (dp) atomicAdd(&h->sum_dp, dp);
            if (dd) atomicAdd(&h->sum_dd, dd);
            const uint32_t mr = P.pk[r].y & 0xFFFFu;
            if (m & ~mr) atomicOr(reinterpret_cast<uint32_t *>(&h->popcount), m << 16);
        }
    }
}

uint32_t grid_for(const hough_ctx *c, uint64_t n)
{
    return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, uint64_t(c->n_cu) * 16)));
}

}  // namespace

uint64_t cluster_blocks(uint64_t n)
{
    return (n + kClBlock - 1) / kClBlock;
}

hipError_t launch_clusters(hough_ctx *c, const hough_peak *peaks, uint64_t peak_capacity, const uint64_t *poff,
                           uint32_t n_events, uint32_t *labels, hough_cluster *clusters, uint64_t capacity,
                           uint64_t *coff, hipStream_t s)
{
    if (n_events == 0) return launch_fill_u32(c, reinterpret_cast<uint32_t *>(coff), 0u, 2, s);
    ClParams P{};
    P.pk = reinterpret_cast<const uint2 *>(peaks);
    P.poff = poff;
    P.E = n_events;
    P.cap = peak_capacity;
    P.par = labels;
    P.rank = c->d_cl_rank;
    P.part = c->d_cl_part;
    P.part_off = c->d_cl_part_off;
    P.nb = cluster_blocks(peak_capacity);
    P.cl = clusters;
    P.cl_cap = capacity;
    P.coff = coff;
    P.n_phi = c->spec.n_phi;
    P.log2_phi = c->log2_phi;
    P.n_qpt = c->spec.n_qpt;
    P.n_d0 = c->spec.n_d0;
    const uint32_t g = grid_for(c, peak_capacity);
    KernelTimer t;
    prof_begin(c, "cluster_init", s, &t);
    hipLaunchKernelGGL(k_cl_init, dim3(g), dim3(256), 0, s, P);
    prof_end(c, s, &t);
    prof_begin(c, "cluster_link", s, &t);
    hipLaunchKernelGGL(k_cl_link, dim3(g), dim3(256), 0, s, P);
    prof_end(c, s, &t);
    if (P.nb) {
        prof_begin(c, "cluster_flat", s, &t);
        hipLaunchKernelGGL(k_cl_flat, dim3(uint32_t(P.nb)), dim3(kClThreads), 0, s, P);
        prof_end(c, s, &t);
    }
    hipError_t e = launch_scan_counts(c, c->d_cl_part, P.nb, c->d_cl_part_off, 0, nullptr, s);
    if (e != hipSuccess) return e;
    if (P.nb) {
        prof_begin(c, "cluster_rank", s, &t);
        hipLaunchKernelGGL(k_cl_rank, dim3(uint32_t(P.nb)), dim3(kClThreads), 0, s, P);
        prof_end(c, s, &t);
    }
    prof_begin(c, "cluster_acc", s, &t);
    hipLaunchKernelGGL(k_cl_acc, dim3(std::max(g, (n_events + 256u) / 256u)), dim3(256), 0, s, P);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
