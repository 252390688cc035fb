// Internal declarations of the MI355X Hough-transform library: the context,
// host tables and the launchers of every kernel.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hough.h"
#include "rank_tables.h"
#include "tables.h"

// A kernel's dynamically sized LDS array (its byte size is given at launch).
#ifndef HOUGH_DYNAMIC_LDS
#define HOUGH_DYNAMIC_LDS(type, name) extern __shared__ type name[]
#endif

namespace hough {

// Coarse azimuth buckets used to find the member hits of an rz candidate:
// log2(n_phi) + 2 bits, at most 12 (4096 buckets per layer).
constexpr uint32_t kMaxBucketBits = 12;

// The offset table is followed by this many zero entries, so a kernel may
// read a whole tile's worth of offsets past the last row.
constexpr size_t kOPad = 64;

struct KernelTimer {
    const char *name;
    hipEvent_t start, stop;
};

struct KernelStat {
    std::string name;
    uint64_t launches = 0;
    double total_ms = 0.0;
};

}  // namespace hough

struct hough_ctx {
    hough_grid_spec spec{};
    hough_limits lim{};
    hough_tuning tun{};
    int device = 0;
    int n_cu = 256;
    size_t max_lds = 65536;

    uint32_t log2_phi = 0;
    uint32_t shift = 0;          // 32 - log2_phi
    uint32_t rows = 0;           // n_d0 * n_qpt
    uint64_t cells = 0;          // rows * n_phi
    uint32_t bucket_bits = 0;    // member search buckets (0 without rz and without max_peaks)

    // tables (device)
    uint32_t *d_O = nullptr;     // [L][rows] + kOPad zero entries
    uint8_t *d_V = nullptr;      // [L][rows]
    int32_t *d_Z = nullptr;      // [n_qpt][L][n_cot]
    int32_t *d_Zl = nullptr;     // [n_qpt][n_cot][16] = Z + z0_lo (0 past n_layers), when rz_fast
    bool all_valid = true;       // every (layer, row) reachable
    // rz fast path: z - (Z + z0_lo) is exact in uint32 arithmetic and the z0
    // bin is one multiply-high (see fastdiv.h BinMagic)
    bool rz_fast = false;
    uint32_t rz_magic_m = 0, rz_magic_s = 0;

    // scratch (device)
    uint32_t *d_phi_a = nullptr;     // [max_hits] hits grouped by layer
    int32_t *d_z_a = nullptr;        // [max_hits]
    uint32_t *d_phi_b = nullptr;     // [max_hits] grouped by (layer, bucket) for rz
    int32_t *d_z_b = nullptr;        // [max_hits]
    uint32_t *d_layer_off = nullptr; // [max_events][L + 1] relative to the event start
    uint32_t *d_bucket_off = nullptr;// [max_events][L][NB + 1]
    uint32_t *d_order = nullptr;     // [max_events] events, longest first
    uint32_t *d_counters = nullptr;  // [kCounterDwords] work-queue counters
    uint32_t *d_tile_counts = nullptr; // [max peak tiles]
    uint64_t *d_tile_off = nullptr;    // [max peak tiles + 1]
    uint32_t *d_cand = nullptr;        // [max_events * rz_max_candidates]
    uint32_t *d_cand_counts = nullptr; // [max_events]
    // split forms of the per-event passes for batches of few events (K
    // parts per event, E * K <= max_events + kSplitPartsPerCu * n_cu):
    uint32_t *d_part_cnt = nullptr;    // [parts][kSplitBins] per-part counts
    uint32_t *d_part_base = nullptr;   // [parts][kSplitBins] per-part starts
    uint64_t max_parts = 0;
    uint32_t *d_rz_hist = nullptr;     // [rz blocks][n_z0] zeroed uint32 (rz slow path)
    uint64_t *d_redo_list = nullptr;   // [kRedoListCap] records the fast rz kernel leaves to the exact path
    uint4 *d_gap_info = nullptr;       // [max_events][L] gap vote: {mode, entries, list start, 0}
    uint2 *d_gap_list = nullptr;       // [max_hits] gap vote: per-layer hit or gap lists
    uint64_t *d_scan_part = nullptr;   // [scan_blocks_max] block sums of a multi-block scan
    uint64_t *d_scan_off = nullptr;    // [scan_blocks_max + 1] their exclusive prefix
    uint64_t scan_blocks_max = 0;
    uint2 *d_dir_tab = nullptr;        // [max_events][L][n_phi] direct vote: per-bucket {lo, span}
    uint32_t *d_rk_info = nullptr;     // [rows][32] rank vote: J | unreachable << 31, then (0x80 + rank) x 0x01010101
    uint32_t *d_rk_sorted = nullptr;   // rank vote: [tiles][L][kRankSortStride] sorted fine offsets, then
                                       // the whole-event tables (RankGlobLayout)
    size_t max_lds_direct = 65536;     // LDS budget of the direct vote's table staging
    size_t max_lds_rank = 65536;       // LDS budget of the rank vote (two workgroups per compute unit)
    uint64_t n_peak_tiles = 0;
    uint32_t *d_cl_rank = nullptr;     // [max_peaks] plateau clusters: cluster index of each root
    uint32_t *d_cl_part = nullptr;     // [cluster blocks] roots per block of the peak list
    uint64_t *d_cl_part_off = nullptr; // [cluster blocks + 1] their exclusive prefix

    // profiling
    bool prof = false;
    bool capturing = false;
    std::vector<hough::KernelTimer> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<hough::KernelStat> stats;

    std::string last_error;
};

namespace hough {

// Launch bracket for per-kernel timing (no-op unless profiling is enabled).
void prof_begin(hough_ctx *c, const char *name, hipStream_t s, KernelTimer *t);
void prof_end(hough_ctx *c, hipStream_t s, KernelTimer *t);

// ---- launchers (each returns the HIP status of its launch) --------------
hipError_t launch_fill_u32(hough_ctx *c, uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_bucket_layers(hough_ctx *c, const hough_hits *h, bool with_z, hipStream_t s);
hipError_t launch_bucket_phi(hough_ctx *c, const hough_hits *h, hipStream_t s, bool with_z = true);
hipError_t launch_event_order(hough_ctx *c, const hough_hits *h, hipStream_t s);
hipError_t launch_vote(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s);
hipError_t launch_vote_count(hough_ctx *c, const hough_hits *h, uint32_t *counts, hipStream_t s);
hipError_t launch_peaks_count(hough_ctx *c, const uint32_t *counts, uint32_t n_events, uint2 *peaks,
                              uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s);
// Scratch of the peak search: per-tile peak counts, their exclusive prefix
// and the block sums of a multi-block scan over them.
struct PeakScratch {
    uint32_t *tile_counts;        // [tiles]
    uint64_t *tile_off;           // [tiles + 1]
    uint64_t *scan_part;          // [scan_blocks_max]
    uint64_t *scan_off;           // [scan_blocks_max + 1]
    uint64_t scan_blocks_max;
};
PeakScratch ctx_peak_scratch(hough_ctx *c);
// Row-window peak form (k_peaks_rows.hip): cells per lane (4, 8 or 16)
// when it applies to this context, accumulator and batch size, else 0;
// rows per wavefront strip; one pass (count or write) over n_events
// accumulators with the tile counts and offsets of ps.
constexpr uint32_t kPeakThreads = 256;
uint32_t peak_rows_cells_per_lane(const hough_ctx *c, const uint16_t *acc, uint32_t n_events);
uint32_t peak_rows_strip(const hough_ctx *c);
hipError_t launch_peaks_rows_pass(hough_ctx *c, bool write, const uint16_t *acc, uint32_t n_events,
                                  hough_peak *peaks, uint64_t capacity, const PeakScratch &ps, hipStream_t s);
// Split forms (k_bucket.hip, k_rz.hip): a batch of E events is cut into K
// parts per event when E is small, so that a per-event pass runs on many
// workgroups; K = 0 when the one-workgroup-per-event form is used.
constexpr uint32_t kSplitPartsPerCu = 4;
constexpr uint32_t kSplitMaxParts = 64;
constexpr uint32_t kSplitBins = 17;      // layers (<= 16) or popcount levels 0..16
inline uint32_t split_parts(const hough_ctx *c, uint32_t E)
{
    if (E == 0 || E >= 2u * uint32_t(c->n_cu) || !c->d_part_cnt) return 0;
    const uint32_t K = (kSplitPartsPerCu * uint32_t(c->n_cu) + E - 1) / E;
    return K < 2 ? 0 : (K > kSplitMaxParts ? kSplitMaxParts : K);
}
// The split forms' plan pass (k_bucket.hip): per event, the start of each of
// n_bins bins and each part's first position per bin (bin_off may be null).
hipError_t launch_split_plan(uint32_t n_events, uint32_t n_bins, uint32_t K, const uint32_t *part_cnt,
                             uint32_t *part_base, uint32_t *bin_off, hipStream_t s);
// Number of tiles the peak search of n_events accumulators at `acc` uses.
uint64_t peak_items(const hough_ctx *c, uint32_t n_events, const uint16_t *acc);
// timed = false: no per-kernel timing (no HIP events are created)
hipError_t launch_peaks(hough_ctx *c, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                        uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s,
                        const PeakScratch &ps, bool timed = true);
hipError_t launch_peaks(hough_ctx *c, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                        uint64_t capacity, uint64_t *event_peak_offsets, hipStream_t s);
// hough_peaks_noalloc's file-scope device scratch: its byte size, the
// lookup of its address on a device (once per device, with that device
// current) and that address (nullptr until looked up).
extern const size_t kNoAllocScratchBytes;
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
// Bytes of peak scratch for n tiles when carved from one buffer, and the carving.
size_t peak_scratch_bytes(uint64_t n_tiles);
PeakScratch carve_peak_scratch(void *base, uint64_t n_tiles);
hipError_t launch_rz(hough_ctx *c, const hough_hits *h, const hough_peak *peaks,
                     uint64_t peak_capacity, const uint64_t *event_peak_offsets, hough_rz *out,
                     uint64_t capacity, uint64_t *event_rz_offsets, hipStream_t s);
hipError_t launch_gather_events(const uint8_t *sl, const uint32_t *sp, const int32_t *sz, const uint64_t *src_off,
                                const uint64_t *len, const uint64_t *dst_off, uint32_t n, uint8_t *dl,
                                uint32_t *dp, int32_t *dz, uint64_t cap, hipStream_t s);
uint32_t vote_rows(const hough_ctx *c);
hipError_t launch_vote_gaps(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s);
hipError_t launch_vote_direct(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s);
bool direct_vote_usable(const hough_ctx *c);
hipError_t launch_vote_bounds(hough_ctx *c, const hough_hits *h, hipStream_t s);
// rank form: spec support, host tables (built at create), usability, launch
bool rank_vote_usable(const hough_ctx *c, const uint16_t *acc);
hipError_t launch_vote_rank(hough_ctx *c, const hough_hits *h, uint16_t *acc, hipStream_t s);
uint32_t gap_rows(const hough_ctx *c);
bool gap_vote_usable(const hough_ctx *c);
uint32_t rz_blocks(const hough_ctx *c);
// Persistent rz workgroups at most (each owns an n_z0 histogram of the
// context's slow-path scratch).
constexpr uint32_t kMaxRzWavesPerCu = 16;
// size of the context's array of work-queue counters (dwords)
constexpr uint32_t kCounterDwords = 512;
// capacity of the list of records the fast rz kernel leaves to the exact path
// (past it, the exact-path kernel scans every record for the marks)
constexpr uint32_t kRedoListCap = 1u << 16;
inline uint32_t rz_blocks_max(const hough_ctx *c) { return uint32_t(c->n_cu) * kMaxRzWavesPerCu; }
uint64_t max_peak_tiles(const hough_ctx *c);

// Exclusive prefix of n uint32 counts into n + 1 uint64 offsets (one
// workgroup for short inputs, three launches for long ones).
uint64_t scan_blocks(uint64_t n);
hipError_t launch_scan_counts(hough_ctx *c, const uint32_t *counts, uint64_t n, uint64_t *offsets,
                              uint64_t stride_out, uint64_t *out_strided, hipStream_t s);
// The same with explicit block-sum scratch (scan_part[blocks_max],
// scan_off[blocks_max + 1]); timed = false skips per-kernel timing.
hipError_t launch_scan_counts(hough_ctx *c, const uint32_t *counts, uint64_t n, uint64_t *offsets,
                              uint64_t stride_out, uint64_t *out_strided, hipStream_t s, uint64_t *scan_part,
                              uint64_t *scan_off, uint64_t blocks_max, bool timed);

// Plateau clusters of a peak list (lock-free union-find, see k_cluster.hip).
uint64_t cluster_blocks(uint64_t n);
hipError_t launch_clusters(hough_ctx *c, const hough_peak *peaks, uint64_t peak_capacity, const uint64_t *poff,
                           uint32_t n_events, uint32_t *labels, hough_cluster *clusters, uint64_t capacity,
                           uint64_t *coff, hipStream_t s);
hipError_t launch_fit(hough_ctx *c, const hough_hits *h, const hough_peak *peaks, uint64_t peak_capacity,
                      const uint64_t *poff, const hough_cluster *clusters, uint64_t capacity, const uint64_t *coff,
                      hough_fit *out, hipStream_t s);
inline uint32_t peak_rows(const hough_ctx *c)
{
    return c->tun.peak_rows ? c->tun.peak_rows : 16u;
}

}  // namespace hough
