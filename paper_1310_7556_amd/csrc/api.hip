// C ABI of the track finder: context lifetime, argument checks, the hot-path
// entry points, HIP-graph capture of the whole path and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "fastdiv.h"
#include "hough_internal.h"

using namespace hough;

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int device_error(hough_ctx *c, hipError_t e, const char *where)
{
    if (c) {
        c->last_error = std::string(where) + ": " + hipGetErrorString(e);
    }
    return HOUGH_EDEVICE;
}

template <typename T>
bool dev_alloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) return true;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)) == hipSuccess;
}

void free_all(hough_ctx *c)
{
    void *ptrs[] = {c->d_O, c->d_V, c->d_Z, c->d_Zl, c->d_rk_info, c->d_rk_sorted, c->d_phi_a, c->d_z_a, c->d_phi_b, c->d_z_b,
                    c->d_layer_off, c->d_bucket_off, c->d_order, c->d_counters, c->d_tile_counts,
                    c->d_tile_off, c->d_cand, c->d_cand_counts, c->d_rz_hist, c->d_redo_list, c->d_gap_info, c->d_gap_list,
                    c->d_scan_part, c->d_scan_off, c->d_dir_tab, c->d_cl_rank, c->d_cl_part,
                    c->d_cl_part_off, c->d_part_cnt, c->d_part_base};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &t : c->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
}

bool hits_ok(const hough_ctx *c, const hough_hits *h, bool need_z)
{
    if (!h) return false;
    if (h->n_events == 0) return true;
    if (!h->event_offsets) return false;
    if (h->n_hits && (!h->layer || !h->phi)) return false;
    if (need_z && h->n_hits && !h->z_um) return false;
    (void)c;
    return true;
}

bool tuning_ok(const hough_ctx *c, const hough_tuning &t)
{
    if (t.vote_rows) {
        if (t.vote_rows > 64 || (t.vote_rows & (t.vote_rows - 1))) return false;
        if (size_t(t.vote_rows) * c->spec.n_phi * 4 > c->max_lds) return false;
    }
    if (t.vote_threads && (t.vote_threads % 64 || t.vote_threads > 1024)) return false;
    if (t.vote_wgs_per_cu > 32) return false;
    if (t.peak_rows > 4096) return false;
    if (t.rz_waves_per_cu > kMaxRzWavesPerCu) return false;
    if (t.vote_algo > 5) return false;
    if (t.vote_algo == 3 && !hough::gap_vote_usable(c)) return false;
    if (t.vote_algo == 4 && !hough::direct_vote_usable(c)) return false;
    if (t.vote_algo == 5 && !c->d_rk_info) return false;
    if (t.vote_items > 2) return false;
    if (t.peak_algo > 2) return false;
    if (t.rz_member_cap && (t.rz_member_cap < 256 || t.rz_member_cap > 4096 ||
                            (t.rz_member_cap & (t.rz_member_cap - 1))))
        return false;
    if (t.rz_redo_list > hough::kRedoListCap) return false;
    if (t.rz_slow_path > 1) return false;
    if (t.rz_counter_bits != 0 && t.rz_counter_bits != 4 && t.rz_counter_bits != 8 && t.rz_counter_bits != 16)
        return false;
    return true;
}

}  // namespace

namespace hough {

void prof_begin(hough_ctx *c, const char *name, hipStream_t s, KernelTimer *t)
{
    t->name = nullptr;
    if (!c->prof || c->capturing) return;
    for (int i = 0; i < 2; ++i) {
        hipEvent_t ev;
        if (c->event_pool.empty()) {
            if (hipEventCreate(&ev) != hipSuccess) return;
        } else {
            ev = c->event_pool.back();
            c->event_pool.pop_back();
        }
        (i ? t->stop : t->start) = ev;
    }
    t->name = name;
    (void)hipEventRecord(t->start, s);
}

void prof_end(hough_ctx *c, hipStream_t s, KernelTimer *t)
{
    if (!t->name) return;
    (void)hipEventRecord(t->stop, s);
    c->pending.push_back(*t);
}

}  // namespace hough

extern "C" {

const char *hough_strerror(int status)
{
    switch (status) {
    case HOUGH_OK: return "ok";
    case HOUGH_EINVAL: return "invalid argument";
    case HOUGH_ENOMEM: return "out of memory";
    case HOUGH_EDEVICE: return "HIP runtime error";
    case HOUGH_ECAPACITY: return "capacity exceeded";
    case HOUGH_ELIMIT: return "call exceeds context limits";
    default: return "unknown status";
    }
}

const char *hough_last_error(const hough_ctx *ctx)
{
    return ctx ? ctx->last_error.c_str() : "";
}

int hough_check_spec(const hough_grid_spec *spec)
{
    return spec && spec_valid(*spec) ? HOUGH_OK : HOUGH_EINVAL;
}

int hough_build_tables(const hough_grid_spec *spec, uint32_t *O, uint8_t *V, size_t nOV,
                       int32_t *Z, size_t nZ)
{
    if (!spec || !spec_valid(*spec) || !O || !V) return HOUGH_EINVAL;
    const size_t need = size_t(spec->n_layers) * spec->n_d0 * spec->n_qpt;
    if (nOV < need) return HOUGH_EINVAL;
    build_offsets(*spec, O, V);
    if (Z) {
        const size_t needz = size_t(spec->n_qpt) * spec->n_layers * spec->n_cot;
        if (!spec->n_z0 || nZ < needz) return HOUGH_EINVAL;
        build_zshift(*spec, Z);
    }
    return HOUGH_OK;
}

int hough_create(const hough_grid_spec *spec, const hough_limits *limits, int device, hough_ctx **out)
{
    if (!out) return HOUGH_EINVAL;
    *out = nullptr;
    if (!spec || !limits || !spec_valid(*spec)) return HOUGH_EINVAL;
    if (limits->max_events < 1 || limits->max_hits >= (uint64_t(1) << 32) || limits->max_peaks >= (uint64_t(1) << 32))
        return HOUGH_EINVAL;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return HOUGH_EINVAL;
    DeviceGuard guard(device);

    hough_ctx *c = new (std::nothrow) hough_ctx;
    if (!c) return HOUGH_ENOMEM;
    c->spec = *spec;
    c->lim = *limits;
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->n_cu = cus;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = std::min<size_t>(size_t(lds) - 512, 65536);   // headroom for static LDS
    c->max_lds_direct = c->max_lds;
    // the rank vote may use up to half of a compute unit's LDS (two of its
    // 512-thread workgroups per compute unit)
    if (lds > 0) c->max_lds_rank = std::max<size_t>(c->max_lds, std::min<size_t>(size_t(lds) - 512, 81920));
    while ((1u << c->log2_phi) < spec->n_phi) ++c->log2_phi;
    c->shift = 32 - c->log2_phi;
    c->rows = spec->n_d0 * spec->n_qpt;
    c->cells = uint64_t(c->rows) * spec->n_phi;
    const bool rz = spec->n_z0 > 0;
    // azimuth buckets: member search of the rz stage and of the cluster fit
    const bool buckets = rz || limits->max_peaks > 0;
    c->bucket_bits = buckets ? std::min(c->log2_phi + 2, kMaxBucketBits) : 0;

    // host tables
    const size_t nOV = size_t(spec->n_layers) * c->rows;
    std::vector<uint32_t> O(nOV);
    std::vector<uint8_t> V(nOV);
    build_offsets(*spec, O.data(), V.data());
    c->all_valid = std::all_of(V.begin(), V.end(), [](uint8_t v) { return v != 0; });
    std::vector<int32_t> Z, Zl;
    if (rz) {
        Z.resize(size_t(spec->n_qpt) * spec->n_layers * spec->n_cot);
        build_zshift(*spec, Z.data());
        // fast rz path: with zl = Z + z0_lo in [-2^31, 2^31 - span], the
        // uint32 difference u = z - zl is < span exactly when 0 <= z - zl <
        // span for every int32 z; the bin is then one multiply-high
        const int64_t span = int64_t(spec->z0_hi_um) - int64_t(spec->z0_lo_um);
        const BinMagic bm = make_binmagic_min(uint64_t(span), spec->n_z0);
        bool ok = bm.ok;
        // stored [k][j][16 layers] so that a lane (one cot bin) reads all
        // its layers' values as 64 contiguous bytes; layers past n_layers
        // hold 0 (the fast kernel's padding members use layer 15)
        Zl.assign(size_t(spec->n_qpt) * spec->n_cot * kMaxLayers, 0);
        for (uint32_t k = 0; ok && k < spec->n_qpt; ++k)
            for (uint32_t l = 0; ok && l < spec->n_layers; ++l)
                for (uint32_t j = 0; ok && j < spec->n_cot; ++j) {
                    const size_t i = (size_t(k) * spec->n_layers + l) * spec->n_cot + j;
                    const int64_t zl = int64_t(Z[i]) + spec->z0_lo_um;
                    ok = zl >= INT32_MIN && zl <= int64_t(INT32_MAX) + 1 - span;
                    Zl[(size_t(k) * spec->n_cot + j) * kMaxLayers + l] = int32_t(zl);
                }
        c->rz_fast = ok && spec->n_layers < kMaxLayers;
        c->rz_magic_m = bm.m;
        c->rz_magic_s = bm.s;
        if (!c->rz_fast) Zl.clear();
    }

    std::vector<uint32_t> rk_info, rk_sorted;
    if (rank_vote_form(*spec)) build_rank_tables(*spec, c->rows, c->shift, O.data(), V.data(), rk_info, rk_sorted);

    const uint64_t H = limits->max_hits ? limits->max_hits : 1;
    const uint32_t E = limits->max_events;
    const uint32_t L = spec->n_layers;
    c->n_peak_tiles = std::max<uint64_t>(uint64_t(E) * c->rows, E);
    c->scan_blocks_max = scan_blocks(c->n_peak_tiles);
    // split_parts keeps E * K <= E + kSplitPartsPerCu * n_cu (K <= ceil(4 n_cu / E))
    c->max_parts = uint64_t(E) + uint64_t(kSplitPartsPerCu) * c->n_cu;
    const size_t nb = buckets ? (size_t(1) << c->bucket_bits) + 1 : 0;
    const size_t ncand = rz ? size_t(E) * spec->rz_max_candidates : 0;
    const size_t rzh = rz ? size_t(c->n_cu) * kMaxRzWavesPerCu * spec->n_z0 : 0;
    bool ok = dev_alloc(&c->d_O, nOV + kOPad) && dev_alloc(&c->d_V, nOV) && dev_alloc(&c->d_Z, Z.size()) &&
              dev_alloc(&c->d_Zl, Zl.size()) &&
              dev_alloc(&c->d_phi_a, H) && dev_alloc(&c->d_z_a, rz ? H : 0) &&
              dev_alloc(&c->d_phi_b, buckets ? H : 0) && dev_alloc(&c->d_z_b, rz ? H : 0) &&
              dev_alloc(&c->d_layer_off, size_t(E) * (L + 1)) &&
              dev_alloc(&c->d_bucket_off, size_t(E) * L * nb) && dev_alloc(&c->d_order, E) &&
              dev_alloc(&c->d_counters, kCounterDwords) && dev_alloc(&c->d_tile_counts, c->n_peak_tiles) &&
              dev_alloc(&c->d_tile_off, c->n_peak_tiles + 1) && dev_alloc(&c->d_cand, ncand) &&
              dev_alloc(&c->d_cand_counts, E) && dev_alloc(&c->d_rz_hist, rzh) &&
              dev_alloc(&c->d_redo_list, rz ? kRedoListCap : 0) &&
              dev_alloc(&c->d_part_cnt, c->max_parts * kSplitBins) &&
              dev_alloc(&c->d_part_base, c->max_parts * kSplitBins) &&
              dev_alloc(&c->d_gap_info, size_t(E) * L) && dev_alloc(&c->d_gap_list, H) &&
              dev_alloc(&c->d_scan_part, c->scan_blocks_max) && dev_alloc(&c->d_scan_off, c->scan_blocks_max + 1) &&
              dev_alloc(&c->d_dir_tab, size_t(E) * L * spec->n_phi) &&
              dev_alloc(&c->d_cl_rank, limits->max_peaks) &&
              dev_alloc(&c->d_cl_part, cluster_blocks(limits->max_peaks)) &&
              dev_alloc(&c->d_cl_part_off, cluster_blocks(limits->max_peaks) + 1) &&
              dev_alloc(&c->d_rk_info, rk_info.size()) && dev_alloc(&c->d_rk_sorted, rk_sorted.size());
    if (!ok) {
        free_all(c);
        delete c;
        return HOUGH_ENOMEM;
    }
    hipError_t err = hipMemset(c->d_O, 0, (nOV + kOPad) * 4);
    if (err == hipSuccess) err = hipMemcpy(c->d_O, O.data(), nOV * 4, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(c->d_V, V.data(), nOV, hipMemcpyHostToDevice);
    if (err == hipSuccess && rz) err = hipMemcpy(c->d_Z, Z.data(), Z.size() * 4, hipMemcpyHostToDevice);
    if (err == hipSuccess && !Zl.empty())
        err = hipMemcpy(c->d_Zl, Zl.data(), Zl.size() * 4, hipMemcpyHostToDevice);
    if (err == hipSuccess && rzh) err = hipMemset(c->d_rz_hist, 0, rzh * 4);
    if (err == hipSuccess && !rk_info.empty())
        err = hipMemcpy(c->d_rk_info, rk_info.data(), rk_info.size() * 4, hipMemcpyHostToDevice);
    if (err == hipSuccess && !rk_sorted.empty())
        err = hipMemcpy(c->d_rk_sorted, rk_sorted.data(), rk_sorted.size() * 4, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemset(c->d_counters, 0, kCounterDwords * 4);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    // the static scratch of hough_peaks_noalloc: its address on this device,
    // looked up once per device (a failure is reported by that call)
    if (err == hipSuccess) (void)noalloc_scratch_init(device);
    if (err != hipSuccess) {
        free_all(c);
        delete c;
        return HOUGH_EDEVICE;
    }
    *out = c;
    return HOUGH_OK;
}

void hough_destroy(hough_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    free_all(ctx);
    delete ctx;
}

int hough_vote(hough_ctx *ctx, const hough_hits *hits, uint16_t *acc, void *stream)
{
    if (!ctx || !hits_ok(ctx, hits, false) || (hits->n_events && !acc)) return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(acc) & 3) return HOUGH_EINVAL;
    if (hits->n_events > ctx->lim.max_events || hits->n_hits > ctx->lim.max_hits) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_vote(ctx, hits, acc, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_vote");
}

int hough_peaks(hough_ctx *ctx, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                uint64_t capacity, uint64_t *event_peak_offsets, void *stream)
{
    if (!ctx || !event_peak_offsets || (n_events && !acc) || (capacity && !peaks)) return HOUGH_EINVAL;
    if (n_events > ctx->lim.max_events) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_peaks(ctx, acc, n_events, peaks, capacity, event_peak_offsets,
                                      static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_peaks");
}

int hough_peaks_noalloc(hough_ctx *ctx, const uint16_t *acc, uint32_t n_events, hough_peak *peaks,
                        uint64_t capacity, uint64_t *event_peak_offsets, void *stream)
{
    if (!ctx || !event_peak_offsets || (n_events && !acc) || (capacity && !peaks)) return HOUGH_EINVAL;
    if (n_events > ctx->lim.max_events) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    void *base = noalloc_scratch(ctx->device);
    if (!base) {
        const hipError_t e = noalloc_scratch_init(ctx->device);
        base = noalloc_scratch(ctx->device);
        if (!base) return device_error(ctx, e, "hough_peaks_noalloc: address of the static scratch");
    }
    const uint64_t tiles = peak_items(ctx, n_events, acc);
    if (n_events && tiles == 0) return device_error(ctx, hipErrorInvalidConfiguration, "hough_peaks_noalloc");
    const size_t need = peak_scratch_bytes(tiles);
    if (need > kNoAllocScratchBytes) {
        ctx->last_error = "hough_peaks_noalloc: " + std::to_string(tiles) + " peak tiles need " +
                          std::to_string(need) + " bytes of static scratch, more than its " +
                          std::to_string(kNoAllocScratchBytes);
        return HOUGH_ELIMIT;
    }
    const hipError_t e = launch_peaks(ctx, acc, n_events, peaks, capacity, event_peak_offsets,
                                      static_cast<hipStream_t>(stream), carve_peak_scratch(base, tiles), false);
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_peaks_noalloc");
}

int hough_vote_count(hough_ctx *ctx, const hough_hits *hits, uint32_t *counts, void *stream)
{
    if (!ctx || !hits_ok(ctx, hits, false) || (hits->n_events && !counts)) return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(counts) & 3) return HOUGH_EINVAL;
    if (hits->n_events > ctx->lim.max_events || hits->n_hits > ctx->lim.max_hits) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_vote_count(ctx, hits, counts, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_vote_count");
}

int hough_peaks_count(hough_ctx *ctx, const uint32_t *counts, uint32_t n_events, hough_count_peak *peaks,
                      uint64_t capacity, uint64_t *event_peak_offsets, void *stream)
{
    if (!ctx || !event_peak_offsets || (n_events && !counts) || (capacity && !peaks)) return HOUGH_EINVAL;
    if (n_events > ctx->lim.max_events) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_peaks_count(ctx, counts, n_events, reinterpret_cast<uint2 *>(peaks), capacity,
                                            event_peak_offsets, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_peaks_count");
}

int hough_peak_clusters(hough_ctx *ctx, const hough_peak *peaks, uint64_t peak_capacity,
                        const uint64_t *event_peak_offsets, uint32_t n_events, uint32_t *peak_cluster,
                        hough_cluster *clusters, uint64_t capacity, uint64_t *event_cluster_offsets,
                        void *stream)
{
    if (!ctx || !event_peak_offsets || !event_cluster_offsets || (peak_capacity && (!peaks || !peak_cluster)) ||
        (capacity && !clusters))
        return HOUGH_EINVAL;
    if ((reinterpret_cast<uintptr_t>(peaks) & 7) || (reinterpret_cast<uintptr_t>(clusters) & 7) ||
        (reinterpret_cast<uintptr_t>(peak_cluster) & 3))
        return HOUGH_EINVAL;
    if (n_events > ctx->lim.max_events || peak_capacity > ctx->lim.max_peaks) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_clusters(ctx, peaks, peak_capacity, event_peak_offsets, n_events, peak_cluster,
                                         clusters, capacity, event_cluster_offsets, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_peak_clusters");
}

int hough_cluster_fit(hough_ctx *ctx, const hough_hits *hits, const hough_peak *peaks, uint64_t peak_capacity,
                      const uint64_t *event_peak_offsets, const hough_cluster *clusters, uint64_t capacity,
                      const uint64_t *event_cluster_offsets, hough_fit *out, void *stream)
{
    if (!ctx || ctx->spec.n_d0 != 1 || !hits_ok(ctx, hits, false) || !event_peak_offsets ||
        !event_cluster_offsets || (peak_capacity && !peaks) || (capacity && (!clusters || !out)))
        return HOUGH_EINVAL;
    if ((reinterpret_cast<uintptr_t>(peaks) & 7) || (reinterpret_cast<uintptr_t>(clusters) & 7) ||
        (reinterpret_cast<uintptr_t>(out) & 7))
        return HOUGH_EINVAL;
    // the member search reads the (layer, azimuth bucket) index, which the
    // context keeps only with an rz grid or limits.max_peaks > 0
    if (ctx->bucket_bits == 0 || !ctx->d_phi_b || !ctx->d_bucket_off) return HOUGH_EINVAL;
    if (hits->n_events > ctx->lim.max_events || hits->n_hits > ctx->lim.max_hits) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_fit(ctx, hits, peaks, peak_capacity, event_peak_offsets, clusters, capacity,
                                    event_cluster_offsets, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_cluster_fit");
}

int hough_rz_refine(hough_ctx *ctx, const hough_hits *hits, const hough_peak *peaks,
                    uint64_t peak_capacity, const uint64_t *event_peak_offsets, hough_rz *out,
                    uint64_t capacity, uint64_t *event_rz_offsets, void *stream)
{
    if (!ctx || !ctx->spec.n_z0 || !hits_ok(ctx, hits, true) || !event_peak_offsets ||
        !event_rz_offsets || (peak_capacity && !peaks) || (capacity && !out))
        return HOUGH_EINVAL;
    if (hits->n_events > ctx->lim.max_events || hits->n_hits > ctx->lim.max_hits) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    const hipError_t e = launch_rz(ctx, hits, peaks, peak_capacity, event_peak_offsets, out, capacity,
                                   event_rz_offsets, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(ctx, e, "hough_rz_refine");
}

struct hough_graph {
    hough_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int hough_graph_capture(hough_ctx *ctx, const hough_hits *hits, uint16_t *acc, hough_peak *peaks,
                        uint64_t peak_capacity, uint64_t *event_peak_offsets, hough_rz *rz_out,
                        uint64_t rz_capacity, uint64_t *event_rz_offsets, void *stream,
                        hough_graph **out)
{
    if (!out) return HOUGH_EINVAL;
    *out = nullptr;
    const bool with_rz = rz_out != nullptr || event_rz_offsets != nullptr;
    if (!ctx || !stream || !hits_ok(ctx, hits, with_rz) || !acc || !event_peak_offsets ||
        (peak_capacity && !peaks) || (with_rz && (!ctx->spec.n_z0 || !event_rz_offsets)))
        return HOUGH_EINVAL;
    if (hits->n_events > ctx->lim.max_events || hits->n_hits > ctx->lim.max_hits) return HOUGH_ELIMIT;
    DeviceGuard guard(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hough_graph *g = new (std::nothrow) hough_graph;
    if (!g) return HOUGH_ENOMEM;
    g->ctx = ctx;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return device_error(ctx, e, "hipStreamBeginCapture");
    }
    ctx->capturing = true;
    hipError_t le = launch_vote(ctx, hits, acc, s);
    if (le == hipSuccess) le = launch_peaks(ctx, acc, hits->n_events, peaks, peak_capacity, event_peak_offsets, s);
    if (le == hipSuccess && with_rz)
        le = launch_rz(ctx, hits, peaks, peak_capacity, event_peak_offsets, rz_out, rz_capacity,
                       event_rz_offsets, s);
    ctx->capturing = false;
    e = hipStreamEndCapture(s, &g->graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return device_error(ctx, le != hipSuccess ? le : e, "graph capture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return device_error(ctx, e, "hipGraphInstantiate");
    }
    *out = g;
    return HOUGH_OK;
}

int hough_graph_launch(hough_graph *graph, void *stream)
{
    if (!graph || !graph->exec) return HOUGH_EINVAL;
    DeviceGuard guard(graph->ctx->device);
    const hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : device_error(graph->ctx, e, "hipGraphLaunch");
}

void hough_graph_destroy(hough_graph *graph)
{
    if (!graph) return;
    DeviceGuard guard(graph->ctx->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

int hough_gather_events(const uint8_t *src_layer, const uint32_t *src_phi, const int32_t *src_z,
                        const uint64_t *src_off, const uint64_t *len, const uint64_t *dst_off,
                        uint32_t n, uint8_t *dst_layer, uint32_t *dst_phi, int32_t *dst_z,
                        uint64_t dst_capacity, void *stream)
{
    if (n && (!src_layer || !src_phi || !src_off || !len || !dst_off || !dst_layer || !dst_phi))
        return HOUGH_EINVAL;
    if ((src_z == nullptr) != (dst_z == nullptr)) return HOUGH_EINVAL;
    const hipError_t e = launch_gather_events(src_layer, src_phi, src_z, src_off, len, dst_off, n, dst_layer,
                                              dst_phi, dst_z, dst_capacity, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_get_tables(const hough_ctx *ctx, uint32_t *O, uint8_t *V, size_t nOV, int32_t *Z, size_t nZ,
                     int32_t *Zl, size_t nZl)
{
    if (!ctx) return HOUGH_EINVAL;
    const hough_grid_spec &g = ctx->spec;
    const size_t need = size_t(g.n_layers) * ctx->rows;
    const size_t needz = g.n_z0 ? size_t(g.n_qpt) * g.n_layers * g.n_cot : 0;
    if ((O && nOV < need) || (V && nOV < need)) return HOUGH_EINVAL;
    if (Z && (!g.n_z0 || nZ < needz)) return HOUGH_EINVAL;
    // the (Z + z0_lo) copy exists only when the rz stage takes its 32-bit path
    if (Zl && (!ctx->rz_fast || !ctx->d_Zl || nZl < needz)) return HOUGH_EINVAL;
    DeviceGuard guard(ctx->device);
    hipError_t e = hipSuccess;
    if (O) e = hipMemcpy(O, ctx->d_O, need * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && V) e = hipMemcpy(V, ctx->d_V, need, hipMemcpyDeviceToHost);
    if (e == hipSuccess && Z) e = hipMemcpy(Z, ctx->d_Z, needz * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && Zl) {
        // the device copy is [k][j][16 layers]; return it as [k][l][j]
        std::vector<int32_t> t(size_t(g.n_qpt) * g.n_cot * kMaxLayers);
        e = hipMemcpy(t.data(), ctx->d_Zl, t.size() * 4, hipMemcpyDeviceToHost);
        for (uint32_t k = 0; e == hipSuccess && k < g.n_qpt; ++k)
            for (uint32_t l = 0; l < g.n_layers; ++l)
                for (uint32_t j = 0; j < g.n_cot; ++j)
                    Zl[(size_t(k) * g.n_layers + l) * g.n_cot + j] = t[(size_t(k) * g.n_cot + j) * kMaxLayers + l];
    }
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_set_tuning(hough_ctx *ctx, const hough_tuning *tuning)
{
    if (!ctx || !tuning || !tuning_ok(ctx, *tuning)) return HOUGH_EINVAL;
    ctx->tun = *tuning;
    return HOUGH_OK;
}

int hough_get_tuning(const hough_ctx *ctx, hough_tuning *tuning)
{
    if (!ctx || !tuning) return HOUGH_EINVAL;
    *tuning = ctx->tun;
    return HOUGH_OK;
}

int hough_set_profiling(hough_ctx *ctx, int enable)
{
    if (!ctx) return HOUGH_EINVAL;
    ctx->prof = enable != 0;
    return HOUGH_OK;
}

int hough_kernel_times(hough_ctx *ctx, const char **names, uint64_t *launches, double *total_ms, int n)
{
    if (!ctx) return HOUGH_EINVAL;
    DeviceGuard guard(ctx->device);
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(t.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            auto it = std::find_if(ctx->stats.begin(), ctx->stats.end(),
                                   [&](const KernelStat &s) { return s.name == t.name; });
            if (it == ctx->stats.end()) {
                ctx->stats.push_back(KernelStat{t.name, 0, 0.0});
                it = ctx->stats.end() - 1;
            }
            it->launches += 1;
            it->total_ms += ms;
        }
        ctx->event_pool.push_back(t.start);
        ctx->event_pool.push_back(t.stop);
    }
    ctx->pending.clear();
    const int m = int(ctx->stats.size());
    for (int i = 0; i < m && i < n; ++i) {
        if (names) names[i] = ctx->stats[i].name.c_str();
        if (launches) launches[i] = ctx->stats[i].launches;
        if (total_ms) total_ms[i] = ctx->stats[i].total_ms;
    }
    return m;
}

void hough_kernel_times_reset(hough_ctx *ctx)
{
    if (!ctx) return;
    (void)hough_kernel_times(ctx, nullptr, nullptr, nullptr, 0);
    ctx->stats.clear();
}

int hough_device_cus(const hough_ctx *ctx)
{
    return ctx ? ctx->n_cu : 0;
}

}  // extern "C"
