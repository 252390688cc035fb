/*
 * hough.h -- C ABI of the MI355X (gfx950) Hough-transform track finder.
 *
 * The paper's method (Section 4, "Hough Transform Algorithm") has two steps:
 * every hit adds votes to the cells of a discretised (curvature, azimuth)
 * parameter space that are consistent with it, and cells with many votes are
 * then found as local maxima of that space.  This library computes:
 *
 *   hough_vote       step 1: per event, a uint16 layer-bitmask accumulator
 *                    A[d0][q/pT][phi0] (a cell holds the OR of 1 << layer of
 *                    every hit voting into it; its vote count is the popcount)
 *   hough_peaks      step 2: cells with popcount >= threshold that are >= all
 *                    neighbours in their 3x3 (q/pT, phi0) window, 3x3x3 with
 *                    a d0 axis; phi0 wraps, q/pT and d0 do not
 *   hough_rz_refine  the confirmation step the paper leaves to "more
 *                    expensive computations" (end of the first paragraph of
 *                    Section 4): per candidate cell, its member hits vote in
 *                    a (cot theta, z0) grid and the argmax is reported
 *
 * Geometry.  Curvature rho = 0.299792458e-3 * b_tesla * q/pT [1/mm]; B along
 * +z; positive q/pT bends clockwise.  A track with perigee (d0, phi0) crosses
 * radius r at phi = phi0 + asin((d0 - rho (r^2 + d0^2)/2) / (r (1 - rho d0))).
 * Angles are uint32 turn fractions (2^32 == one full turn); phi0 bin p covers
 * [p, p+1) * 2^32 / n_phi.  The library tabulates, once per context in FP64
 * on the host, O[l][d][k] = llround(asin(arg) / 2pi * 2^32) for the bin-centre
 * track of row (d, k) at layer radius l, so a vote is one subtract and one
 * shift: p = (phi - O[l][d][k]) >> (32 - log2 n_phi).  Rows whose layer is
 * unreachable (1 - rho d0 <= 0 or |arg| > 1) receive no vote.  The rz stage
 * uses Z[k][l][j] = llround(cot_j * s_l(k) * 1000) um with s = (2/rho)
 * asin(rho r / 2) the transverse arc length (s = r when rho == 0), then
 * z0 = z - Z and z0 bin b = floor((z0 - z0_lo) * n_z0 / (z0_hi - z0_lo)).
 * Bin centres: kappa_k = qpt_lo + (k + 0.5) (qpt_hi - qpt_lo) / n_qpt, and
 * likewise for d0 (d0 = 0 exactly when n_d0 == 1) and cot.
 *
 * Conventions for every call below:
 *   - Pointers named "device" are HIP device pointers; everything else is host.
 *   - Stream arguments are hipStream_t values passed as void* (NULL = the
 *     null stream).  Calls enqueue work on that stream and return without
 *     waiting for it; argument checks happen synchronously, before anything
 *     is enqueued.  The hot calls allocate nothing and never synchronise the
 *     host, so they may be captured into a HIP graph.
 *   - The caller owns every hit, accumulator and output buffer.  The context
 *     owns its tables and scratch, sized at hough_create from hough_limits;
 *     calls that share a context must not overlap in time (one stream per
 *     context, or external ordering).
 *   - Return value: HOUGH_OK (0) or a negative hough_status; on
 *     HOUGH_EDEVICE the HIP error text is kept for hough_last_error().
 */
#ifndef HOUGH_H
#define HOUGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HOUGH_OK = 0,
    HOUGH_EINVAL = -1,      /* invalid spec, limits or argument */
    HOUGH_ENOMEM = -2,      /* device or host allocation failed at create */
    HOUGH_EDEVICE = -3,     /* a HIP runtime call failed */
    HOUGH_ECAPACITY = -4,   /* reserved: capacity overflow is reported through offsets */
    HOUGH_ELIMIT = -5       /* call exceeds the limits given at hough_create */
} hough_status;

typedef struct hough_ctx hough_ctx;
typedef struct hough_graph hough_graph;

/* Parameter-space grid.  Accumulator rows are (d, k) pairs, d-major; a row
 * holds n_phi cells.  Cell index = (d * n_qpt + k) * n_phi + p. */
typedef struct {
    uint32_t n_layers;              /* 1..16; bit l of a mask = layer l */
    double   layer_r_mm[16];        /* strictly ascending, > 0 */
    double   b_tesla;
    uint32_t n_qpt;                 /* >= 1 */
    double   qpt_lo, qpt_hi;        /* q/pT range, 1/GeV */
    uint32_t n_phi;                 /* power of two, 2..65536 */
    uint32_t n_d0;                  /* >= 1; 1 means prompt (d0 = 0) */
    double   d0_lo_mm, d0_hi_mm;
    uint32_t threshold;             /* peak needs popcount >= threshold */
    uint32_t n_z0;                  /* 0 disables the rz stage; else 1..65535 */
    int32_t  z0_lo_um, z0_hi_um;    /* z0_hi > z0_lo */
    uint32_t n_cot;                 /* 1..65535 when n_z0 > 0 */
    double   cot_lo, cot_hi;
    uint32_t rz_max_candidates;     /* 0: every peak; else the first this many
                                       peaks by (popcount desc, cell asc) */
} hough_grid_spec;

/* Upper bounds of any single call, fixing the context's scratch. */
typedef struct {
    uint32_t max_events;            /* events per call, >= 1 */
    uint64_t max_hits;              /* hits per call (all events), < 2^32 */
    uint64_t max_peaks;             /* largest peak_capacity hough_peak_clusters accepts (< 2^32;
                                       the context keeps 4 bytes of scratch per peak); 0 when
                                       that call is not used */
} hough_limits;

/* Hits of n_events events, concatenated (structure of arrays). */
typedef struct {
    const uint8_t  *layer;          /* device [n_hits]; values >= n_layers are ignored */
    const uint32_t *phi;            /* device [n_hits]; uint32 turn fraction */
    const int32_t  *z_um;           /* device [n_hits]; z in micrometres (rz only, else may be NULL) */
    const uint64_t *event_offsets;  /* device [n_events + 1]; event e = [off[e], off[e+1]);
                                       out-of-range offsets are clamped to [0, n_hits] */
    uint32_t n_events;              /* host copy */
    uint64_t n_hits;                /* host copy */
} hough_hits;

/* One local maximum. */
typedef struct {
    uint32_t cell;                  /* index within its event's accumulator */
    uint16_t mask;                  /* the cell's layer mask */
    uint16_t popcount;              /* number of layers in the mask */
} hough_peak;

/* One local maximum of a counting accumulator (hough_peaks_count). */
typedef struct {
    uint32_t cell;                  /* (d * n_qpt + k) * n_phi + p within its event */
    uint32_t count;                 /* the cell's vote count */
} hough_count_peak;

/* One rz refinement result. */
typedef struct {
    uint32_t peak;                  /* index of the candidate in its event's peak list */
    uint16_t cot_bin, z0_bin;       /* argmax; ties -> smallest cot bin, then z0 bin */
    uint32_t count;                 /* member votes in that (cot, z0) bin */
    uint32_t n_members;             /* hits that voted into the candidate's cell */
} hough_rz;

/* One plateau cluster (hough_peak_clusters).  Offsets are taken from the
 * cluster's first peak (d_f, k_f, p_f); the centroid in bin coordinates is
 * (d_f + sum_dd / n_peaks, k_f + sum_dk / n_peaks, p_f + sum_dp / n_peaks
 * modulo n_phi).  24 bytes, 8-byte aligned arrays. */
typedef struct {
    uint32_t first;                 /* index in its event's peak list of the member with the
                                       smallest cell */
    uint16_t popcount;              /* the members' popcount (adjacent local maxima are equal) */
    uint16_t mask_or;               /* OR of the members' layer masks */
    uint32_t n_peaks;               /* members */
    int32_t  sum_dk;                /* sum over members of k - k_f */
    int32_t  sum_dp;                /* sum over members of (p - p_f) mod n_phi, taken in
                                       [-n_phi/2, n_phi/2) */
    int32_t  sum_dd;                /* sum over members of d - d_f */
} hough_cluster;

/* Helix fit of one plateau cluster (hough_cluster_fit).  80 bytes. */
typedef struct {
    double   qpt;                   /* fitted q/pT, 1/GeV (0 when status == 0) */
    double   phi0;                  /* fitted phi0, radians in [0, 2 pi) (0 when status == 0) */
    double   qpt_c;                 /* q/pT at the cluster centroid (bin-centre formula) */
    double   phi0_c;                /* phi0 at the cluster centroid, radians in [0, 2 pi) */
    double   rms_mm;                /* rms residual of the members, mm (0 when status == 0) */
    double   cot;                   /* fitted cot(theta) (0 when status_z == 0) */
    double   z0_mm;                 /* fitted z0, mm (0 when status_z == 0) */
    double   rms_z_mm;              /* rms of the members' z residuals, mm (0 when status_z == 0) */
    uint32_t n_hits;                /* members: hits that voted into the first peak's cell */
    uint32_t status;                /* 1 = fitted; 0 = fewer than 3 members or singular */
    uint32_t status_z;              /* 1 = line fitted (grids with an rz stage, z given) */
    uint32_t reserved;
} hough_fit;

/* Autotuning knobs of the kernels (all 0 = library default). */
typedef struct {
    uint32_t vote_rows;             /* accumulator rows per LDS tile */
    uint32_t vote_threads;          /* threads per vote workgroup (multiple of 64, <= 1024) */
    uint32_t vote_wgs_per_cu;       /* persistent vote grid: workgroups per compute unit */
    uint32_t peak_rows;             /* accumulator rows per peak-finding tile (per wavefront strip in
                                       peak form 2) */
    uint32_t rz_waves_per_cu;       /* persistent rz grid: waves per compute unit */
    uint32_t vote_algo;             /* 0 = default (5 where usable, else 4), 1 = per-hit LDS atomics,
                                       2 = global atomics, 3 = hit-gap lists, 4 = bucket bounds (direct
                                       occupancy), 5 = bucket bounds in tile rank space, four cells per
                                       operation (n_phi 256, 512 or 1024; accumulator 8-byte aligned,
                                       else form 4 is used) */
    uint32_t rz_slow_path;          /* 1 forces the global-memory histogram path of the rz vote */
    uint32_t rz_counter_bits;       /* rz LDS counter width: 0 = automatic, 4, 8 or 16 */
    uint32_t vote_items;            /* vote form 5: 0 = automatic, 1 = a whole event per workgroup (bucket
                                       bounds found in LDS; grids of at most 1024 rows whose tables fit in
                                       LDS, else as 2), 2 = one row tile per workgroup (bounds from a table
                                       pass over the hits) */
    uint32_t peak_algo;             /* peak search: 0 = default (2 where usable, else 1), 1 = tiles staged
                                       in LDS, 2 = row window in registers (n_phi 256, 512 or 1024,
                                       accumulator 16-byte aligned, 8 for n_phi 256) */
    uint32_t rz_member_cap;         /* rz: members a candidate may have on the fast path (a power of two,
                                       256 to 4096; more go to the exact path); 0 = 112 with 4-bit
                                       counters, else as many as fit the LDS budget (at most 2048) */
    uint32_t rz_redo_list;          /* rz: capacity of the list of candidates left to the exact path
                                       (1 to 65536, 0 = 65536); when more are left, the exact-path kernel
                                       scans every record for them instead */
} hough_tuning;

/* ---- context --------------------------------------------------------- */

/* Validates the spec (rules in the field comments; the rz stage needs
 * n_d0 == 1), builds the FP64 tables on the host, allocates tables and
 * scratch on `device` and uploads the tables (a blocking host-to-device
 * copy, done once).  *out receives the context; nothing is allocated on
 * failure.  Returns HOUGH_EINVAL, HOUGH_ENOMEM or HOUGH_EDEVICE on error.
 * The tables carry what Section 6.1 lists among the GPU optimisations,
 * keeping expensive trigonometric functions out of the kernels: every asin
 * of the vote and of the rz stage is evaluated here, once.  The context then
 * stays resident on the device across calls, the data persistence that
 * Section 6.2 uses to avoid re-allocating for every frame offloaded. */
int hough_create(const hough_grid_spec *spec, const hough_limits *limits,
                 int device, hough_ctx **out);

/* Frees the context's device memory (the resident tables and scratch of
 * hough_create, Section 6.2).  NULL is accepted.  Work still enqueued with
 * this context must have completed. */
void hough_destroy(hough_ctx *ctx);

/* ---- hot path ---------------------------------------------------------- */

/* Step 1, voting (Section 4: increment the voxels each hit maps to; the
 * Discussion's A[B[i]] += 1 in its layer-mask form).  For every event e,
 * every hit h of e with layer l < n_layers and every reachable row (d, k):
 *     acc[e][d][k][(phi_h - O[l][d][k]) >> (32 - log2 n_phi)] |= 1 << l.
 * acc: device, n_events * n_d0 * n_qpt * n_phi uint16, 4-byte aligned
 * (HOUGH_EINVAL otherwise), fully overwritten (no need to clear it).  Requires n_events <= max_events and
 * n_hits <= max_hits (HOUGH_ELIMIT).  hits->z_um is not read. */
int hough_vote(hough_ctx *ctx, const hough_hits *hits, uint16_t *acc, void *stream);

/* Step 2, local maxima (Section 4: finding cells with many votes amounts to
 * looking for local maxima).  A cell c of event e is a peak iff
 * popcount(acc[c]) >= threshold and popcount(acc[c]) >= popcount of each
 * neighbour (3x3 in (q/pT, phi0), 3x3x3 when n_d0 > 1; phi0 periodic,
 * missing q/pT or d0 neighbours ignored).  Peaks of event 0, then event 1,
 * ..., each in ascending cell order, are written to `peaks` (device,
 * `capacity` records); event e's peaks are [off[e], off[e+1]) with
 * off = event_peak_offsets (device, n_events + 1 uint64, written by the
 * call).  When the total exceeds capacity, records past capacity are dropped
 * and the offsets still hold the true counts: compare off[n_events] with
 * capacity after the stream completes. */
int hough_peaks(hough_ctx *ctx, const uint16_t *acc, uint32_t n_events,
                hough_peak *peaks, uint64_t capacity, uint64_t *event_peak_offsets,
                void *stream);

/* hough_peaks for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results from the same kernels, but the peak search's scratch
 * (per-tile peak counts, their prefix and the scan's block sums) lives in
 * one static device array of 8 MiB per GPU, held until the process ends,
 * instead of the context's buffers.  The call itself allocates nothing
 * (host or device) and records no per-kernel timing.  A call needing more
 * than 8 MiB (about 12 bytes per peak tile, a tile being peak_rows rows of
 * one d0 plane of one event: some 690,000 tiles) returns HOUGH_ELIMIT, with
 * the sizes in hough_last_error.  Every noalloc call on one GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (from any context
 * or stream) race; a call needs nothing from the array's earlier contents. */
int hough_peaks_noalloc(hough_ctx *ctx, const uint16_t *acc, uint32_t n_events,
                        hough_peak *peaks, uint64_t capacity, uint64_t *event_peak_offsets,
                        void *stream);

/* Step 1 in the paper's counting form (the Discussion's A[B[i]] += 1): for
 * every event e, every hit h of e with layer l < n_layers and every
 * reachable row (d, k):
 *     counts[e][d][k][(phi_h - O[l][d][k]) >> (32 - log2 n_phi)] += 1.
 * counts: device, n_events * n_d0 * n_qpt * n_phi uint32, fully overwritten.
 * Each cell counts every hit that falls in it (several hits of one layer
 * count several times), unlike the layer mask of hough_vote.  Limits and
 * errors as hough_vote; hits->z_um is not read.  Per-hit LDS atomics (or
 * global atomics for rows too wide for an LDS tile); tuned by vote_rows,
 * vote_threads and vote_wgs_per_cu (vote_algo 2 forces global atomics). */
int hough_vote_count(hough_ctx *ctx, const hough_hits *hits, uint32_t *counts, void *stream);

/* Step 2 on a counting accumulator: a cell of event e is a peak iff its count
 * is >= threshold and >= the count of each neighbour (same neighbourhood,
 * periodicity and boundaries as hough_peaks).  Records {cell, count} in
 * ascending cell order per event into `peaks` (device, `capacity` records);
 * offsets and capacity overflow as hough_peaks. */
int hough_peaks_count(hough_ctx *ctx, const uint32_t *counts, uint32_t n_events,
                      hough_count_peak *peaks, uint64_t capacity, uint64_t *event_peak_offsets,
                      void *stream);

/* Candidate confirmation, plateau de-duplication.  The local-maximum rule
 * is non-strict, so a flat-topped ridge of votes gives several adjacent
 * peaks (Section 4 leaves the confirmation of candidates to later, more
 * expensive steps).  Two peaks of one event are adjacent when their cells
 * are neighbours in the local-maximum neighbourhood (3x3, 3x3x3 with a d0
 * axis; phi0 periodic, q/pT and d0 not); a cluster is a connected component
 * of that relation.  Clusters of event e are numbered in the order of their
 * first peak and written to clusters[coff[e] ...] (device, `capacity`
 * records, 8-byte aligned), coff = event_cluster_offsets (device, n_events +
 * 1 uint64, written by the call); overflow is handled as in hough_peaks.
 * peak_cluster (device, peak_capacity uint32, 4-byte aligned) receives for
 * every stored peak its cluster's index within the event.  peaks (8-byte
 * aligned) and event_peak_offsets are hough_peaks' outputs for n_events
 * events; peaks it dropped for lack of capacity are not seen.  Requires
 * peak_capacity <= max_peaks (HOUGH_ELIMIT). */
int hough_peak_clusters(hough_ctx *ctx, const hough_peak *peaks, uint64_t peak_capacity,
                        const uint64_t *event_peak_offsets, uint32_t n_events, uint32_t *peak_cluster,
                        hough_cluster *clusters, uint64_t capacity, uint64_t *event_cluster_offsets,
                        void *stream);

/* Candidate confirmation, helix fit (grids without a d0 axis; HOUGH_EINVAL
 * when n_d0 > 1).  On such a grid a hit (r, phi) lies on the track (q/pT,
 * phi0) when y cos phi0 - x sin phi0 + rho r^2 / 2 = 0, x = r cos phi,
 * y = r sin phi, rho = 0.299792458e-3 B q/pT (the track model of the vote's
 * offset tables with d0 = 0).  For every cluster c < min(coff[n_events],
 * capacity): members are the hits of its event that voted into its first
 * peak's cell (k, p); in the frame rotated by the centre azimuth of phi0 bin
 * p the model reads y' = t x' - alpha r^2 with t = tan(phi0 - phi_ref),
 * alpha = rho / (2 cos(phi0 - phi_ref)), and (t, alpha) is the least-squares
 * solution over the members (normal equations, Cramer's rule; status 1 when
 * there are >= 3 members and det > 1e-12 Sxx Sww).  rms_mm is the rms of
 * (y' - t x' + alpha r^2) cos(phi0 - phi_ref) over the members.  On a grid
 * with an rz stage, when hits->z_um is set and the circle is fitted, the
 * members' (s, z) with s = (2 / rho) asin(rho r / 2) (s = r for rho = 0),
 * the transverse arc length along the fitted circle, give the least-squares
 * line z = z0 + cot s (status_z 1 when det = M Sss - Ss^2 > 1e-12 M Sss;
 * rms_z_mm the rms of its residuals): with the circle, the helix.  qpt_c and
 * phi0_c evaluate the bin-centre formulas at the centroid.  Records go to
 * out[c] (device, `capacity` records, 8-byte aligned).  hits are the hits
 * the peaks were found from (same n_events); peaks/event_peak_offsets are
 * hough_peaks' outputs, clusters/event_cluster_offsets hough_peak_clusters'.
 * fp64 arithmetic; members are summed in a fixed order on the device, so
 * results agree with a serial evaluation to rounding.  The member search
 * uses the context's (layer, azimuth bucket) index of the hits, which exists
 * only on a grid with an rz stage or when limits.max_peaks > 0 was given at
 * hough_create: otherwise HOUGH_EINVAL, before anything is enqueued. */
int hough_cluster_fit(hough_ctx *ctx, const hough_hits *hits, const hough_peak *peaks, uint64_t peak_capacity,
                      const uint64_t *event_peak_offsets, const hough_cluster *clusters, uint64_t capacity,
                      const uint64_t *event_cluster_offsets, hough_fit *out, void *stream);

/* Confirmation: rz refinement of the candidates of each event (needs
 * n_z0 > 0).  Candidates of event e are its peaks in list order, or, when
 * rz_max_candidates = M > 0, the first M of them ordered by (popcount
 * descending, cell ascending).  For a candidate with cell (k, p), members
 * are the hits of e that voted into that exact cell; every member votes once
 * per cot bin j at b = floor((z - Z[k][l][j] - z0_lo) * n_z0 / (z0_hi -
 * z0_lo)) when 0 <= b < n_z0.  The record holds the (j, b) of the largest
 * count (ties -> smallest j, then smallest b; all-zero -> (0, 0), count 0).
 * Records of event e are [roff[e], roff[e+1]) of `out` (device, `capacity`
 * records) in candidate order, roff = event_rz_offsets (device, n_events + 1
 * uint64, written by the call); overflow is handled as in hough_peaks.
 * `hits` must be the hits the peaks were found from, with z_um set;
 * peaks (device, peak_capacity records) and event_peak_offsets (device) are
 * hough_peaks' outputs; peaks it dropped for lack of capacity are not seen.
 * When rz_max_candidates > 0 the context holds max_events *
 * rz_max_candidates candidate indices of scratch. */
int hough_rz_refine(hough_ctx *ctx, const hough_hits *hits, const hough_peak *peaks,
                    uint64_t peak_capacity, const uint64_t *event_peak_offsets, hough_rz *out,
                    uint64_t capacity, uint64_t *event_rz_offsets, void *stream);

/* ---- HIP graph of the whole path (batched mode) ------------------------ */

/* Captures vote -> peaks [-> rz when rz_out != NULL] for these exact buffers
 * into a HIP graph, so that one hough_graph_launch replays the whole batch
 * with one host call.  The buffers must stay valid while the graph lives;
 * their contents may change between launches, their sizes may not.  The
 * capture uses `stream` and leaves it idle. */
int hough_graph_capture(hough_ctx *ctx, const hough_hits *hits, uint16_t *acc,
                        hough_peak *peaks, uint64_t peak_capacity, uint64_t *event_peak_offsets,
                        hough_rz *rz_out, uint64_t rz_capacity, uint64_t *event_rz_offsets,
                        void *stream, hough_graph **out);
int hough_graph_launch(hough_graph *graph, void *stream);
void hough_graph_destroy(hough_graph *graph);

/* ---- serving support ---------------------------------------------------- */

/* Micro-batch assembly for the serving loop (keeping events resident on the
 * device across frames, Section 6.2): copies n events out of a
 * device-resident source SoA into one contiguous destination SoA.  Event i
 * occupies source hits [src_off[i], src_off[i] + len[i]) and lands at
 * destination hits [dst_off[i], dst_off[i] + len[i]); dst_off has n + 1
 * entries and dst_off[n] is the destination's hit count, so dst_off is
 * directly usable as the destination's event_offsets.  src_off, len and
 * dst_off are device arrays; the caller guarantees every source range lies
 * inside its buffer.  The destination arrays hold dst_capacity hits: no hit
 * is written at or past dst_capacity (such hits are dropped, so the caller
 * checks dst_off[n] <= dst_capacity before relying on the result).  z
 * pointers may both be NULL.  Asynchronous on `stream`. */
int hough_gather_events(const uint8_t *src_layer, const uint32_t *src_phi, const int32_t *src_z,
                        const uint64_t *src_off, const uint64_t *len, const uint64_t *dst_off,
                        uint32_t n, uint8_t *dst_layer, uint32_t *dst_phi, int32_t *dst_z,
                        uint64_t dst_capacity, void *stream);

/* ---- helpers (not on the hot path) ------------------------------------ */

/* HOUGH_OK if the spec is valid, else HOUGH_EINVAL.  Host only. */
int hough_check_spec(const hough_grid_spec *spec);

/* The library's own host tables, rebuilt from a spec (FP64, the same code
 * hough_create runs; Section 6.1's trigonometry kept off the device), for
 * inspection without a device: O and V as [l][d][k]
 * (n_layers * n_d0 * n_qpt entries each, V = 1 if reachable), Z as [k][l][j]
 * (n_qpt * n_layers * n_cot entries; may be NULL when n_z0 == 0).  Host
 * only, needs no device.  Buffer sizes are checked against nOV and nZ. */
int hough_build_tables(const hough_grid_spec *spec, uint32_t *O, uint8_t *V, size_t nOV,
                       int32_t *Z, size_t nZ);

/* The tables a context uploaded at hough_create, read back from its device
 * (blocking copies; the stream order of other work is not involved).  O and
 * V as [l][d][k] (n_layers * n_d0 * n_qpt entries each, V = 1 if the row is
 * reachable from layer l), Z as [k][l][j] (n_qpt * n_layers * n_cot
 * entries, grids with an rz stage), and Zl = Z + z0_lo, the copy the rz
 * kernel reads when every such sum fits int32 arithmetic exactly (same
 * layout).  Any output pointer may be NULL to skip it; sizes are checked
 * against nOV, nZ and nZl, and asking for Z without an rz stage or for Zl
 * when the context keeps none gives HOUGH_EINVAL. */
int hough_get_tables(const hough_ctx *ctx, uint32_t *O, uint8_t *V, size_t nOV, int32_t *Z, size_t nZ,
                     int32_t *Zl, size_t nZl);

/* Kernel tuning.  Values outside the supported set give HOUGH_EINVAL and
 * leave the previous tuning in place. */
int hough_set_tuning(hough_ctx *ctx, const hough_tuning *tuning);
int hough_get_tuning(const hough_ctx *ctx, hough_tuning *tuning);

/* Per-kernel timing: when enabled, every kernel launch is bracketed by HIP
 * events on its stream.  hough_kernel_times() synchronises those events and
 * fills up to `n` entries (name, launches, total milliseconds), returning
 * the number of distinct kernels; hough_kernel_times_reset() clears them. */
int hough_set_profiling(hough_ctx *ctx, int enable);
int hough_kernel_times(hough_ctx *ctx, const char **names, uint64_t *launches,
                       double *total_ms, int n);
void hough_kernel_times_reset(hough_ctx *ctx);

const char *hough_strerror(int status);
const char *hough_last_error(const hough_ctx *ctx);
/* Number of compute units of the context's device. */
int hough_device_cus(const hough_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HOUGH_H */
