/*
 * CPU ORACLE for the Hough-transform track finder -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct C.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library; the product
 * path never does.  It shares no code, header, table or helper with the GPU
 * library: it builds its own tables from the definitions below.
 *
 * What is computed (Section 4 of the paper, "Hough Transform Algorithm"):
 *   step 1 -- every hit adds a vote to each parameter-space cell whose track
 *             would contain it (the two-variable curvature/azimuth grid);
 *   step 2 -- cells with many votes are candidates; finding them is a
 *             local-maximum search over the grid.
 * The Discussion section describes step 1 as the indirect update A[B[i]] += 1;
 * orc_vote_count() is that counting form.  orc_vote_mask() is the form the
 * tracker uses: a cell holds the OR of the layer bits of its voters, and the
 * "number of votes" of a cell is the popcount of that mask.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - track model: circle of signed curvature rho = 0.299792458e-3 * B * q/pT
 *     [1/mm], perigee (d0, phi0), B along +z, q/pT > 0 bends clockwise; a hit
 *     at radius r lies at phi = phi0 + asin(arg) with
 *     arg = (d0 - rho (r^2 + d0^2) / 2) / (r (1 - rho d0));
 *   - bins: q/pT, d0 and cot(theta) at bin centres; phi0 bin p covers the turn
 *     fractions [p/Nphi, (p+1)/Nphi); angles are uint32 turn fractions;
 *   - rounding: llround (half away from zero) for tables, floor for z0 bins;
 *   - local maximum: popcount >= threshold and >= every neighbour in the
 *     3x3 (q/pT, phi0) window (3x3x3 with d0); phi0 wraps, the others do not;
 *   - rz refinement: members of a candidate are the hits that voted into its
 *     exact cell; each member votes once per cot(theta) bin for
 *     z0 = z - cot * s(r), s the transverse arc length; result is the argmax
 *     with ties to the smallest cot bin, then the smallest z0 bin.
 *
 * Every function is pinned by the CPU test-suite (brute force, closed forms,
 * invariants, bin-centre tracks); none is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    uint32_t n_layers;
    double   layer_r_mm[16];
    double   b_tesla;
    uint32_t n_qpt;
    double   qpt_lo, qpt_hi;
    uint32_t n_phi;
    uint32_t n_d0;
    double   d0_lo_mm, d0_hi_mm;
    uint32_t threshold;
    uint32_t n_z0;
    int32_t  z0_lo_um, z0_hi_um;
    uint32_t n_cot;
    double   cot_lo, cot_hi;
    uint32_t rz_max_candidates;
} orc_spec;

/* ---- spec ------------------------------------------------------------- */

static int is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

static uint32_t log2u(uint32_t v) { uint32_t s = 0; while ((1u << s) < v) s++; return s; }

int orc_check_spec(const orc_spec *g)
{
    if (g->n_layers < 1 || g->n_layers > 16) return -1;
    for (uint32_t l = 0; l < g->n_layers; l++) {
        if (!(g->layer_r_mm[l] > 0.0)) return -1;
        if (l && !(g->layer_r_mm[l] > g->layer_r_mm[l - 1])) return -1;
    }
    if (!is_pow2(g->n_phi) || g->n_phi < 2 || g->n_phi > 65536) return -1;
    if (g->n_qpt < 1 || g->n_d0 < 1) return -1;
    if ((uint64_t)g->n_d0 * g->n_qpt * g->n_phi > 0xFFFFFFFFull) return -1;
    if (g->n_z0) {
        if (g->n_d0 != 1 || g->n_cot < 1 || g->n_cot > 65535 || g->n_z0 > 65535) return -1;
        if (!((int64_t)g->z0_hi_um > (int64_t)g->z0_lo_um)) return -1;
    }
    return 0;
}

/* Bin centres (O1). */
static double kappa_of(const orc_spec *g, uint32_t k)
{
    return g->qpt_lo + (k + 0.5) * ((g->qpt_hi - g->qpt_lo) / g->n_qpt);
}
static double d0_of(const orc_spec *g, uint32_t d)
{
    if (g->n_d0 == 1) return 0.0;
    return g->d0_lo_mm + (d + 0.5) * ((g->d0_hi_mm - g->d0_lo_mm) / g->n_d0);
}
static double cot_of(const orc_spec *g, uint32_t j)
{
    return g->cot_lo + (j + 0.5) * ((g->cot_hi - g->cot_lo) / g->n_cot);
}

/* ---- tables (O2, O5) --------------------------------------------------- */

/* O[l][d][k]: uint32 turn fraction of (phi_hit - phi0) for the bin-centre
 * track (kappa_k, d0_d) at radius r_l; V = 0 where the layer is unreachable. */
void orc_offsets(const orc_spec *g, uint32_t *O, uint8_t *V)
{
    for (uint32_t l = 0; l < g->n_layers; l++)
        for (uint32_t d = 0; d < g->n_d0; d++)
            for (uint32_t k = 0; k < g->n_qpt; k++) {
                double r = g->layer_r_mm[l];
                double d0 = d0_of(g, d);
                double rho = (0.299792458e-3 * g->b_tesla) * kappa_of(g, k);
                double den = r * (1.0 - rho * d0);
                double arg = (d0 - rho * (r * r + d0 * d0) * 0.5) / den;
                int ok = (1.0 - rho * d0) > 0.0 && fabs(arg) <= 1.0;
                size_t i = ((size_t)l * g->n_d0 + d) * g->n_qpt + k;
                V[i] = (uint8_t)ok;
                O[i] = ok ? (uint32_t)(int64_t)llround(asin(arg) / (2.0 * M_PI) * 4294967296.0) : 0u;
            }
}

/* Z[k][l][j]: cot_j times the transverse arc length to radius r_l of the
 * prompt bin-centre track kappa_k, in integer micrometres. */
void orc_zshift(const orc_spec *g, int32_t *Z)
{
    for (uint32_t k = 0; k < g->n_qpt; k++)
        for (uint32_t l = 0; l < g->n_layers; l++)
            for (uint32_t j = 0; j < g->n_cot; j++) {
                double r = g->layer_r_mm[l];
                double rho = (0.299792458e-3 * g->b_tesla) * kappa_of(g, k);
                double s = (rho == 0.0) ? r : (2.0 / rho) * asin(rho * r * 0.5);
                Z[((size_t)k * g->n_layers + l) * g->n_cot + j] =
                    (int32_t)llround(cot_of(g, j) * s * 1000.0);
            }
}

/* ---- step 1: voting (O3, O3') ----------------------------------------- */

/* A[d][k][p] |= 1 << layer for every hit and every reachable row. */
void orc_vote_mask(const orc_spec *g, const uint32_t *O, const uint8_t *V,
                   uint64_t n_hits, const uint8_t *layer, const uint32_t *phi,
                   uint16_t *A)
{
    uint32_t s = 32 - log2u(g->n_phi);
    size_t cells = (size_t)g->n_d0 * g->n_qpt * g->n_phi;
    memset(A, 0, cells * sizeof(uint16_t));
    for (uint64_t h = 0; h < n_hits; h++) {
        uint32_t l = layer[h];
        if (l >= g->n_layers) continue;
        for (uint32_t d = 0; d < g->n_d0; d++)
            for (uint32_t k = 0; k < g->n_qpt; k++) {
                size_t t = ((size_t)l * g->n_d0 + d) * g->n_qpt + k;
                if (!V[t]) continue;
                uint32_t p = (uint32_t)(phi[h] - O[t]) >> s;
                A[((size_t)d * g->n_qpt + k) * g->n_phi + p] |= (uint16_t)(1u << l);
            }
    }
}

/* The paper's counting form: C[d][k][p] += 1. */
void orc_vote_count(const orc_spec *g, const uint32_t *O, const uint8_t *V,
                    uint64_t n_hits, const uint8_t *layer, const uint32_t *phi,
                    uint32_t *C)
{
    uint32_t s = 32 - log2u(g->n_phi);
    size_t cells = (size_t)g->n_d0 * g->n_qpt * g->n_phi;
    memset(C, 0, cells * sizeof(uint32_t));
    for (uint64_t h = 0; h < n_hits; h++) {
        uint32_t l = layer[h];
        if (l >= g->n_layers) continue;
        for (uint32_t d = 0; d < g->n_d0; d++)
            for (uint32_t k = 0; k < g->n_qpt; k++) {
                size_t t = ((size_t)l * g->n_d0 + d) * g->n_qpt + k;
                if (!V[t]) continue;
                uint32_t p = (uint32_t)(phi[h] - O[t]) >> s;
                C[((size_t)d * g->n_qpt + k) * g->n_phi + p] += 1;
            }
    }
}

/* ---- step 2: local maxima (O4) ---------------------------------------- */

static int popc16(uint16_t v) { return __builtin_popcount((unsigned)v); }

/* Peaks in ascending cell order; writes at most cap records, returns the
 * true number of peaks. */
uint64_t orc_peaks(const orc_spec *g, const uint16_t *A,
                   uint32_t *cell, uint16_t *mask, uint16_t *pc, uint64_t cap)
{
    uint64_t n = 0;
    int nd = (int)g->n_d0, nk = (int)g->n_qpt, np = (int)g->n_phi;
    for (int d = 0; d < nd; d++)
        for (int k = 0; k < nk; k++)
            for (int p = 0; p < np; p++) {
                size_t c = ((size_t)d * nk + k) * np + p;
                int v = popc16(A[c]);
                if (v < (int)g->threshold) continue;
                int is_max = 1;
                for (int dd = -1; dd <= 1 && is_max; dd++) {
                    if (nd == 1 && dd != 0) continue;          /* 2D grid: no d0 axis */
                    int d2 = d + dd;
                    if (d2 < 0 || d2 >= nd) continue;
                    for (int dk = -1; dk <= 1 && is_max; dk++) {
                        int k2 = k + dk;
                        if (k2 < 0 || k2 >= nk) continue;
                        for (int dp = -1; dp <= 1; dp++) {
                            if (dd == 0 && dk == 0 && dp == 0) continue;
                            int p2 = ((p + dp) % np + np) % np;
                            if (popc16(A[((size_t)d2 * nk + k2) * np + p2]) > v) { is_max = 0; break; }
                        }
                    }
                }
                if (!is_max) continue;
                if (n < cap) {
                    cell[n] = (uint32_t)c;
                    mask[n] = A[c];
                    pc[n] = (uint16_t)v;
                }
                n++;
            }
    return n;
}

/* Local maxima of the counting accumulator (the paper's A[B[i]] += 1 form,
 * Section 8): the same rule as orc_peaks with the cell's vote count in place
 * of its popcount -- count >= threshold and >= the count of every
 * neighbour (3x3, 3x3x3 with a d0 axis; phi0 periodic).  Ascending cell
 * order; returns the true number of peaks, records past cap dropped. */
uint64_t orc_peaks_count(const orc_spec *g, const uint32_t *C, uint32_t *cell, uint32_t *count,
                         uint64_t cap)
{
    uint64_t n = 0;
    int nd = (int)g->n_d0, nk = (int)g->n_qpt, np = (int)g->n_phi;
    for (int d = 0; d < nd; d++)
        for (int k = 0; k < nk; k++)
            for (int p = 0; p < np; p++) {
                size_t c = ((size_t)d * nk + k) * np + p;
                uint32_t v = C[c];
                if (v < g->threshold) continue;
                int is_max = 1;
                for (int dd = -1; dd <= 1 && is_max; dd++) {
                    if (nd == 1 && dd != 0) continue;
                    int d2 = d + dd;
                    if (d2 < 0 || d2 >= nd) continue;
                    for (int dk = -1; dk <= 1 && is_max; dk++) {
                        int k2 = k + dk;
                        if (k2 < 0 || k2 >= nk) continue;
                        for (int dp = -1; dp <= 1; dp++) {
                            if (dd == 0 && dk == 0 && dp == 0) continue;
                            int p2 = ((p + dp) % np + np) % np;
                            if (C[((size_t)d2 * nk + k2) * np + p2] > v) { is_max = 0; break; }
                        }
                    }
                }
                if (!is_max) continue;
                if (n < cap) {
                    cell[n] = (uint32_t)c;
                    count[n] = v;
                }
                n++;
            }
    return n;
}

/* ---- rz refinement (O5) ----------------------------------------------- */

static int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) q--;
    return q;
}

/* Candidate order: all peaks in list order, or the first rz_max_candidates
 * peaks ordered by (popcount descending, cell ascending). */
uint64_t orc_rz_candidates(const orc_spec *g, uint64_t n_peaks, const uint16_t *pc,
                           uint32_t *cand)
{
    uint64_t cap = g->rz_max_candidates;
    if (cap == 0) {
        for (uint64_t i = 0; i < n_peaks; i++) cand[i] = (uint32_t)i;
        return n_peaks;
    }
    uint64_t n = 0;
    for (int v = 16; v >= 0 && n < cap; v--)
        for (uint64_t i = 0; i < n_peaks && n < cap; i++)
            if (pc[i] == v) cand[n++] = (uint32_t)i;
    return n;
}

/* For each candidate: member hits, then the (cot, z0) vote and its argmax.
 * Returns the number of records (= number of candidates). */
uint64_t orc_rz(const orc_spec *g, const uint32_t *O, const uint8_t *V, const int32_t *Z,
                uint64_t n_hits, const uint8_t *layer, const uint32_t *phi, const int32_t *z,
                uint64_t n_peaks, const uint32_t *cell, const uint16_t *pc,
                uint32_t *out_peak, uint16_t *out_cot, uint16_t *out_z0,
                uint32_t *out_count, uint32_t *out_nmem)
{
    uint32_t s = 32 - log2u(g->n_phi);
    uint32_t *cand = (uint32_t *)malloc((n_peaks + 1) * sizeof(uint32_t));
    uint64_t n_cand = orc_rz_candidates(g, n_peaks, pc, cand);
    uint64_t *mem = (uint64_t *)malloc((n_hits + 1) * sizeof(uint64_t));
    int32_t *hist = (int32_t *)calloc(g->n_z0, sizeof(int32_t));
    int64_t *bins = (int64_t *)malloc((n_hits + 1) * sizeof(int64_t));
    int64_t span = (int64_t)g->z0_hi_um - (int64_t)g->z0_lo_um;

    for (uint64_t c = 0; c < n_cand; c++) {
        uint32_t pk = cand[c];
        uint32_t k = (cell[pk] / g->n_phi) % g->n_qpt;     /* n_d0 == 1 here */
        uint32_t p = cell[pk] % g->n_phi;
        /* members: hits that voted into this exact cell */
        uint64_t nm = 0;
        for (uint64_t h = 0; h < n_hits; h++) {
            uint32_t l = layer[h];
            if (l >= g->n_layers) continue;
            size_t t = (size_t)l * g->n_qpt + k;
            if (!V[t]) continue;
            if (((uint32_t)(phi[h] - O[t]) >> s) == p) mem[nm++] = h;
        }
        /* dense argmax over (j, b) of R[j][b], evaluated one cot row at a time */
        int64_t best = 0; uint32_t best_j = 0, best_b = 0;
        for (uint32_t j = 0; j < g->n_cot; j++) {
            for (uint64_t m = 0; m < nm; m++) {
                uint64_t h = mem[m];
                int64_t z0 = (int64_t)z[h] - (int64_t)Z[((size_t)k * g->n_layers + layer[h]) * g->n_cot + j];
                int64_t b = floor_div64((z0 - (int64_t)g->z0_lo_um) * (int64_t)g->n_z0, span);
                bins[m] = b;
                if (b >= 0 && b < (int64_t)g->n_z0) hist[b]++;
            }
            /* the row's maximum, smallest bin among ties */
            int64_t row_best = 0; int64_t row_b = 0;
            for (uint64_t m = 0; m < nm; m++) {
                int64_t b = bins[m];
                if (b < 0 || b >= (int64_t)g->n_z0) continue;
                if (hist[b] > row_best || (hist[b] == row_best && b < row_b)) {
                    row_best = hist[b]; row_b = b;
                }
            }
            for (uint64_t m = 0; m < nm; m++) {
                int64_t b = bins[m];
                if (b >= 0 && b < (int64_t)g->n_z0) hist[b] = 0;
            }
            if (row_best > best) { best = row_best; best_j = j; best_b = (uint32_t)row_b; }
        }
        out_peak[c] = pk;
        out_cot[c] = (uint16_t)best_j;
        out_z0[c] = (uint16_t)best_b;
        out_count[c] = (uint32_t)best;
        out_nmem[c] = (uint32_t)nm;
    }
    free(cand); free(mem); free(hist); free(bins);
    return n_cand;
}

/* ---- candidate confirmation: plateau clusters --------------------------
 *
 * The non-strict local-maximum rule reports every cell of a flat-topped
 * ridge, so one track can give several adjacent peaks (Section 4 leaves the
 * confirmation of candidates to more expensive later computations).  Two
 * peaks of one event are adjacent when their cells are neighbours in the
 * local-maximum neighbourhood (3x3 in (q/pT, phi0), 3x3x3 with a d0 axis;
 * phi0 periodic, q/pT and d0 not).  A cluster is a connected component of
 * that adjacency relation over the event's peak list.
 *
 * Clusters are numbered in the order of their first peak (the member with
 * the smallest list index, hence the smallest cell); label[i] is peak i's
 * cluster number.  Per cluster: first, n_peaks, and the sums over its
 * members of d - d_first, k - k_first and the signed phi0 offset
 * ((p - p_first) mod n_phi, taken in [-n_phi/2, n_phi/2)); popcount of the
 * first peak and the OR of the members' masks.  The centroid is
 * (d_first + sum_dd / n, k_first + sum_dk / n, p_first + sum_dp / n mod n_phi).
 * Found by breadth-first search from each unlabelled peak in list order over
 * a dense cell -> peak map.  Returns the number of clusters; every output
 * array is sized by the caller for n entries. */
uint64_t orc_clusters(const orc_spec *g, uint64_t n, const uint32_t *cell, const uint16_t *mask,
                      const uint16_t *pc, uint32_t *label, uint32_t *first, uint32_t *n_peaks,
                      int32_t *sum_dd, int32_t *sum_dk, int32_t *sum_dp, uint16_t *cl_pc,
                      uint16_t *cl_mask)
{
    int nd = (int)g->n_d0, nk = (int)g->n_qpt, np = (int)g->n_phi;
    size_t cells = (size_t)nd * nk * np;
    int64_t *at = (int64_t *)malloc(cells * sizeof(int64_t));
    uint32_t *queue = (uint32_t *)malloc((n + 1) * sizeof(uint32_t));
    for (size_t c = 0; c < cells; c++) at[c] = -1;
    for (uint64_t i = 0; i < n; i++) {
        at[cell[i]] = (int64_t)i;
        label[i] = 0xFFFFFFFFu;
    }
    uint64_t n_cl = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (label[i] != 0xFFFFFFFFu) continue;
        uint32_t id = (uint32_t)n_cl++;
        first[id] = (uint32_t)i;
        label[i] = id;
        uint64_t head = 0, tail = 0;
        queue[tail++] = (uint32_t)i;
        while (head < tail) {
            uint32_t x = queue[head++];
            int p = (int)(cell[x] % (uint32_t)np);
            int k = (int)((cell[x] / (uint32_t)np) % (uint32_t)nk);
            int d = (int)(cell[x] / ((uint32_t)np * (uint32_t)nk));
            for (int dd = -1; dd <= 1; dd++) {
                int d2 = d + dd;
                if (d2 < 0 || d2 >= nd) continue;
                for (int dk = -1; dk <= 1; dk++) {
                    int k2 = k + dk;
                    if (k2 < 0 || k2 >= nk) continue;
                    for (int dp = -1; dp <= 1; dp++) {
                        int p2 = ((p + dp) % np + np) % np;
                        int64_t y = at[((size_t)d2 * nk + k2) * np + p2];
                        if (y < 0 || label[y] != 0xFFFFFFFFu) continue;
                        label[y] = id;
                        queue[tail++] = (uint32_t)y;
                    }
                }
            }
        }
    }
    for (uint64_t c = 0; c < n_cl; c++) {
        n_peaks[c] = 0;
        sum_dd[c] = sum_dk[c] = sum_dp[c] = 0;
        cl_pc[c] = pc[first[c]];
        cl_mask[c] = 0;
    }
    for (uint64_t i = 0; i < n; i++) {
        uint32_t c = label[i], f = cell[first[c]];
        int p = (int)(cell[i] % (uint32_t)np), pf = (int)(f % (uint32_t)np);
        int k = (int)((cell[i] / (uint32_t)np) % (uint32_t)nk), kf = (int)((f / (uint32_t)np) % (uint32_t)nk);
        int d = (int)(cell[i] / ((uint32_t)np * (uint32_t)nk)), df = (int)(f / ((uint32_t)np * (uint32_t)nk));
        int dp = ((p - pf) % np + np) % np;
        if (dp >= np / 2) dp -= np;
        n_peaks[c]++;
        sum_dd[c] += d - df;
        sum_dk[c] += k - kf;
        sum_dp[c] += dp;
        cl_mask[c] |= mask[i];
    }
    free(at); free(queue);
    return n_cl;
}

/* ---- candidate confirmation: track fit of a cluster --------------------
 *
 * For a beam-line grid (n_d0 == 1, d0 = 0) a hit at radius r and azimuth
 * phi lies on the track (q/pT, phi0) when r sin(phi - phi0) + rho r^2 / 2 = 0
 * (the track model above with d0 = 0), i.e. with x = r cos phi, y = r sin phi:
 *     y cos phi0 - x sin phi0 + rho r^2 / 2 = 0.
 * In a frame rotated by a reference azimuth phi_ref close to the track
 * (x', y' the rotated coordinates, phi0' = phi0 - phi_ref, |phi0'| < pi/2)
 * dividing by cos phi0' makes this linear in t = tan phi0' and
 * alpha = rho / (2 cos phi0'):   y' = t x' - alpha r^2.
 * The fit is the least-squares solution over the members, from the normal
 * equations  [Sxx  -Sxw; -Sxw  Sww] [t; alpha] = [Sxy; -Syw]  (w = r^2),
 * by Cramer's rule; then phi0 = phi_ref + atan t, rho = 2 alpha cos phi0',
 * q/pT = rho / (0.299792458e-3 B).  The residual of a member is
 * (y' - t x' + alpha w) cos phi0' (mm, its distance from the curve to first
 * order); rms over the members.
 *
 * Members: the hits that voted into the cluster's first peak cell (k_f, p_f)
 * -- layer l < n_layers, row valid, ((phi - O[l][k_f]) >> shift) == p_f.
 * phi_ref: the centre of that cell's phi0 bin.  status = 1 when there are at
 * least 3 members and det = Sxx Sww - Sxw^2 > 1e-12 Sxx Sww, else 0 with
 * zero fit outputs.  The centroid parameters are the bin-centre formulas
 * evaluated at the centroid: q/pT_c = qpt_lo + (k_c + 1/2) (qpt_hi - qpt_lo)
 * / n_qpt, phi0_c = 2 pi ((p_c + 1/2) / n_phi mod 1). */
/* Longitudinal part (when z is given, z != NULL, and the transverse fit
 * succeeded): a member at radius r lies at z = z0 + cot(theta) s, s the
 * transverse arc length from the perigee along the fitted circle,
 * s = (2 / rho) asin(rho r / 2) (s = r for rho = 0).  (z0, cot) is the
 * least-squares line through the members' (s, z) points (z in mm), from
 * [M  Ss; Ss  Sss] [z0; cot] = [Sz; Ssz]; status_z = 1 when det =
 * M Sss - Ss^2 > 1e-12 M Sss, and rms_z_mm is the rms of z - z0 - cot s. */
static double arc_length(double rho, double r)
{
    double x = 0.5 * rho * r;
    return x == 0.0 ? r : r * (asin(x) / x);
}

void orc_fit(const orc_spec *g, const uint32_t *O, const uint8_t *V,
             uint64_t n_hits, const uint8_t *layer, const uint32_t *phi, const int32_t *z,
             uint64_t n_clusters, const uint32_t *first_cell, const uint32_t *n_peaks,
             const int32_t *sum_dk, const int32_t *sum_dp,
             double *qpt, double *phi0, double *qpt_c, double *phi0_c, double *rms,
             double *cot, double *z0_mm, double *rms_z,
             uint32_t *n_fit, uint32_t *status, uint32_t *status_z)
{
    const double two_pi = 2.0 * M_PI;
    const double turn_rad = two_pi / 4294967296.0;
    uint32_t s = 32 - log2u(g->n_phi);
    for (uint64_t c = 0; c < n_clusters; c++) {
        uint32_t k = (first_cell[c] / g->n_phi) % g->n_qpt;
        uint32_t p = first_cell[c] % g->n_phi;
        double n = (double)n_peaks[c];
        double kc = (double)k + (double)sum_dk[c] / n;
        double pc = (double)p + (double)sum_dp[c] / n;
        qpt_c[c] = g->qpt_lo + (kc + 0.5) * ((g->qpt_hi - g->qpt_lo) / g->n_qpt);
        double f = fmod((pc + 0.5) / (double)g->n_phi, 1.0);
        if (f < 0) f += 1.0;
        phi0_c[c] = two_pi * f;

        uint32_t ref = (p << s) + (1u << (s - 1));
        double sxx = 0, sxw = 0, sww = 0, sxy = 0, syw = 0;
        uint32_t m = 0;
        for (int pass = 0; pass < 2; pass++) {
            double t = 0, alpha = 0, cosp = 0, ss = 0;
            if (pass == 1) {
                double det = sxx * sww - sxw * sxw;
                if (m < 3 || !(det > 1e-12 * sxx * sww)) break;
                t = (sxy * sww - sxw * syw) / det;
                alpha = (sxw * sxy - sxx * syw) / det;
                cosp = 1.0 / sqrt(1.0 + t * t);
            }
            for (uint64_t h = 0; h < n_hits; h++) {
                uint32_t l = layer[h];
                if (l >= g->n_layers) continue;
                size_t ti = (size_t)l * g->n_qpt + k;
                if (!V[ti] || ((uint32_t)(phi[h] - O[ti]) >> s) != p) continue;
                double ang = (double)(int32_t)(phi[h] - ref) * turn_rad;
                double r = g->layer_r_mm[l];
                double x = r * cos(ang), y = r * sin(ang), w = r * r;
                if (pass == 0) {
                    sxx += x * x; sxw += x * w; sww += w * w; sxy += x * y; syw += y * w;
                    m++;
                } else {
                    double res = (y - t * x + alpha * w) * cosp;
                    ss += res * res;
                }
            }
            if (pass == 1) {
                double ph = (double)ref * turn_rad + atan(t);
                ph = fmod(ph, two_pi);
                if (ph < 0) ph += two_pi;
                phi0[c] = ph;
                qpt[c] = 2.0 * alpha * cosp / (0.299792458e-3 * g->b_tesla);
                rms[c] = sqrt(ss / m);
                status[c] = 1;
            }
        }
        n_fit[c] = m;
        cot[c] = z0_mm[c] = rms_z[c] = 0.0;
        status_z[c] = 0;
        if (m < 3 || !(sxx * sww - sxw * sxw > 1e-12 * sxx * sww)) {
            qpt[c] = phi0[c] = rms[c] = 0.0;
            status[c] = 0;
            continue;
        }
        if (!z) continue;
        /* longitudinal line over the same members */
        double rho = qpt[c] * 0.299792458e-3 * g->b_tesla;
        double s1 = 0, s2 = 0, sz = 0, ssz = 0;
        double zz0 = 0, zcot = 0, zss = 0;
        for (int pass = 0; pass < 2; pass++) {
            for (uint64_t h = 0; h < n_hits; h++) {
                uint32_t l = layer[h];
                if (l >= g->n_layers) continue;
                size_t ti = (size_t)l * g->n_qpt + k;
                if (!V[ti] || ((uint32_t)(phi[h] - O[ti]) >> s) != p) continue;
                double sa = arc_length(rho, g->layer_r_mm[l]);
                double zm = (double)z[h] * 1e-3;
                if (pass == 0) {
                    s1 += sa; s2 += sa * sa; sz += zm; ssz += sa * zm;
                } else {
                    double res = zm - zz0 - zcot * sa;
                    zss += res * res;
                }
            }
            if (pass == 0) {
                double det = (double)m * s2 - s1 * s1;
                if (!(det > 1e-12 * (double)m * s2)) break;
                zz0 = (s2 * sz - s1 * ssz) / det;
                zcot = ((double)m * ssz - s1 * sz) / det;
            } else {
                cot[c] = zcot;
                z0_mm[c] = zz0;
                rms_z[c] = sqrt(zss / m);
                status_z[c] = 1;
            }
        }
    }
}
