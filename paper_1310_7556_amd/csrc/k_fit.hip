// Candidate confirmation, second part: a track fit per plateau cluster.
//
// For a beam-line grid (no d0 axis) a hit (r, phi) lies on the track
// (q/pT, phi0) when y cos phi0 - x sin phi0 + rho r^2 / 2 = 0 with
// x = r cos phi, y = r sin phi and rho = 0.299792458e-3 B q/pT (the track
// model of the offset tables with d0 = 0).  Rotated by a reference azimuth
// phi_ref close to the track and divided by cos(phi0 - phi_ref) this is
// linear: y' = t x' - alpha r^2 with t = tan(phi0 - phi_ref) and
// alpha = rho / (2 cos(phi0 - phi_ref)).  Least squares over the members
// gives the 2x2 normal equations, solved by Cramer's rule.
//
// Members are the hits that voted into the cluster's first peak cell; the
// reference azimuth is the centre of that cell's phi0 bin.  One wave per
// cluster: pass 1 sums x'^2, x' r^2, r^4, x' y', y' r^2 over the members,
// found in the few azimuth buckets per layer that cover the cell (hits
// sorted by (layer, bucket) per event), pass 2 the squared residuals of the
// solution.  With z (grids with an rz stage), the residual pass also sums
// the members' (arc length, z) and a third pass takes the residuals of the
// least-squares line z = z0 + cot(theta) s, s the transverse arc length
// (2 / rho) asin(rho r / 2) along the fitted circle: the helix.  fp64
// throughout, wave sums by a fixed butterfly.
#include "hough_internal.h"

namespace hough {
namespace {

struct FitParams {
    const uint32_t *phi_b;        // hits grouped by (layer, azimuth bucket) per event
    const int32_t *z_b;           // their z (um), or null: no longitudinal fit
    const uint32_t *bucket_off;   // [E][L][NB + 1] relative to the event start
    uint32_t bucket_bits;
    const uint64_t *hoff;         // [E + 1] hit offsets
    uint64_t n_hits;
    const uint2 *pk;              // peak records
    uint64_t peak_cap;
    const uint64_t *poff;         // [E + 1]
    const hough_cluster *cl;
    uint64_t cl_cap;
    const uint64_t *coff;         // [E + 1]
    uint32_t E;
    hough_fit *out;
    const uint32_t *O;            // [L][n_qpt]
    const uint8_t *V;
    double r_mm[kMaxLayers];
    uint32_t n_layers, n_qpt, n_phi, log2_phi, shift;
    double qpt_lo, qpt_w;         // bin width (qpt_hi - qpt_lo) / n_qpt
    double inv_curv;              // 1 / (0.299792458e-3 B)
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v)
{
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// The member hits of cell (k, p) lie in a few azimuth buckets per layer.
// Lane l < L finds layer l's bucket window (one range of the layer's
// bucket-sorted hits, two when it wraps past 2 pi); a lane scan of the
// window lengths concatenates them, and visit(layer lane, hit) walks the
// concatenation with the lanes side by side.  Every shuffle runs on all
// lanes; visit sees only hits that pass the membership test.
struct Windows {
    uint32_t o, hs1, len1, hs2, excl, total;
};

__device__ __forceinline__ Windows layer_windows(const FitParams &P, uint32_t e, uint32_t k, uint32_t p,
                                                 uint32_t lane)
{
    const uint32_t nb = 1u << P.bucket_bits, bs = 32 - P.bucket_bits;
    const uint64_t W = uint64_t(1) << P.shift, BW = uint64_t(1) << bs;
    Windows w{};
    uint32_t len2 = 0;
    if (lane < P.n_layers) {
        const size_t ti = size_t(lane) * P.n_qpt + k;
        if (P.V[ti]) {
            w.o = P.O[ti];
            const uint32_t start = w.o + (p << P.shift);
            const uint32_t b0 = start >> bs;
            const uint32_t nbk = min(uint32_t(((uint64_t(start) & (BW - 1)) + W - 1) / BW + 1), nb);
            const uint32_t *bl = P.bucket_off + (size_t(e) * P.n_layers + lane) * (nb + 1);
            const uint32_t e1 = b0 + nbk;
            w.hs1 = bl[b0];
            if (e1 <= nb) {
                w.len1 = bl[e1] - w.hs1;
            } else {
                w.len1 = bl[nb] - w.hs1;
                w.hs2 = bl[0];
                len2 = bl[e1 - nb] - w.hs2;
            }
        }
    }
    const uint32_t len = w.len1 + len2;
    uint32_t incl = len;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        incl += lane >= d ? y : 0u;
    }
    w.excl = incl - len;
    w.total = __shfl(incl, 63, 64);
    return w;
}

template <typename Fn>
__device__ __forceinline__ void for_members(const FitParams &P, const Windows &w, uint64_t eb, uint32_t p,
                                            uint32_t lane, Fn &&visit)
{
    for (uint32_t g0 = 0; g0 < w.total; g0 += 64) {
        const uint32_t gi = g0 + lane;
        uint32_t ls = 0;
        for (uint32_t q = 0; q < P.n_layers; ++q) ls = __shfl(w.excl, q, 64) <= gi ? q : ls;
        const uint32_t local = gi - __shfl(w.excl, ls, 64);
        const uint32_t l1 = __shfl(w.len1, ls, 64);
        const uint32_t h1 = __shfl(w.hs1, ls, 64), h2 = __shfl(w.hs2, ls, 64);
        const uint32_t o = __shfl(w.o, ls, 64);
        if (gi < w.total) {
            const uint32_t h = local < l1 ? h1 + local : h2 + (local - l1);
            const uint32_t ph = P.phi_b[eb + h];
            if (((ph - o) >> P.shift) == p) visit(ls, ph, h);
        }
    }
}

// Z: the longitudinal line is fitted too (P.z_b set); a separate instance
// keeps the transverse-only kernel's register count (and occupancy) down.
template <bool Z>
__global__ void __launch_bounds__(256) k_fit(FitParams P)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave0 = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    const uint64_t n_cl = min(P.coff[P.E], P.cl_cap);
    const double two_pi = 6.283185307179586476925286766559;
    const double turn_rad = two_pi / 4294967296.0;
    const uint32_t pmask = P.n_phi - 1;
    for (uint64_t c = wave0; c < n_cl; c += waves) {
        // event of cluster c: largest e with start(e) <= c
        uint32_t lo = 0, hi = P.E;
        while (hi - lo > 1) {
            const uint32_t m = (lo + hi) >> 1;
            if (min(P.coff[m], n_cl) <= c) lo = m;
            else hi = m;
        }
        const uint32_t e = lo;
        const hough_cluster rec = P.cl[c];
        const uint64_t pe0 = min(P.poff[e], P.peak_cap), pe1 = min(max(P.poff[e + 1], P.poff[e]), P.peak_cap);
        const uint64_t gi = pe0 + rec.first;
        hough_fit f{};
        if (gi < pe1 && rec.n_peaks > 0) {
            const uint32_t cell = P.pk[gi].x;
            const uint32_t p = cell & pmask, k = (cell >> P.log2_phi) % P.n_qpt;
            const double n = double(rec.n_peaks);
            const double kc = double(k) + double(rec.sum_dk) / n;
            const double pc = double(p) + double(rec.sum_dp) / n;
            f.qpt_c = P.qpt_lo + (kc + 0.5) * P.qpt_w;
            double fr = fmod((pc + 0.5) / double(P.n_phi), 1.0);
            if (fr < 0) fr += 1.0;
            f.phi0_c = two_pi * fr;

            const uint64_t eb = min(P.hoff[e], P.n_hits);
            const uint32_t ref = (p << P.shift) + (1u << (P.shift - 1));
            const Windows w = layer_windows(P, e, k, p, lane);
            double sxx = 0, sxw = 0, sww = 0, sxy = 0, syw = 0;
            uint32_t m = 0;
            for_members(P, w, eb, p, lane, [&](uint32_t l, uint32_t ph, uint32_t) {
                double sa, ca;
                sincos(double(int32_t(ph - ref)) * turn_rad, &sa, &ca);
                const double r = P.r_mm[l], wr = r * r;
                const double x = r * ca, y = r * sa;
                sxx += x * x;
                sxw += x * wr;
                sww += wr * wr;
                sxy += x * y;
                syw += y * wr;
                ++m;
            });
            sxx = wave_sum(sxx);
            sxw = wave_sum(sxw);
            sww = wave_sum(sww);
            sxy = wave_sum(sxy);
            syw = wave_sum(syw);
            m = wave_sum_u(m);
            f.n_hits = m;
            const double det = sxx * sww - sxw * sxw;
            if (m >= 3 && det > 1e-12 * sxx * sww) {
                const double t = (sxy * sww - sxw * syw) / det;
                const double alpha = (sxw * sxy - sxx * syw) / det;
                const double cosp = 1.0 / sqrt(1.0 + t * t);
                const double qpt = 2.0 * alpha * cosp * P.inv_curv;
                const double rho = qpt / P.inv_curv;
                // arc length from the perigee along the fitted circle
                auto arc = [&](double r) {
                    const double x = 0.5 * rho * r;
                    return x == 0.0 ? r : r * (asin(x) / x);
                };
                double ss = 0, s1 = 0, s2 = 0, sz = 0, ssz = 0;
                for_members(P, w, eb, p, lane, [&](uint32_t l, uint32_t ph, uint32_t h) {
                    double sa, ca;
                    sincos(double(int32_t(ph - ref)) * turn_rad, &sa, &ca);
                    const double r = P.r_mm[l];
                    const double res = (r * sa - t * (r * ca) + alpha * (r * r)) * cosp;
                    ss += res * res;
                    if (Z) {
                        const double s = arc(r), zm = double(P.z_b[eb + h]) * 1e-3;
                        s1 += s;
                        s2 += s * s;
                        sz += zm;
                        ssz += s * zm;
                    }
                });
                ss = wave_sum(ss);
                if (Z) {
                    s1 = wave_sum(s1);
                    s2 = wave_sum(s2);
                    sz = wave_sum(sz);
                    ssz = wave_sum(ssz);
                    // the line z = z0 + cot s through the members
                    const double dm = double(m), detz = dm * s2 - s1 * s1;
                    if (detz > 1e-12 * dm * s2) {
                        const double z0 = (s2 * sz - s1 * ssz) / detz;
                        const double ct = (dm * ssz - s1 * sz) / detz;
                        double sr = 0;
                        for_members(P, w, eb, p, lane, [&](uint32_t l, uint32_t, uint32_t h) {
                            const double res = double(P.z_b[eb + h]) * 1e-3 - z0 - ct * arc(P.r_mm[l]);
                            sr += res * res;
                        });
                        sr = wave_sum(sr);
                        f.cot = ct;
                        f.z0_mm = z0;
                        f.rms_z_mm = sqrt(sr / m);
                        f.status_z = 1;
                    }
                }
                double ph0 = fmod(double(ref) * turn_rad + atan(t), two_pi);
                if (ph0 < 0) ph0 += two_pi;
                f.phi0 = ph0;
                f.qpt = qpt;
                f.rms_mm = sqrt(ss / m);
                f.status = 1;
            }
        }
        if (lane == 0) P.out[c] = f;
    }
}

}  // namespace

hipError_t launch_fit(hough_ctx *c, const hough_hits *h, const hough_peak *peaks, uint64_t peak_capacity,
                      const uint64_t *poff, const hough_cluster *clusters, uint64_t capacity, const uint64_t *coff,
                      hough_fit *out, hipStream_t s)
{
    if (h->n_events == 0 || capacity == 0) return hipSuccess;
    // the longitudinal line needs z, bucketed with the azimuths (rz grids)
    const bool with_z = c->spec.n_z0 > 0 && h->z_um != nullptr;
    hipError_t err = launch_bucket_layers(c, h, with_z, s);
    if (err == hipSuccess) err = launch_bucket_phi(c, h, s, with_z);
    if (err != hipSuccess) return err;
    FitParams P{};
    P.phi_b = c->d_phi_b;
    P.z_b = with_z ? c->d_z_b : nullptr;
    P.bucket_off = c->d_bucket_off;
    P.bucket_bits = c->bucket_bits;
    P.hoff = h->event_offsets;
    P.n_hits = h->n_hits;
    P.pk = reinterpret_cast<const uint2 *>(peaks);
    P.peak_cap = peak_capacity;
    P.poff = poff;
    P.cl = clusters;
    P.cl_cap = capacity;
    P.coff = coff;
    P.E = h->n_events;
    P.out = out;
    P.O = c->d_O;
    P.V = c->d_V;
    for (uint32_t l = 0; l < c->spec.n_layers && l < kMaxLayers; ++l) P.r_mm[l] = c->spec.layer_r_mm[l];
    P.n_layers = c->spec.n_layers;
    P.n_qpt = c->spec.n_qpt;
    P.n_phi = c->spec.n_phi;
    P.log2_phi = c->log2_phi;
    P.shift = c->shift;
    P.qpt_lo = c->spec.qpt_lo;
    P.qpt_w = (c->spec.qpt_hi - c->spec.qpt_lo) / c->spec.n_qpt;
    P.inv_curv = 1.0 / (0.299792458e-3 * c->spec.b_tesla);
    const uint64_t blocks = std::min<uint64_t>((capacity + 3) / 4, uint64_t(c->n_cu) * 16);
    KernelTimer t;
    prof_begin(c, "cluster_fit", s, &t);
    if (with_z)
        hipLaunchKernelGGL(k_fit<true>, dim3(uint32_t(std::max<uint64_t>(blocks, 1))), dim3(256), 0, s, P);
    else
        hipLaunchKernelGGL(k_fit<false>, dim3(uint32_t(std::max<uint64_t>(blocks, 1))), dim3(256), 0, s, P);
    prof_end(c, s, &t);
    return hipGetLastError();
}

}  // namespace hough
