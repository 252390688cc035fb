// Host FP64 tables of the track finder: per-(layer, row) azimuth offsets and
// per-(q/pT, layer, cot) z shifts.  Built once per context; the GPU never
// evaluates a transcendental function.  Compiled with -ffp-contract=off and
// without fast-math so every expression is evaluated exactly as written
// (IEEE double, one rounding per operation, the host libm's asin).
//
// Offsets: the crossing azimuth of a circle of signed curvature rho with
// perigee (d0, phi0) at radius r is phi0 + asin(arg),
//   arg = (d0 - rho (r^2 + d0^2) / 2) / (r (1 - rho d0)),
// stored as the uint32 turn fraction of asin(arg) (two's complement wrap).
// z shifts: cot(theta) times the transverse arc length s = (2/rho) asin(rho r/2).
#include "tables.h"

#include <cmath>

namespace hough {

namespace {

constexpr double kCurvPerTesla = 0.299792458e-3;   // 1/mm per (T * 1/GeV)
constexpr double kTwoPi = 2.0 * 3.14159265358979323846;
constexpr double kTurn = 4294967296.0;

double centre(double lo, double hi, uint32_t n, uint32_t i)
{
    return lo + (i + 0.5) * ((hi - lo) / n);
}

double d0_centre(const hough_grid_spec &g, uint32_t d)
{
    return g.n_d0 == 1 ? 0.0 : centre(g.d0_lo_mm, g.d0_hi_mm, g.n_d0, d);
}

}  // namespace

bool spec_valid(const hough_grid_spec &g)
{
    if (g.n_layers < 1 || g.n_layers > kMaxLayers) return false;
    for (uint32_t l = 0; l < g.n_layers; ++l) {
        if (!(g.layer_r_mm[l] > 0.0)) return false;
        if (l > 0 && !(g.layer_r_mm[l] > g.layer_r_mm[l - 1])) return false;
    }
    if (g.n_phi < 2 || g.n_phi > 65536 || (g.n_phi & (g.n_phi - 1))) return false;
    if (g.n_qpt < 1 || g.n_d0 < 1) return false;
    if (uint64_t(g.n_d0) * g.n_qpt * g.n_phi > 0xFFFFFFFFull) return false;
    if (g.n_z0) {
        if (g.n_d0 != 1 || g.n_cot < 1 || g.n_cot > 65535 || g.n_z0 > 65535) return false;
        if (!(int64_t(g.z0_hi_um) > int64_t(g.z0_lo_um))) return false;
    }
    return true;
}

void build_offsets(const hough_grid_spec &g, uint32_t *O, uint8_t *V)
{
    const uint32_t rows = g.n_d0 * g.n_qpt;
    for (uint32_t l = 0; l < g.n_layers; ++l) {
        const double r = g.layer_r_mm[l];
        for (uint32_t d = 0; d < g.n_d0; ++d) {
            const double d0 = d0_centre(g, d);
            for (uint32_t k = 0; k < g.n_qpt; ++k) {
                const double rho = (kCurvPerTesla * g.b_tesla) * centre(g.qpt_lo, g.qpt_hi, g.n_qpt, k);
                const double den = r * (1.0 - rho * d0);
                const double arg = (d0 - rho * (r * r + d0 * d0) * 0.5) / den;
                const bool reach = (1.0 - rho * d0) > 0.0 && std::fabs(arg) <= 1.0;
                const size_t i = size_t(l) * rows + size_t(d) * g.n_qpt + k;
                V[i] = reach ? 1 : 0;
                O[i] = reach ? uint32_t(int64_t(std::llround(std::asin(arg) / kTwoPi * kTurn))) : 0u;
            }
        }
    }
}

void build_zshift(const hough_grid_spec &g, int32_t *Z)
{
    for (uint32_t k = 0; k < g.n_qpt; ++k) {
        const double rho = (kCurvPerTesla * g.b_tesla) * centre(g.qpt_lo, g.qpt_hi, g.n_qpt, k);
        for (uint32_t l = 0; l < g.n_layers; ++l) {
            const double r = g.layer_r_mm[l];
            const double s = (rho == 0.0) ? r : (2.0 / rho) * std::asin(rho * r * 0.5);
            for (uint32_t j = 0; j < g.n_cot; ++j) {
                const double cot = centre(g.cot_lo, g.cot_hi, g.n_cot, j);
                Z[(size_t(k) * g.n_layers + l) * g.n_cot + j] = int32_t(std::llround(cot * s * 1000.0));
            }
        }
    }
}

}  // namespace hough
