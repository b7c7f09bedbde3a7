// Host side of the unbalanced Young force (Sec. IV E, Eq. 17-18), shared by
// the single-lattice and the batched entry points: the counting parameters
// of one measured substrate, and Eq. 18 / Eq. 17 from the footprint counts.
#pragma once

#include <cmath>
#include <cstring>

#include "host.hpp"
#include "kernels.hpp"
#include "lbm.h"

namespace lbm {

// default density band of the footprint when both bounds are zero
inline void young_band(const lbm_young_opts& yo, double& lo, double& hi) {
    lo = yo.band_lo;
    hi = yo.band_hi;
    if (lo == 0.0 && hi == 0.0) {
        lo = 0.1;
        hi = 0.9;
    }
}

inline bool young_opts_ok(const lbm_young_opts& yo) {
    double lo, hi;
    young_band(yo, lo, hi);
    return std::isfinite(yo.gamma) && yo.roughness > 0.0 && lo > 0.0 && lo < hi && hi < 1.0;
}

// counting parameters: the substrate, its stripes, the drop axis and sectors
// of the measurement, and the density band rho_g + [lo, hi] (rho_l - rho_g)
inline YoungParams young_params(const Solid& so, const lbm_angle& a, int dim, double rho_g, double rho_l,
                                double lo, double hi) {
    YoungParams yp{};
    for (int k = 0; k < 3; ++k) {
        yp.c[k] = k < dim ? so.c[k] : 0.0;
        yp.pole[k] = so.pole[k];
        yp.axis[k] = a.axis[k];
    }
    yp.R = so.r;
    yp.concave = so.concave;
    yp.width = so.width;
    yp.wet_mode = so.wet_mode;
    yp.n_sectors = a.n_sectors;
    yp.dim = dim;
    yp.lo = rho_g + lo * (rho_l - rho_g);
    yp.hi = rho_g + hi * (rho_l - rho_g);
    return yp;
}

// Eq. 18 with phi_d the footprint share on the mu_w surface, then Eq. 17,
// in FP64; h holds (count on the mu_w surface, count on the mu_w2 surface)
// per sector
inline void young_from_counts(const lbm_young_opts& yo, const lbm_angle& a, const unsigned* h, lbm_young* out) {
    const double c1 = std::cos(yo.theta1_deg * M_PI / 180.0), c2 = std::cos(yo.theta2_deg * M_PI / 180.0);
    for (int k = 0; k < a.n_sectors; ++k) {
        out->count[k][0] = (int32_t)h[2 * k];
        out->count[k][1] = (int32_t)h[2 * k + 1];
        const unsigned tot = h[2 * k] + h[2 * k + 1];
        if (!tot) continue;
        const double phi = (double)h[2 * k] / (double)tot;
        double ce = yo.roughness * phi * c1 + (1.0 - phi) * c2;
        ce = ce > 1.0 ? 1.0 : (ce < -1.0 ? -1.0 : ce);
        out->phi_d[k] = phi;
        out->theta_eq_deg[k] = std::acos(ce) * 180.0 / M_PI;
        if (!std::isnan(a.sector_deg[k])) out->force[k] = yo.gamma * (std::cos(a.sector_deg[k] * M_PI / 180.0) - ce);
    }
}

// an empty result: every value NaN, the measurement's step and status
inline void young_clear(const lbm_angle& a, lbm_status status, lbm_young* out) {
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < LBM_MAX_SECTORS; ++k) out->phi_d[k] = out->theta_eq_deg[k] = out->force[k] = NAN;
    out->step = a.step;
    out->n_sectors = a.n_sectors;
    out->status = status;
}

}  // namespace lbm
