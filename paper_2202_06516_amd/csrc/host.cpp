// host.cpp -- thermodynamics (Peng-Robinson, Maxwell) and lattice geometry on
// the host, computed once per context.
#include "host.hpp"

#include <cmath>
#include <cstdio>

namespace lbm {

// --- Peng-Robinson (Eq. 10-11) ---------------------------------------------

double pr_alpha(double Tr, double omega) {
    const double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + m * (1.0 - std::sqrt(Tr));
    return s * s;
}

double pr_pressure(double rho, double T, double a, double b, double R, double alpha) {
    const double br = b * rho;
    return rho * R * T / (1.0 - br) - a * alpha * rho * rho / (1.0 + 2.0 * br - br * br);
}

double pr_chem(double rho, double T, double a, double b, double R, double alpha) {
    const double br = b * rho, r2 = std::sqrt(2.0);
    return R * T * std::log(rho / (1.0 - br)) -
           a * alpha / (2.0 * r2 * b) * std::log((r2 - 1.0 + br) / (r2 + 1.0 - br)) + R * T / (1.0 - br) -
           a * alpha * rho / (1.0 + 2.0 * br - br * br);
}

static double pr_dpdrho(double rho, double T, double a, double b, double R, double alpha) {
    const double br = b * rho, D = 1.0 + 2.0 * br - br * br;
    return R * T / ((1.0 - br) * (1.0 - br)) - a * alpha * 2.0 * rho * (1.0 + br) / (D * D);
}

// Critical point from the triple-root condition of the cubic form of Eq. 10:
// B_c = b p_c / (R T_c) is the real root of 64 B^3 + 6 B^2 + 12 B - 1 = 0,
// Z_c = (1 - B_c) / 3, A_c = 3 Z_c^2 + 3 B_c^2 + 2 B_c, T_c = (B_c/A_c) a/(b R).
static void pr_critical(PRState& s) {
    double B = 0.08;
    for (int it = 0; it < 60; ++it) {
        const double f = ((64.0 * B + 6.0) * B + 12.0) * B - 1.0;
        const double df = (192.0 * B + 12.0) * B + 12.0;
        B -= f / df;
    }
    const double Z = (1.0 - B) / 3.0;
    const double A = 3.0 * Z * Z + 3.0 * B * B + 2.0 * B;
    s.Tc = B / A * s.a / (s.b * s.R);
    s.rhoc = B / (Z * s.b);
}

bool pr_solve(PRState& s, std::string& err) {
    pr_critical(s);
    s.T = s.Tr * s.Tc;
    s.alpha = pr_alpha(s.Tr, s.omega);
    const double T = s.T, a = s.a, b = s.b, R = s.R, al = s.alpha;
    if (!(s.Tr > 0.0 && s.Tr < 1.0)) {
        err = "Tr must lie in (0, 1) for two coexisting phases";
        return false;
    }
    // spinodals: the two zeros of dp/drho on (0, 1/b)
    const int n = 40000;
    double sg = -1, sl = -1;
    double prev = pr_dpdrho(1e-12, T, a, b, R, al);
    for (int i = 1; i < n; ++i) {
        const double r = (double)i / n / b;
        const double v = pr_dpdrho(r, T, a, b, R, al);
        if (sg < 0 && prev > 0 && v <= 0) sg = r;
        if (sg > 0 && sl < 0 && prev <= 0 && v > 0) sl = r;
        prev = v;
    }
    if (sg < 0 || sl < 0) {
        err = "no spinodal pair: not in the two-phase region";
        return false;
    }
    auto refine = [&](double r, double sign) {
        double lo = r - 1.0 / n / b, hi = r;
        for (int k = 0; k < 200; ++k) {
            const double m = 0.5 * (lo + hi);
            if (sign * pr_dpdrho(m, T, a, b, R, al) > 0) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    sg = refine(sg, 1.0);
    sl = refine(sl, -1.0);
    // mu is increasing on both stable branches; for a trial mu0 between the
    // spinodal values find rho_g(mu0) and rho_l(mu0); the coexisting pair
    // has equal pressures.  Bisection on mu0.
    auto chem = [&](double r) { return pr_chem(r, T, a, b, R, al); };
    auto invert = [&](double mu0, double lo, double hi) {
        for (int k = 0; k < 300; ++k) {
            const double m = 0.5 * (lo + hi);
            if (chem(m) < mu0) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    double mlo = chem(sl), mhi = chem(sg);
    double rg = 0, rl = 0;
    for (int it = 0; it < 200; ++it) {
        const double m0 = 0.5 * (mlo + mhi);
        rg = invert(m0, 1e-300, sg);
        rl = invert(m0, sl, (1.0 - 1e-15) / b);
        const double dp = pr_pressure(rl, T, a, b, R, al) - pr_pressure(rg, T, a, b, R, al);
        // raising mu0 raises p_l faster than p_g (dp = rho dmu)
        if (dp > 0) mhi = m0; else mlo = m0;
    }
    // Newton polish on (rho_g, rho_l): p_l - p_g = 0, mu_l - mu_g = 0
    for (int it = 0; it < 8; ++it) {
        const double f1 = pr_pressure(rl, T, a, b, R, al) - pr_pressure(rg, T, a, b, R, al);
        const double f2 = chem(rl) - chem(rg);
        const double pg = pr_dpdrho(rg, T, a, b, R, al), pl = pr_dpdrho(rl, T, a, b, R, al);
        // d mu / d rho = (dp/drho) / rho
        const double J11 = -pg, J12 = pl, J21 = -pg / rg, J22 = pl / rl;
        const double det = J11 * J22 - J12 * J21;
        if (det == 0.0 || !std::isfinite(det)) break;
        const double dg = (f1 * J22 - J12 * f2) / det, dl = (J11 * f2 - J21 * f1) / det;
        const double ng = rg - dg, nl = rl - dl;
        if (!(ng > 0 && nl > 0 && nl * b < 1.0)) break;
        rg = ng;
        rl = nl;
    }
    s.rho_g = rg;
    s.rho_l = rl;
    s.p_sat = pr_pressure(rg, T, a, b, R, al);
    s.mu_sat = chem(rg);
    return true;
}

// --- geometry (Sec. III A) ----------------------------------------------------

namespace {

struct Lat {
    int Q;
    int e[19][3];
    double w[19];
};

Lat make_lat(int dim) {
    Lat L{};
    static const int e2[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static const int e3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L.Q = dim == 2 ? 9 : 19;
    for (int i = 0; i < L.Q; ++i) {
        for (int k = 0; k < 3; ++k) L.e[i][k] = dim == 2 ? e2[i][k] : e3[i][k];
        const int c2 = L.e[i][0] * L.e[i][0] + L.e[i][1] * L.e[i][1] + L.e[i][2] * L.e[i][2];
        if (dim == 2) L.w[i] = c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else L.w[i] = c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    return L;
}

}  // namespace

bool build_geometry(Geometry& g, int dim, const int n[3], const int wall[3], const std::vector<Solid>& solids,
                    const double* mu_map, double wall_mu, std::string& err) {
    const Lat L = make_lat(dim);
    g.dim = dim;
    g.Q = L.Q;
    g.nx = n[0];
    g.ny = n[1];
    g.nz = dim == 2 ? 1 : n[2];
    g.N = (long long)g.nx * g.ny * g.nz;
    const long long N = g.N;
    const int nn[3] = {g.nx, g.ny, g.nz};
    const bool per[3] = {!wall[0], !wall[1], dim == 2 ? true : !wall[2]};

    auto coords = [&](long long i, int& x, int& y, int& z) {
        x = (int)(i % g.nx);
        y = (int)((i / g.nx) % g.ny);
        z = (int)(i / ((long long)g.nx * g.ny));
    };
    // neighbour index or -1 beyond a wall axis
    auto nb = [&](int x, int y, int z, int i) -> long long {
        int v[3] = {x + L.e[i][0], y + L.e[i][1], z + L.e[i][2]};
        for (int k = 0; k < 3; ++k) {
            if (v[k] < 0 || v[k] >= nn[k]) {
                if (!per[k]) return -1;
                v[k] = v[k] < 0 ? v[k] + nn[k] : v[k] - nn[k];
            }
        }
        return ((long long)v[2] * g.ny + v[1]) * g.nx + v[0];
    };
    auto wall_layer = [&](int x, int y, int z) {
        const int v[3] = {x, y, z};
        for (int k = 0; k < dim; ++k)
            if (wall[k] && (v[k] < 2 || v[k] >= nn[k] - 2)) return true;
        return false;
    };
    auto inside = [&](const Solid& s, double x, double y, double z) {
        const double dx = x - s.c[0], dy = y - s.c[1], dz = dim == 3 ? z - s.c[2] : 0.0;
        const double d2 = dx * dx + dy * dy + dz * dz;
        return s.concave ? d2 >= s.r * s.r : d2 <= s.r * s.r;
    };

    std::vector<uint8_t> solid(N);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < N; ++i) {
        int x, y, z;
        coords(i, x, y, z);
        bool s = wall_layer(x, y, z);
        for (size_t k = 0; k < solids.size() && !s; ++k) s = inside(solids[k], x, y, z);
        solid[i] = s;
    }
    g.cls.assign(N, 0);
    g.nbmask.assign(N, 0);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < N; ++i) {
        int x, y, z;
        coords(i, x, y, z);
        uint32_t m = 0;
        bool fluid_nb = false;
        for (int q = 1; q < L.Q; ++q) {
            const long long j = nb(x, y, z, q);
            if (j < 0) continue;
            if (solid[j]) m |= 1u << q;
            else fluid_nb = true;
        }
        if (!solid[i]) {
            g.cls[i] = m ? (CLS_FLUID_ | CLS_BOUNDARY_) : CLS_FLUID_;
            g.nbmask[i] = m;
        } else {
            g.cls[i] = fluid_nb ? 1 : 3;
        }
    }
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < N; ++i) {
        if (g.cls[i] != 3) continue;
        int x, y, z;
        coords(i, x, y, z);
        for (int q = 1; q < L.Q; ++q) {
            const long long j = nb(x, y, z, q);
            if (j >= 0 && g.cls[j] == 1) { g.cls[i] = 2; break; }
        }
    }
    // a fluid node's fourth-order stencils reach two nodes along each axis;
    // those must be fluid or one of the two solid layers
    bool reach_ok = true;
#pragma omp parallel for schedule(static) reduction(&& : reach_ok)
    for (long long i = 0; i < N; ++i) {
        if ((g.cls[i] & 3) != 0) continue;
        int x, y, z;
        coords(i, x, y, z);
        const int v[3] = {x, y, z};
        for (int ax = 0; ax < dim; ++ax)
            for (int o = -2; o <= 2; o += 1) {
                if (!o) continue;
                int w[3] = {v[0], v[1], v[2]};
                w[ax] += o;
                if (w[ax] < 0 || w[ax] >= nn[ax]) {
                    if (!per[ax]) { reach_ok = false; continue; }
                    w[ax] = (w[ax] + nn[ax]) % nn[ax];
                }
                const long long j = ((long long)w[2] * g.ny + w[1]) * g.nx + w[0];
                if ((g.cls[j] & 3) == 3) reach_ok = false;
            }
    }
    if (!reach_ok) {
        err = "a fluid node's stencil reaches beyond the two solid layers (lattice too small for the walls)";
        return false;
    }

    auto wall_mu_of = [&](long long i, int x, int y, int z) {
        if (mu_map) return mu_map[i];
        for (const Solid& s : solids) {
            if (!inside(s, x, y, z)) continue;
            if (s.wet_mode == 0) return s.mu1;
            const double r[3] = {x - s.c[0], y - s.c[1], dim == 3 ? z - s.c[2] : 0.0};
            const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            double cp = rn > 0.0 ? (r[0] * s.pole[0] + r[1] * s.pole[1] + r[2] * s.pole[2]) / rn : 1.0;
            cp = cp > 1.0 ? 1.0 : (cp < -1.0 ? -1.0 : cp);
            const long long stripe = (long long)std::floor(s.r * std::acos(cp) / s.width);
            return (stripe % 2 == 0) ? s.mu1 : s.mu2;
        }
        return wall_mu;
    };

    g.l1_node.clear(); g.l1_mask.clear(); g.l1_inv.clear(); g.l1_mu.clear();
    g.l2_node.clear(); g.l2_mask.clear(); g.l2_inv.clear(); g.l2_mu.clear();
    g.b_node.clear(); g.b_mask.clear(); g.b_q.clear();
    g.n_fluid = 0;
    for (long long i = 0; i < N; ++i) {
        const int c = g.cls[i] & 3;
        int x, y, z;
        coords(i, x, y, z);
        if (c == 0) {
            ++g.n_fluid;
            if (!(g.cls[i] & CLS_BOUNDARY_)) continue;
            g.b_node.push_back(i);
            g.b_mask.push_back(g.nbmask[i]);
            for (int q = 0; q < L.Q; ++q) {
                double qq = 0.0;
                if (g.nbmask[i] & (1u << q)) {
                    const int X = x + L.e[q][0], Y = y + L.e[q][1], Z = z + L.e[q][2];
                    qq = 2.0;
                    // box wall layers sit halfway; a sphere cuts the link at a
                    // root of |x + q e - c| = r: the smaller one for a ball (x is
                    // outside it), the larger one for a cavity (x is inside)
                    int Xw = X, Yw = Y, Zw = Z;
                    if (Xw < 0 || Xw >= nn[0] || Yw < 0 || Yw >= nn[1] || Zw < 0 || Zw >= nn[2]) qq = 0.5;
                    else if (wall_layer(Xw, Yw, Zw)) qq = 0.5;
                    for (const Solid& s : solids) {
                        if (!inside(s, X, Y, Z)) continue;
                        const double d0[3] = {x - s.c[0], y - s.c[1], dim == 3 ? z - s.c[2] : 0.0};
                        const double ee = L.e[q][0] * L.e[q][0] + L.e[q][1] * L.e[q][1] + L.e[q][2] * L.e[q][2];
                        const double hb = d0[0] * L.e[q][0] + d0[1] * L.e[q][1] + d0[2] * L.e[q][2];
                        const double c0 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2] - s.r * s.r;
                        double disc = hb * hb - ee * c0;
                        if (disc < 0) disc = 0;
                        double root = s.concave ? (-hb + std::sqrt(disc)) / ee : (-hb - std::sqrt(disc)) / ee;
                        root = root <= 0 ? 1e-12 : (root > 1 ? 1.0 : root);
                        if (root < qq) qq = root;
                    }
                    if (qq > 1.0) qq = 0.5;
                    if (qq != 0.5) g.cls[i] |= CLS_CURVED_;
                }
                g.b_q.push_back(qq);
            }
        } else if (c == 1 || c == 2) {
            uint32_t m = 0;
            double den = 0.0;
            const int want = c == 1 ? 0 : 1;
            for (int q = 1; q < L.Q; ++q) {
                const long long j = nb(x, y, z, q);
                if (j < 0 || (g.cls[j] & 3) != want) continue;
                m |= 1u << q;
                den += L.w[q];
            }
            const double mu = wall_mu_of(i, x, y, z);
            if (c == 1) {
                g.l1_node.push_back(i); g.l1_mask.push_back(m); g.l1_inv.push_back(1.0 / den); g.l1_mu.push_back(mu);
            } else {
                g.l2_node.push_back(i); g.l2_mask.push_back(m); g.l2_inv.push_back(1.0 / den); g.l2_mu.push_back(mu);
            }
        }
    }
    return true;
}

}  // namespace lbm
