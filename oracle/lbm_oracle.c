/*
 * lbm_oracle.c -- plain FP64 CPU reference of the method of arXiv:2202.06516.
 *
 * TEST INFRASTRUCTURE ONLY: the correctness oracle for the GPU library.  It
 * is loaded by the tests, the smoke check and the benchmark's CPU-baseline leg
 * and by nothing else.  No code is shared with the GPU path.
 *
 * One time step, in the paper's order (Sec. II and Sec. III A):
 *   density      rho = sum_i f_i                                   (moments of Eq. 1)
 *   solid fill   two solid layers get densities by Eq. 14          (Sec. III A)
 *   mu           mu^ = k^2 psi'(rho) - kappa^ lap(rho), Eq. 11-12; wall mu on solids
 *   force        F = -rho grad(mu^) + cs^2 grad(rho) (+ rho g), Eq. 7
 *   collide      MRT, Eq. 1 with S of Sec. II A, m_eq = M f_eq(rho,u) (Eq. 2),
 *                exact-difference forcing, Eq. 13
 *   stream       Eq. 4, with the missing populations from the curved wall
 *                (linear interpolated bounce-back + exact mass correction)
 * Gradients use fourth-order central differences (Sec. II B).
 * Measurement (Sec. III B, Eq. 15, Fig. 1): isodensity rho_m crossings on
 * liquid-gas links, the crossings nearest 1 and 2 lu from the substrate, the
 * secant through them meets the substrate at the contact point, angle
 * against the substrate tangent, measured through the liquid.
 *
 * Compile with -ffp-contract=off.  OpenMP only splits independent per-node loops.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 19
#define MAXPRIM 16
enum { C_FLUID = 0, C_L1 = 1, C_L2 = 2, C_DEEP = 3 };

typedef struct {
    double c[3], r;
    int concave; /* 0: solid ball |x - c| <= r; 1: solid outside, |x - c| >= r */
    int wet_mode;
    double mu1, mu2, width, pole[3];
} ora_prim;

struct ora_ctx {
    ora_params p;
    int dim, Q, nx, ny, nz;
    long long N;
    int e[MAXQ][3];
    double w[MAXQ];
    int opp[MAXQ];
    double M[MAXQ][MAXQ], Minv[MAXQ][MAXQ], s[MAXQ];
    double Tc, T, alpha, rho_g, rho_l, mu_sat, p_sat, wall_mu;
    double *f, *fpost, *rho, *mu, *F, *muw_map;
    double *g, *gpost, *phi;   /* phase-field model: order-parameter populations and phi */
    unsigned char* cls;
    unsigned char* solid;
    int nprim;
    ora_prim prim[MAXPRIM];
    long long step;
};

/* ------------------------------------------------------------------ */
/* Peng-Robinson thermodynamics (Eq. 10, Eq. 11)                       */
/* ------------------------------------------------------------------ */

/* temperature function alpha(T) printed below Eq. 11 */
double ora_pr_alpha(double Tr, double omega) {
    double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    double t = 1.0 + m * (1.0 - sqrt(Tr));
    return t * t;
}

/* Eq. 10 */
double ora_pr_p0(double rho, double T, double a, double b, double R, double alpha) {
    return rho * R * T / (1.0 - b * rho) - a * alpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* Eq. 11 without the -kappa lap(rho) term, i.e. psi'(rho) with C = 0 (Eq. 9) */
double ora_pr_mu(double rho, double T, double a, double b, double R, double alpha) {
    double s2 = sqrt(2.0);
    double t1 = R * T * log(rho / (1.0 - b * rho));
    double t2 = a * alpha / (2.0 * s2 * b) * log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho));
    double t3 = R * T / (1.0 - b * rho);
    double t4 = a * alpha * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    return t1 - t2 + t3 - t4;
}

static double pr_dp(double rho, double T, double a, double b, double R, double alpha) {
    double D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    return R * T / ((1.0 - b * rho) * (1.0 - b * rho)) - a * alpha * (2.0 * rho + 2.0 * b * rho * rho) / (D * D);
}

static double pr_d2p(double rho, double T, double a, double b, double R, double alpha) {
    double D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    double Dp = 2.0 * b - 2.0 * b * b * rho;
    double num = 2.0 * rho + 2.0 * b * rho * rho;
    double dnum = 2.0 + 4.0 * b * rho;
    double om = 1.0 - b * rho;
    return 2.0 * b * R * T / (om * om * om) - a * alpha * (dnum * D - 2.0 * num * Dp) / (D * D * D);
}

/* critical point of Eq. 10 at alpha = 1: dp/drho = d2p/drho2 = 0 (bisection in T,
 * and for each T bisection in rho for the inflection point) */
int ora_pr_critical(double a, double b, double R, double* Tc, double* rhoc, double* pc) {
    double Tlo = 1e-6, Thi = 10.0 * a / (b * R);
    double rho_i = 0.0;
    for (int it = 0; it < 200; ++it) {
        double T = 0.5 * (Tlo + Thi);
        /* inflection: d2p changes sign from - to + ... find root of d2p on (0, 1/b) */
        double lo = 1e-9 / b, hi = (1.0 - 1e-9) / b;
        /* d2p < 0 at moderate rho for subcritical T; scan for a sign change */
        double best = lo, bestv = 1e300;
        int nscan = 4000;
        for (int i = 1; i < nscan; ++i) {
            double r = lo + (hi - lo) * i / nscan;
            double v = pr_dp(r, T, a, b, R, 1.0);
            if (v < bestv) { bestv = v; best = r; }
        }
        /* refine minimum of dp by bisection on d2p around best */
        double l2 = best - (hi - lo) / nscan, h2 = best + (hi - lo) / nscan;
        if (l2 < lo) l2 = lo;
        if (h2 > hi) h2 = hi;
        for (int j = 0; j < 200; ++j) {
            double m = 0.5 * (l2 + h2);
            if (pr_d2p(m, T, a, b, R, 1.0) < 0.0) l2 = m; else h2 = m;
        }
        rho_i = 0.5 * (l2 + h2);
        double mindp = pr_dp(rho_i, T, a, b, R, 1.0);
        if (mindp < 0.0) Tlo = T; else Thi = T;
    }
    *Tc = 0.5 * (Tlo + Thi);
    *rhoc = rho_i;
    *pc = ora_pr_p0(rho_i, *Tc, a, b, R, 1.0);
    return 0;
}

/* roots of p0(rho) = P on the gas (smallest) and liquid (largest) branches */
static int pr_branch_roots(double P, double T, double a, double b, double R, double al,
                           double rs_g, double rs_l, double* rg, double* rl) {
    /* gas branch: (0, rs_g], p increasing; liquid branch: [rs_l, 1/b), p increasing */
    double lo = 1e-300, hi = rs_g;
    if (ora_pr_p0(hi, T, a, b, R, al) < P) return -1;
    for (int i = 0; i < 300; ++i) {
        double m = 0.5 * (lo + hi);
        if (ora_pr_p0(m, T, a, b, R, al) < P) lo = m; else hi = m;
    }
    *rg = 0.5 * (lo + hi);
    lo = rs_l; hi = (1.0 - 1e-15) / b;
    if (ora_pr_p0(lo, T, a, b, R, al) > P) return -1;
    for (int i = 0; i < 300; ++i) {
        double m = 0.5 * (lo + hi);
        if (ora_pr_p0(m, T, a, b, R, al) < P) lo = m; else hi = m;
    }
    *rl = 0.5 * (lo + hi);
    return 0;
}

/* Maxwell equal-area construction (Sec. IV): p0(rho_g) = p0(rho_l) and
 * mu(rho_g) = mu(rho_l).  Bisection on the saturation pressure. */
int ora_maxwell(double T, double a, double b, double R, double al,
                double* rho_g, double* rho_l, double* p_sat, double* mu_sat) {
    /* spinodals: local max (gas side) and local min (liquid side) of p0 */
    int nscan = 20000;
    double rmax = (1.0 - 1e-9) / b;
    double rs_g = -1, rs_l = -1;
    double prev = pr_dp(rmax * 1.0 / nscan, T, a, b, R, al);
    for (int i = 2; i < nscan; ++i) {
        double r = rmax * i / nscan;
        double v = pr_dp(r, T, a, b, R, al);
        if (prev > 0 && v <= 0 && rs_g < 0) {
            double lo = rmax * (i - 1) / nscan, hi = r;
            for (int j = 0; j < 200; ++j) { double m = 0.5 * (lo + hi); if (pr_dp(m, T, a, b, R, al) > 0) lo = m; else hi = m; }
            rs_g = 0.5 * (lo + hi);
        }
        if (prev <= 0 && v > 0 && rs_g > 0 && rs_l < 0) {
            double lo = rmax * (i - 1) / nscan, hi = r;
            for (int j = 0; j < 200; ++j) { double m = 0.5 * (lo + hi); if (pr_dp(m, T, a, b, R, al) <= 0) lo = m; else hi = m; }
            rs_l = 0.5 * (lo + hi);
        }
        prev = v;
    }
    if (rs_g < 0 || rs_l < 0) return -1;
    double Plo = ora_pr_p0(rs_l, T, a, b, R, al);
    double Phi = ora_pr_p0(rs_g, T, a, b, R, al);
    if (Plo < 0) Plo = 0;
    double rg = 0, rl = 0;
    for (int it = 0; it < 300; ++it) {
        double P = 0.5 * (Plo + Phi);
        if (pr_branch_roots(P, T, a, b, R, al, rs_g, rs_l, &rg, &rl) != 0) return -2;
        double dmu = ora_pr_mu(rl, T, a, b, R, al) - ora_pr_mu(rg, T, a, b, R, al);
        /* d mu = dp / rho at fixed T, so mu_l - mu_g falls as P rises and is
         * positive below the saturation pressure */
        if (dmu > 0) Plo = P; else Phi = P;
    }
    double P = 0.5 * (Plo + Phi);
    pr_branch_roots(P, T, a, b, R, al, rs_g, rs_l, &rg, &rl);
    *rho_g = rg;
    *rho_l = rl;
    *p_sat = P;
    *mu_sat = ora_pr_mu(rg, T, a, b, R, al);
    return 0;
}

/* ------------------------------------------------------------------ */
/* lattices, equilibrium (Eq. 2), MRT transform (Eq. 1)               */
/* ------------------------------------------------------------------ */

static const int E2[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int E3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

int ora_lattice(int dim, int* Q, int* e, double* w) {
    int q = dim == 2 ? 9 : 19;
    *Q = q;
    for (int i = 0; i < q; ++i) {
        const int* v = dim == 2 ? E2[i] : E3[i];
        int e2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        for (int d = 0; d < 3; ++d) e[i * 3 + d] = v[d];
        if (dim == 2) w[i] = e2 == 0 ? 4.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else w[i] = e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    return 0;
}

/* rows of M as polynomials of the velocity: D2Q9 in the Lallemand-Luo moment
 * order (rho, e, eps, jx, qx, jy, qy, pxx, pxy) matching S of Sec. II A;
 * D3Q19 in the d'Humieres et al. 19-moment order. */
void ora_mrt_matrix(int dim, double* M) {
    int Q, e[MAXQ * 3];
    double w[MAXQ];
    ora_lattice(dim, &Q, e, w);
    for (int i = 0; i < Q; ++i) {
        double x = e[i * 3], y = e[i * 3 + 1], z = e[i * 3 + 2];
        double c2 = x * x + y * y + z * z;
        double col[MAXQ];
        if (dim == 2) {
            col[0] = 1.0;
            col[1] = -4.0 + 3.0 * c2;
            col[2] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
            col[3] = x;
            col[4] = (-5.0 + 3.0 * c2) * x;
            col[5] = y;
            col[6] = (-5.0 + 3.0 * c2) * y;
            col[7] = x * x - y * y;
            col[8] = x * y;
        } else {
            col[0] = 1.0;
            col[1] = 19.0 * c2 - 30.0;
            col[2] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
            col[3] = x;
            col[4] = (5.0 * c2 - 9.0) * x;
            col[5] = y;
            col[6] = (5.0 * c2 - 9.0) * y;
            col[7] = z;
            col[8] = (5.0 * c2 - 9.0) * z;
            col[9] = 3.0 * x * x - c2;
            col[10] = (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
            col[11] = y * y - z * z;
            col[12] = (3.0 * c2 - 5.0) * (y * y - z * z);
            col[13] = x * y;
            col[14] = y * z;
            col[15] = x * z;
            col[16] = (y * y - z * z) * x;
            col[17] = (z * z - x * x) * y;
            col[18] = (x * x - y * y) * z;
        }
        for (int k = 0; k < Q; ++k) M[k * Q + i] = col[k];
    }
}

/* Eq. 2 */
void ora_feq(int dim, double rho, const double u[3], double* feq) {
    int Q, e[MAXQ * 3];
    double w[MAXQ];
    ora_lattice(dim, &Q, e, w);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double eu = e[i * 3] * u[0] + e[i * 3 + 1] * u[1] + e[i * 3 + 2] * u[2];
        feq[i] = rho * w[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Gauss-Jordan inverse with partial pivoting (library-style step) */
static int invert(int n, const double* A, double* Ainv) {
    double m[MAXQ][2 * MAXQ];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) m[i][j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
        if (m[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) { double t = m[c][j]; m[c][j] = m[piv][j]; m[piv][j] = t; }
        double d = m[c][c];
        for (int j = 0; j < 2 * n; ++j) m[c][j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c || m[r][c] == 0.0) continue;
            double fct = m[r][c];
            for (int j = 0; j < 2 * n; ++j) m[r][j] -= fct * m[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = m[i][j + n];
    return 0;
}

static void rates(const ora_params* p, int dim, double* s) {
    double sv = 1.0 / p->tau;
    if (dim == 2) {
        double r[9] = {0, p->s_e, p->s_eps, 0, p->s_q, 0, p->s_q, sv, sv};
        memcpy(s, r, sizeof r);
    } else {
        double r[19] = {0, p->s_e, p->s_eps, 0, p->s_q, 0, p->s_q, 0, p->s_q, sv,
                        p->s_pi, sv, p->s_pi, sv, sv, sv, p->s_m, p->s_m, p->s_m};
        memcpy(s, r, sizeof r);
    }
    if (p->bgk) {
        int Q = dim == 2 ? 9 : 19;
        for (int k = 0; k < Q; ++k) s[k] = 1.0 / p->tau;
    }
}

/* Eq. 1 with m_eq = M f_eq(rho,u) and Eq. 13 forcing, for one node */
static void collide_one(int dim, int Q, const int e[][3], const double M[][MAXQ],
                        const double Minv[][MAXQ], const double* s, const double* f,
                        const double F[3], double* out) {
    double rho = 0, u[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) u[d] += f[i] * e[i][d];
    }
    for (int d = 0; d < 3; ++d) u[d] /= rho;
    double feq[MAXQ], feq2[MAXQ], m[MAXQ], meq[MAXQ], ms[MAXQ];
    ora_feq(dim, rho, u, feq);
    double u2[3] = {u[0] + F[0] / rho, u[1] + F[1] / rho, u[2] + F[2] / rho};
    ora_feq(dim, rho, u2, feq2);
    for (int k = 0; k < Q; ++k) {
        m[k] = 0;
        meq[k] = 0;
        for (int i = 0; i < Q; ++i) {
            m[k] += M[k][i] * f[i];
            meq[k] += M[k][i] * feq[i];
        }
        ms[k] = m[k] - s[k] * (m[k] - meq[k]);
    }
    for (int i = 0; i < Q; ++i) {
        double v = 0;
        for (int k = 0; k < Q; ++k) v += Minv[i][k] * ms[k];
        out[i] = v + (feq2[i] - feq[i]);
    }
}

void ora_collide_node(const ora_params* p, const double* f, const double F[3], double* fout) {
    int dim = p->dim, Q, ev[MAXQ * 3];
    double w[MAXQ], Mf[MAXQ * MAXQ], Mi[MAXQ * MAXQ], s[MAXQ];
    ora_lattice(dim, &Q, ev, w);
    ora_mrt_matrix(dim, Mf);
    invert(Q, Mf, Mi);
    rates(p, dim, s);
    int e[MAXQ][3];
    double M[MAXQ][MAXQ], Minv[MAXQ][MAXQ];
    for (int i = 0; i < Q; ++i)
        for (int d = 0; d < 3; ++d) e[i][d] = ev[i * 3 + d];
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) { M[i][j] = Mf[i * Q + j]; Minv[i][j] = Mi[i * Q + j]; }
    collide_one(dim, Q, (const int(*)[3])e, (const double(*)[MAXQ])M, (const double(*)[MAXQ])Minv, s, f, F, fout);
}

/* ------------------------------------------------------------------ */
/* context, geometry                                                   */
/* ------------------------------------------------------------------ */

static inline long long lin(const ora_ctx* c, int x, int y, int z) {
    return ((long long)z * c->ny + y) * c->nx + x;
}

/* neighbour with periodic wrap on periodic axes; -1 outside a wall axis */
static long long nbr(const ora_ctx* c, int x, int y, int z, int dx, int dy, int dz) {
    int X = x + dx, Y = y + dy, Z = z + dz;
    int n[3] = {c->nx, c->ny, c->nz};
    int v[3] = {X, Y, Z};
    for (int d = 0; d < 3; ++d) {
        if (v[d] < 0 || v[d] >= n[d]) {
            if (c->p.wall[d] || (d == 2 && c->dim == 2)) return -1;
            v[d] = ((v[d] % n[d]) + n[d]) % n[d];
        }
    }
    return lin(c, v[0], v[1], v[2]);
}

ora_ctx* ora_create(const ora_params* p) {
    if (p->dim != 2 && p->dim != 3) return NULL;
    ora_ctx* c = (ora_ctx*)calloc(1, sizeof(ora_ctx));
    c->p = *p;
    c->dim = p->dim;
    c->nx = p->n[0];
    c->ny = p->n[1];
    c->nz = p->dim == 2 ? 1 : p->n[2];
    c->N = (long long)c->nx * c->ny * c->nz;
    int ev[MAXQ * 3];
    ora_lattice(c->dim, &c->Q, ev, c->w);
    for (int i = 0; i < c->Q; ++i)
        for (int d = 0; d < 3; ++d) c->e[i][d] = ev[i * 3 + d];
    for (int i = 0; i < c->Q; ++i)
        for (int j = 0; j < c->Q; ++j)
            if (c->e[j][0] == -c->e[i][0] && c->e[j][1] == -c->e[i][1] && c->e[j][2] == -c->e[i][2]) c->opp[i] = j;
    double Mf[MAXQ * MAXQ], Mi[MAXQ * MAXQ];
    ora_mrt_matrix(c->dim, Mf);
    if (invert(c->Q, Mf, Mi) != 0) { free(c); return NULL; }
    for (int i = 0; i < c->Q; ++i)
        for (int j = 0; j < c->Q; ++j) { c->M[i][j] = Mf[i * c->Q + j]; c->Minv[i][j] = Mi[i * c->Q + j]; }
    rates(p, c->dim, c->s);
    double rhoc, pc;
    ora_pr_critical(p->a, p->b, p->R, &c->Tc, &rhoc, &pc);
    c->T = p->Tr * c->Tc;
    c->alpha = ora_pr_alpha(p->Tr, p->omega);
    if (ora_maxwell(c->T, p->a, p->b, p->R, c->alpha, &c->rho_g, &c->rho_l, &c->p_sat, &c->mu_sat) != 0) {
        free(c);
        return NULL;
    }
    if (p->rho_l > 0) c->rho_l = p->rho_l;
    if (p->rho_g > 0) c->rho_g = p->rho_g;
    c->wall_mu = isnan(p->wall_mu) ? p->k * p->k * c->mu_sat : p->wall_mu;
    if (p->model == 1) {
        /* pseudopotential: the coexistence densities are inputs (they depend
         * on the forcing scheme, not on a closed-form construction), and the
         * wall value is a wall density, neutral default midway */
        if (!(p->rho_l > 0 && p->rho_g > 0 && p->rho_l > p->rho_g)) { free(c); return NULL; }
        if (isnan(p->wall_mu)) c->wall_mu = 0.5 * (p->rho_l + p->rho_g);
    } else if (p->model == 2) {
        /* phase field: the two bulk phases are phi = 1 (liquid) and phi = -1;
         * the measurement's isolevel is their mean, 0; the wall value is a wall
         * order parameter, neutral default 0 */
        if (!(p->pf_A > 0 && p->pf_kappa > 0 && p->pf_gamma > 0 && p->pf_tau > 0.5 && p->pf_rho0 > 0)) {
            free(c);
            return NULL;
        }
        c->rho_l = 1.0;
        c->rho_g = -1.0;
        if (isnan(p->wall_mu)) c->wall_mu = 0.0;
    } else if (p->model != 0) {
        free(c);
        return NULL;
    }
    size_t N = (size_t)c->N, Q = (size_t)c->Q;
    c->f = (double*)calloc(Q * N, sizeof(double));
    c->fpost = (double*)calloc(Q * N, sizeof(double));
    c->rho = (double*)calloc(N, sizeof(double));
    c->mu = (double*)calloc(N, sizeof(double));
    c->F = (double*)calloc(3 * N, sizeof(double));
    c->cls = (unsigned char*)calloc(N, 1);
    c->solid = (unsigned char*)calloc(N, 1);
    if (!c->f || !c->fpost || !c->rho || !c->mu || !c->F || !c->cls || !c->solid) { ora_destroy(c); return NULL; }
    if (p->model == 2) {
        c->g = (double*)calloc(Q * N, sizeof(double));
        c->gpost = (double*)calloc(Q * N, sizeof(double));
        c->phi = (double*)calloc(N, sizeof(double));
        if (!c->g || !c->gpost || !c->phi) { ora_destroy(c); return NULL; }
    }
    ora_build(c);
    return c;
}

void ora_destroy(ora_ctx* c) {
    if (!c) return;
    free(c->f); free(c->fpost); free(c->rho); free(c->mu); free(c->F); free(c->cls);
    free(c->solid); free(c->muw_map);
    free(c->g); free(c->gpost); free(c->phi);
    free(c);
}

static int add_prim(ora_ctx* c, int concave, const double centre[3], double radius, int wet_mode,
                    double mu_w, double mu_w2, double stripe_width, const double pole[3]) {
    if (c->nprim >= MAXPRIM || radius <= 0) return -1;
    ora_prim* pr = &c->prim[c->nprim++];
    memset(pr, 0, sizeof *pr);
    pr->concave = concave;
    for (int d = 0; d < 3; ++d) pr->c[d] = centre[d];
    if (c->dim == 2) pr->c[2] = 0;
    pr->r = radius;
    pr->wet_mode = wet_mode;
    pr->mu1 = mu_w;
    pr->mu2 = mu_w2;
    pr->width = stripe_width;
    double pl[3] = {0, c->dim == 2 ? 1.0 : 0.0, c->dim == 2 ? 0.0 : 1.0};
    if (pole) { pl[0] = pole[0]; pl[1] = pole[1]; pl[2] = c->dim == 2 ? 0.0 : pole[2]; }
    double nrm = sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
    for (int d = 0; d < 3; ++d) pr->pole[d] = pl[d] / nrm;
    return 0;
}

/* convex substrate of Fig. 2(a): a solid circle (2-D) or ball (3-D) */
int ora_add_sphere(ora_ctx* c, const double centre[3], double radius, int wet_mode,
                   double mu_w, double mu_w2, double stripe_width, const double pole[3]) {
    return add_prim(c, 0, centre, radius, wet_mode, mu_w, mu_w2, stripe_width, pole);
}

/* concave substrate of Fig. 2(b): the fluid fills the inside of the circle or
 * ball and everything outside it is solid */
int ora_add_cavity(ora_ctx* c, const double centre[3], double radius, int wet_mode,
                   double mu_w, double mu_w2, double stripe_width, const double pole[3]) {
    return add_prim(c, 1, centre, radius, wet_mode, mu_w, mu_w2, stripe_width, pole);
}

int ora_set_muw_map(ora_ctx* c, const double* map) {
    free(c->muw_map);
    c->muw_map = NULL;
    if (map) {
        c->muw_map = (double*)malloc(sizeof(double) * (size_t)c->N);
        memcpy(c->muw_map, map, sizeof(double) * (size_t)c->N);
    }
    return 0;
}

static int inside_prim(const ora_prim* pr, double x, double y, double z) {
    double dx = x - pr->c[0], dy = y - pr->c[1], dz = z - pr->c[2];
    double d2 = dx * dx + dy * dy + dz * dz, r2 = pr->r * pr->r;
    return pr->concave ? d2 >= r2 : d2 <= r2;
}

static int is_wall_layer(const ora_ctx* c, int x, int y, int z) {
    int v[3] = {x, y, z}, n[3] = {c->nx, c->ny, c->nz};
    for (int d = 0; d < c->dim; ++d)
        if (c->p.wall[d] && (v[d] < 2 || v[d] >= n[d] - 2)) return 1;
    return 0;
}

/* node classes of Sec. III A: fluid, first solid layer (a fluid neighbour among
 * the lattice links), second layer (a first-layer neighbour), deeper solid */
int ora_build(ora_ctx* c) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        int s = is_wall_layer(c, x, y, z);
        for (int k = 0; k < c->nprim && !s; ++k) s = inside_prim(&c->prim[k], x, y, z);
        c->solid[n] = (unsigned char)s;
    }
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        unsigned char k = C_FLUID;
        if (c->solid[n]) {
            k = C_DEEP;
            for (int i = 1; i < c->Q; ++i) {
                long long m = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
                if (m >= 0 && !c->solid[m]) { k = C_L1; break; }
            }
        }
        c->cls[n] = k;
    }
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_DEEP) continue;
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        for (int i = 1; i < c->Q; ++i) {
            long long m = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
            if (m >= 0 && c->cls[m] == C_L1) { c->cls[n] = C_L2; break; }
        }
    }
    return 0;
}

/* chemical potential prescribed on a solid node (Sec. III A): per-node map if
 * given, else the primitive's uniform value or latitude stripes, else the wall */
static double wall_mu_at(const ora_ctx* c, long long n, int x, int y, int z) {
    if (c->muw_map) return c->muw_map[n];
    for (int k = 0; k < c->nprim; ++k) {
        const ora_prim* pr = &c->prim[k];
        if (!inside_prim(pr, x, y, z)) continue;
        if (pr->wet_mode == 0) return pr->mu1;
        double r[3] = {x - pr->c[0], y - pr->c[1], z - pr->c[2]};
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double cosp = rn > 0 ? (r[0] * pr->pole[0] + r[1] * pr->pole[1] + r[2] * pr->pole[2]) / rn : 1.0;
        if (cosp > 1) cosp = 1;
        if (cosp < -1) cosp = -1;
        double psi = acos(cosp);
        long long stripe = (long long)floor(pr->r * psi / pr->width);
        return (stripe % 2 == 0) ? pr->mu1 : pr->mu2;
    }
    return c->wall_mu;
}

/* wall distance fraction of the link from fluid x along e_dir (Sec. III A):
 * the root in (0,1] of |x + q e - C| = R -- the smaller one for a ball, whose
 * outside x is in, the larger one for a cavity, whose inside x is in -- and
 * 1/2 for a box wall */
double ora_link_q(ora_ctx* c, int x, int y, int z, int dir) {
    long long n = lin(c, x, y, z);
    if (c->solid[n]) return -1;
    int* e = c->e[dir];
    long long m = nbr(c, x, y, z, e[0], e[1], e[2]);
    if (m < 0 || !c->solid[m]) return -1;
    double q = 2.0;
    int X = x + e[0], Y = y + e[1], Z = z + e[2];
    if (is_wall_layer(c, X, Y, Z)) q = 0.5;
    for (int k = 0; k < c->nprim; ++k) {
        const ora_prim* pr = &c->prim[k];
        if (!inside_prim(pr, X, Y, Z)) continue;
        double d[3] = {x - pr->c[0], y - pr->c[1], z - pr->c[2]};
        double A = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        double B = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
        double Cc = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - pr->r * pr->r;
        double disc = B * B - A * Cc;
        if (disc < 0) disc = 0;
        double r = pr->concave ? (-B + sqrt(disc)) / A : (-B - sqrt(disc)) / A;
        if (r <= 0) r = 1e-12;
        if (r > 1) r = 1;
        if (r < q) q = r;
    }
    if (q > 1.0) q = 0.5; /* solid by periodic image only; not expected */
    return q;
}

/* ------------------------------------------------------------------ */
/* initial state (Eq. 16)                                              */
/* ------------------------------------------------------------------ */

static void set_equilibrium_state(ora_ctx* c) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        double u[3] = {0, 0, 0}, feq[MAXQ];
        if (c->cls[n] == C_FLUID) ora_feq(c->dim, c->rho[n], u, feq);
        else for (int i = 0; i < c->Q; ++i) feq[i] = 0.0;
        for (int i = 0; i < c->Q; ++i) c->f[(size_t)i * c->N + n] = feq[i];
        if (c->p.model == 2) {
            /* the order parameter at rest in the rest population */
            for (int i = 0; i < c->Q; ++i) c->g[(size_t)i * c->N + n] = 0.0;
            c->g[n] = c->cls[n] == C_FLUID ? c->phi[n] : 0.0;
        }
    }
    c->step = 0;
}

int ora_init_drops(ora_ctx* c, const double* centres, const double* radii, int nd, double W) {
    if (nd < 1 || W <= 0) return -1;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        double best = -1e300;
        for (int d = 0; d < nd; ++d) {
            double dx = x - centres[3 * d], dy = y - centres[3 * d + 1], dz = c->dim == 3 ? z - centres[3 * d + 2] : 0.0;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double v = 0.5 * (c->rho_g + c->rho_l) + 0.5 * (c->rho_g - c->rho_l) * tanh(2.0 * (r - radii[d]) / W);
            if (v > best) best = v;
        }
        /* phase field: Eq. 16 profiles the order parameter (rho_l = 1, rho_g = -1), the fluid density is rho0 */
        if (c->p.model == 2) {
            c->phi[n] = c->cls[n] == C_FLUID ? best : 0.0;
            c->rho[n] = c->cls[n] == C_FLUID ? c->p.pf_rho0 : 0.0;
        } else {
            c->rho[n] = c->cls[n] == C_FLUID ? best : 0.0;
        }
    }
    set_equilibrium_state(c);
    return 0;
}

/* the field the measurement reads (phase field: phi) set on fluid nodes; the
 * populations set at rest around it */
int ora_set_rho(ora_ctx* c, const double* rho) {
    for (long long n = 0; n < c->N; ++n) {
        if (c->p.model == 2) {
            c->phi[n] = c->cls[n] == C_FLUID ? rho[n] : 0.0;
            c->rho[n] = c->cls[n] == C_FLUID ? c->p.pf_rho0 : 0.0;
        } else {
            c->rho[n] = c->cls[n] == C_FLUID ? rho[n] : 0.0;
        }
    }
    set_equilibrium_state(c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* step phases                                                         */
/* ------------------------------------------------------------------ */

void ora_phase_density(ora_ctx* c) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_FLUID) continue;
        double s = 0;
        for (int i = 0; i < c->Q; ++i) s += c->f[(size_t)i * c->N + n];
        c->rho[n] = s;
        if (c->p.model == 2) {
            /* phase field: the order parameter is the zeroth moment of g */
            double q = 0;
            for (int i = 0; i < c->Q; ++i) q += c->g[(size_t)i * c->N + n];
            c->phi[n] = q;
        }
    }
}

/* Eq. 14: first layer from fluid neighbours, then second layer from first-layer ones */
static void fill_layer(ora_ctx* c, int layer, int from) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != layer) continue;
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        double num = 0, den = 0;
        for (int i = 1; i < c->Q; ++i) {
            long long m = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
            if (m < 0 || c->cls[m] != from) continue;
            num += c->w[i] * c->rho[m];
            den += c->w[i];
        }
        c->rho[n] = num / den;
    }
}

void ora_phase_fill(ora_ctx* c) {
    if (c->p.model == 2) {
        /* phase field: both solid layers hold the wall order parameter (a
         * virtual phi, the wetting condition of this model), which the
         * Laplacian of mu and the gradient of the force reach */
        for (long long n = 0; n < c->N; ++n) {
            if (c->cls[n] != C_L1 && c->cls[n] != C_L2) continue;
            int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
            c->phi[n] = wall_mu_at(c, n, x, y, z);
        }
        return;
    }
    fill_layer(c, C_L1, C_FLUID);
    fill_layer(c, C_L2, C_L1);
}

/* fourth-order central differences along one axis */
static double d1(const ora_ctx* c, const double* phi, int x, int y, int z, int ax) {
    int o[3] = {0, 0, 0};
    double v[5];
    for (int k = -2; k <= 2; ++k) {
        o[ax] = k;
        long long m = nbr(c, x, y, z, o[0], o[1], o[2]);
        v[k + 2] = phi[m];
    }
    return (v[0] - 8.0 * v[1] + 8.0 * v[3] - v[4]) / 12.0;
}

static double d2(const ora_ctx* c, const double* phi, int x, int y, int z, int ax) {
    int o[3] = {0, 0, 0};
    double v[5];
    for (int k = -2; k <= 2; ++k) {
        o[ax] = k;
        long long m = nbr(c, x, y, z, o[0], o[1], o[2]);
        v[k + 2] = phi[m];
    }
    return (-v[0] + 16.0 * v[1] - 30.0 * v[2] + 16.0 * v[3] - v[4]) / 12.0;
}

/* pseudopotential of the Shan-Chen model, psi(rho) = 1 - exp(-rho) (rho_0 = 1) */
static double sc_psi(double rho) { return 1.0 - exp(-rho); }

/* Eq. 11 / Eq. 12 on fluid nodes; the prescribed wall value on both solid
 * layers.  Pseudopotential model: psi(rho) on fluid nodes and psi of the
 * wall density on the layers (the virtual-density wetting condition). */
void ora_phase_mu(ora_ctx* c) {
    const ora_params* p = &c->p;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        if (p->model == 2) {
            /* phase field: mu = dF/dphi = A (phi^3 - phi) - kappa lap(phi) */
            if (c->cls[n] == C_FLUID) {
                double lap = 0;
                for (int ax = 0; ax < c->dim; ++ax) lap += d2(c, c->phi, x, y, z, ax);
                double f = c->phi[n];
                c->mu[n] = p->pf_A * (f * f * f - f) - p->pf_kappa * lap;
            } else {
                c->mu[n] = 0.0;
            }
        } else if (p->model == 1) {
            if (c->cls[n] == C_FLUID) c->mu[n] = sc_psi(c->rho[n]);
            else if (c->cls[n] == C_L1 || c->cls[n] == C_L2) c->mu[n] = sc_psi(wall_mu_at(c, n, x, y, z));
            else c->mu[n] = 0.0;
        } else if (c->cls[n] == C_FLUID) {
            double lap = 0;
            for (int ax = 0; ax < c->dim; ++ax) lap += d2(c, c->rho, x, y, z, ax);
            c->mu[n] = p->k * p->k * ora_pr_mu(c->rho[n], c->T, p->a, p->b, p->R, c->alpha) - p->kappa * lap;
        } else if (c->cls[n] == C_L1 || c->cls[n] == C_L2) {
            c->mu[n] = wall_mu_at(c, n, x, y, z);
        } else {
            c->mu[n] = 0.0;
        }
    }
}

/* Eq. 7, plus the body force rho g once the step counter reaches g_start;
 * the pseudopotential model takes the Shan-Chen interaction force instead */
void ora_phase_force(ora_ctx* c) {
    const ora_params* p = &c->p;
    int grav = c->step >= p->g_start;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        for (int d = 0; d < 3; ++d) c->F[(size_t)d * c->N + n] = 0.0;
        if (c->cls[n] != C_FLUID) continue;
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        if (p->model == 2) {
            /* phase field: the capillary force mu grad(phi) (the chemical-potential
             * form, which differs from -phi grad(mu) by a pressure gradient) */
            for (int ax = 0; ax < c->dim; ++ax) {
                double Fv = c->mu[n] * d1(c, c->phi, x, y, z, ax);
                if (grav) Fv += c->rho[n] * p->g[ax];
                c->F[(size_t)ax * c->N + n] = Fv;
            }
            continue;
        }
        if (p->model == 1) {
            /* Shan-Chen interaction with the lattice weights:
             * F = -G psi(x) sum_i w_i psi(x + e_i) e_i */
            double s[3] = {0, 0, 0};
            for (int i = 1; i < c->Q; ++i) {
                long long m = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
                if (m < 0) continue;
                for (int d = 0; d < 3; ++d) s[d] += c->w[i] * c->mu[m] * c->e[i][d];
            }
            for (int ax = 0; ax < c->dim; ++ax) {
                double Fv = -p->sc_G * c->mu[n] * s[ax];
                if (grav) Fv += c->rho[n] * p->g[ax];
                c->F[(size_t)ax * c->N + n] = Fv;
            }
            continue;
        }
        for (int ax = 0; ax < c->dim; ++ax) {
            double gm = d1(c, c->mu, x, y, z, ax);
            double gr = d1(c, c->rho, x, y, z, ax);
            double Fv = -c->rho[n] * gm + gr / 3.0;
            if (grav) Fv += c->rho[n] * p->g[ax];
            c->F[(size_t)ax * c->N + n] = Fv;
        }
    }
}

/* Phase field: BGK relaxation of the order-parameter populations toward
 *   g_i^eq = w_i [gamma mu / cs^2 + phi (e_i.v) / cs^2 + phi ((e_i.v)^2 / (2 cs^4) - v^2 / (2 cs^2))], i > 0,
 *   g_0^eq = phi - sum_{i>0} g_i^eq,
 * whose moments are phi, phi v and gamma mu I + phi v v: the Cahn-Hilliard
 * equation d phi/dt + div(phi v) = M lap(mu) with M = gamma (tau_g - 1/2).
 * v = (sum_i f_i e_i + F/2) / rho is the fluid velocity of the node. */
static void pf_collide_g(ora_ctx* c, long long n, const double* f, const double F[3]) {
    const ora_params* p = &c->p;
    const double cs2 = 1.0 / 3.0;
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < c->Q; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * c->e[i][d];
    }
    double v[3];
    for (int d = 0; d < 3; ++d) v[d] = (j[d] + 0.5 * F[d]) / rho;
    double phi = 0;
    for (int i = 0; i < c->Q; ++i) phi += c->g[(size_t)i * c->N + n];
    const double mu = c->mu[n], vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double geq[MAXQ], rest = phi;
    for (int i = 1; i < c->Q; ++i) {
        double ev = c->e[i][0] * v[0] + c->e[i][1] * v[1] + c->e[i][2] * v[2];
        geq[i] = c->w[i] * (p->pf_gamma * mu / cs2 + phi * ev / cs2 + phi * (ev * ev / (2.0 * cs2 * cs2) - vv / (2.0 * cs2)));
        rest -= geq[i];
    }
    geq[0] = rest;
    for (int i = 0; i < c->Q; ++i) {
        double gi = c->g[(size_t)i * c->N + n];
        c->gpost[(size_t)i * c->N + n] = gi - (gi - geq[i]) / p->pf_tau;
    }
}

void ora_phase_collide(ora_ctx* c) {
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        double f[MAXQ], out[MAXQ];
        if (c->cls[n] != C_FLUID) {
            for (int i = 0; i < c->Q; ++i) c->fpost[(size_t)i * c->N + n] = 0.0;
            continue;
        }
        for (int i = 0; i < c->Q; ++i) f[i] = c->f[(size_t)i * c->N + n];
        double F[3] = {c->F[n], c->F[(size_t)c->N + n], c->F[2 * (size_t)c->N + n]};
        collide_one(c->dim, c->Q, (const int(*)[3])c->e, (const double(*)[MAXQ])c->M,
                    (const double(*)[MAXQ])c->Minv, c->s, f, F, out);
        for (int i = 0; i < c->Q; ++i) c->fpost[(size_t)i * c->N + n] = out[i];
        if (c->p.model == 2) pf_collide_g(c, n, f, F);
    }
    if (c->p.model == 2)
        for (long long n = 0; n < c->N; ++n)
            if (c->cls[n] != C_FLUID)
                for (int i = 0; i < c->Q; ++i) c->gpost[(size_t)i * c->N + n] = 0.0;
}

/* Eq. 4 as a pull; a population whose source is solid is the missing one of
 * Sec. III A: linear interpolated bounce-back with the wall fraction q, and the
 * difference to what left along the link goes to the rest population so that
 * the fluid mass is unchanged. */
void ora_phase_stream(ora_ctx* c) {
    const size_t N = (size_t)c->N;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_FLUID) {
            for (int i = 0; i < c->Q; ++i) c->f[i * N + n] = 0.0;
            if (c->p.model == 2)
                for (int i = 0; i < c->Q; ++i) c->g[i * N + n] = 0.0;
            continue;
        }
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        double dm = 0;
        c->f[n] = c->fpost[n];
        for (int i = 1; i < c->Q; ++i) {
            long long src = nbr(c, x, y, z, -c->e[i][0], -c->e[i][1], -c->e[i][2]);
            if (src >= 0 && c->cls[src] == C_FLUID) {
                c->f[i * N + n] = c->fpost[i * N + src];
                continue;
            }
            int j = c->opp[i]; /* direction from x toward the wall */
            double out_j = c->fpost[j * N + n];
            double val = out_j;
            if (c->p.bc_mode == 1) {
                double q = ora_link_q(c, x, y, z, j);
                if (q < 0.5) {
                    /* the partner behind x must hold the same phase: its population
                     * of direction j within a factor of two of x's own, else the
                     * link keeps the halfway value (an interpolation across the
                     * liquid-gas jump at a contact line would move up to the whole
                     * density difference into the rest population) */
                    long long xb = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
                    if (xb >= 0 && c->cls[xb] == C_FLUID) {
                        double fb = c->fpost[j * N + xb];
                        if (fb <= 2.0 * out_j && out_j <= 2.0 * fb)
                            val = 2.0 * q * out_j + (1.0 - 2.0 * q) * fb;
                    }
                } else {
                    val = out_j / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * c->fpost[i * N + n];
                }
            }
            c->f[i * N + n] = val;
            dm += out_j - val;
        }
        c->f[n] += dm;
        if (c->p.model == 2) {
            /* phase field: the order parameter streams with halfway bounce-back
             * at every wall (no flux of phi through the solid) */
            c->g[n] = c->gpost[n];
            for (int i = 1; i < c->Q; ++i) {
                long long src = nbr(c, x, y, z, -c->e[i][0], -c->e[i][1], -c->e[i][2]);
                c->g[i * N + n] = (src >= 0 && c->cls[src] == C_FLUID) ? c->gpost[i * N + src]
                                                                        : c->gpost[c->opp[i] * N + n];
            }
        }
    }
}

int ora_update_derived(ora_ctx* c) {
    ora_phase_density(c);
    ora_phase_fill(c);
    ora_phase_mu(c);
    ora_phase_force(c);
    return 0;
}

static int one_step(ora_ctx* c) {
    ora_update_derived(c);
    ora_phase_collide(c);
    ora_phase_stream(c);
    c->step++;
    return 0;
}

int ora_step(ora_ctx* c, long long nsteps) {
    for (long long t = 0; t < nsteps; ++t) one_step(c);
    return 0;
}

int ora_step_measured(ora_ctx* c, long long nsteps, int every, int solid, int n_sectors,
                      double rho_m, ora_angle* series, int cap, int* n_written) {
    int nw = 0;
    for (long long t = 0; t < nsteps; ++t) {
        if (every > 0 && c->step % every == 0 && nw < cap) {
            ora_measure(c, solid, n_sectors, rho_m, &series[nw]);
            nw++;
        }
        one_step(c);
    }
    if (n_written) *n_written = nw;
    return 0;
}

void* ora_field(ora_ctx* c, int which) {
    switch (which) {
        case 0: return c->f;
        case 1: return c->rho;
        case 2: return c->mu;
        case 3: return c->F;
        case 4: return c->cls;
        case 5: return c->fpost;
        case 6: return c->phi;
        case 7: return c->g;
        default: return NULL;
    }
}

void ora_velocity(ora_ctx* c, double* v) {
    ora_update_derived(c);
    const size_t N = (size_t)c->N;
    for (long long n = 0; n < c->N; ++n) {
        for (int d = 0; d < 3; ++d) v[d * N + n] = 0.0;
        if (c->cls[n] != C_FLUID) continue;
        double rho = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < c->Q; ++i) {
            double fi = c->f[i * N + n];
            rho += fi;
            for (int d = 0; d < 3; ++d) j[d] += fi * c->e[i][d];
        }
        for (int d = 0; d < 3; ++d) v[d * N + n] = j[d] / rho + c->F[d * N + n] / (2.0 * rho);
    }
}

double ora_mass(ora_ctx* c) {
    double m = 0;
    const size_t N = (size_t)c->N;
    for (long long n = 0; n < c->N; ++n)
        if (c->cls[n] == C_FLUID)
            for (int i = 0; i < c->Q; ++i) m += c->f[i * N + n];
    return m;
}

long long ora_get_step(ora_ctx* c) { return c->step; }

void ora_get_info(ora_ctx* c, double* out) {
    out[0] = c->Tc; out[1] = c->T; out[2] = c->alpha; out[3] = c->rho_g;
    out[4] = c->rho_l; out[5] = c->mu_sat; out[6] = c->p_sat; out[7] = c->wall_mu;
}

/* ------------------------------------------------------------------ */
/* contact-angle measurement (Sec. III B, Eq. 15, Fig. 1)             */
/* ------------------------------------------------------------------ */

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

typedef struct { double key_val; unsigned long long key; double p[3]; } cand_t;

/* measurement frame about the drop axis a: b1 = the lattice axis least aligned
 * with a (|a_k| compared on a 1/1024 grid, ties to the lower axis),
 * orthogonalised; b2 = a x b1 */
static void frame_of(int dim, const double a[3], double b1[3], double b2[3]) {
    int kb = 0;
    long best = 1L << 40;
    for (int d = 0; d < dim; ++d) {
        long qv = lround(fabs(a[d]) * 1024.0);
        if (qv < best) { best = qv; kb = d; }
    }
    for (int d = 0; d < 3; ++d) b1[d] = 0.0;
    b1[kb] = 1.0;
    double ab = dot3(a, b1);
    for (int d = 0; d < 3; ++d) b1[d] -= ab * a[d];
    double bn = sqrt(dot3(b1, b1));
    for (int d = 0; d < 3; ++d) b1[d] /= bn;
    b2[0] = a[1] * b1[2] - a[2] * b1[1];
    b2[1] = a[2] * b1[0] - a[0] * b1[2];
    b2[2] = a[0] * b1[1] - a[1] * b1[0];
}

/* sector of a position r relative to the substrate centre (2-D: the side of the axis) */
static int sector_of(int dim, const double r[3], const double b1[3], const double b2[3], int n_sectors) {
    if (dim == 2) return dot3(r, b1) >= 0.0 ? 0 : 1;
    double psi = atan2(dot3(r, b2), dot3(r, b1));
    int sec = (int)floor((psi + M_PI) / (2.0 * M_PI) * n_sectors);
    if (sec >= n_sectors) sec -= n_sectors;
    if (sec < 0) sec = 0;
    return sec;
}

int ora_measure(ora_ctx* c, int solid, int n_sectors, double rho_m, ora_angle* out) {
    memset(out, 0, sizeof *out);
    out->step = c->step;
    if (solid < 0 || solid >= c->nprim) return -1;
    const ora_prim* pr = &c->prim[solid];
    if (c->dim == 2) n_sectors = 2;
    if (n_sectors < 1 || n_sectors > 64) return -1;
    if (rho_m <= 0) rho_m = 0.5 * (c->rho_l + c->rho_g);
    out->n_sectors = n_sectors;
    ora_phase_density(c);
    const size_t N = (size_t)c->N;
    const double* mf = c->p.model == 2 ? c->phi : c->rho;  /* the field whose isolevel is the interface */

    /* liquid centroid from integer coordinate sums */
    long long cnt = 0, sx = 0, sy = 0, sz = 0;
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_FLUID || !(mf[n] >= rho_m)) continue;
        cnt++;
        sx += n % c->nx;
        sy += (n / c->nx) % c->ny;
        sz += n / ((long long)c->nx * c->ny);
    }
    double a[3] = {0, 0, 0};
    for (int s = 0; s < 64; ++s) out->sector_deg[s] = NAN;
    out->mean_deg = out->adv_deg = out->rec_deg = NAN;
    if (cnt == 0) { out->status = -6; return -6; }
    double G[3] = {(double)sx / cnt, (double)sy / cnt, c->dim == 3 ? (double)sz / cnt : 0.0};
    for (int d = 0; d < 3; ++d) a[d] = G[d] - pr->c[d];
    double an = sqrt(dot3(a, a));
    if (an == 0) { a[0] = 0; a[1] = c->dim == 2 ? 1 : 0; a[2] = c->dim == 2 ? 0 : 1; }
    else for (int d = 0; d < 3; ++d) a[d] /= an;
    for (int d = 0; d < 3; ++d) out->axis[d] = a[d];
    double b1[3], b2[3];
    frame_of(c->dim, a, b1, b2);

    /* all liquid-gas links between fluid nodes; crossing by Eq. 15 */
    cand_t best1[64], best2[64];
    for (int s = 0; s < 64; ++s) { best1[s].key = ~0ULL; best2[s].key = ~0ULL; }
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_FLUID || mf[n] >= rho_m) continue; /* gas end x_g */
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        for (int i = 1; i < c->Q; ++i) {
            long long m = nbr(c, x, y, z, c->e[i][0], c->e[i][1], c->e[i][2]);
            if (m < 0 || c->cls[m] != C_FLUID || !(mf[m] >= rho_m)) continue; /* liquid end x_l */
            double t = (rho_m - mf[n]) / (mf[m] - mf[n]);
            double p[3] = {x + t * c->e[i][0], y + t * c->e[i][1], z + t * c->e[i][2]};
            double r[3] = {p[0] - pr->c[0], p[1] - pr->c[1], p[2] - pr->c[2]};
            double dist = pr->concave ? pr->r - sqrt(dot3(r, r)) : sqrt(dot3(r, r)) - pr->r;
            if (!(dist >= 0.5 && dist < 2.5)) continue;
            int band = dist < 1.5 ? 1 : 2;
            int sec = sector_of(c->dim, r, b1, b2, n_sectors);
            float kv = (float)fabs(dist - band);
            uint32_t bits;
            memcpy(&bits, &kv, 4);
            unsigned long long key = ((unsigned long long)bits << 32) | (unsigned long long)(n * c->Q + i);
            cand_t* slot = band == 1 ? &best1[sec] : &best2[sec];
            if (key < slot->key) {
                slot->key = key;
                for (int d = 0; d < 3; ++d) slot->p[d] = p[d];
            }
        }
    }
    /* per sector: secant through P1, P2 in the meridional plane, contact point
     * on the substrate circle, angle against the tangent through the liquid */
    double sum = 0;
    int nv = 0;
    for (int s = 0; s < n_sectors; ++s) {
        out->key1[s] = best1[s].key;
        out->key2[s] = best2[s].key;
        for (int d = 0; d < 3; ++d) { out->p1[s][d] = best1[s].p[d]; out->p2[s][d] = best2[s].p[d]; out->contact[s][d] = NAN; }
        if (best1[s].key == ~0ULL || best2[s].key == ~0ULL) continue;
        double r1[3], r2[3];
        for (int d = 0; d < 3; ++d) { r1[d] = best1[s].p[d] - pr->c[d]; r2[d] = best2[s].p[d] - pr->c[d]; }
        double s1 = dot3(r1, a), s2 = dot3(r2, a);
        double q1[3], q2[3];
        for (int d = 0; d < 3; ++d) { q1[d] = r1[d] - s1 * a[d]; q2[d] = r2[d] - s2 * a[d]; }
        double w1 = sqrt(dot3(q1, q1)), w2 = sqrt(dot3(q2, q2));
        double Dw = w2 - w1, Ds = s2 - s1;
        double A = Dw * Dw + Ds * Ds;
        if (A == 0) continue;
        double B = w1 * Dw + s1 * Ds;
        double Cc = w1 * w1 + s1 * s1 - pr->r * pr->r;
        double disc = B * B - A * Cc;
        double lam;
        if (disc >= 0) {
            double lp = (-B + sqrt(disc)) / A, lm = (-B - sqrt(disc)) / A;
            if (lp <= 0) lam = lp;
            else if (lm <= 0) lam = lm;
            else lam = lm;
        } else {
            lam = -B / A;
        }
        double w0 = w1 + lam * Dw, s0 = s1 + lam * Ds;
        double r0 = sqrt(w0 * w0 + s0 * s0);
        /* outward radial unit vector; the tangent toward the axis follows from
         * it, and the substrate normal into the fluid is it (convex) or its
         * opposite (concave) */
        double ew = w0 / r0, es = s0 / r0;
        double tw = -es, ts = ew;
        double nw = pr->concave ? -ew : ew, ns = pr->concave ? -es : es;
        double vn = sqrt(A);
        double vw = Dw / vn, vs = Ds / vn;
        double th = atan2(vw * nw + vs * ns, vw * tw + vs * ts) * 180.0 / M_PI;
        double er[3];
        for (int d = 0; d < 3; ++d) er[d] = w1 > 0 ? q1[d] / w1 : 0.0;
        for (int d = 0; d < 3; ++d) out->contact[s][d] = pr->c[d] + s0 * a[d] + w0 * er[d];
        if (th < 0) continue;
        out->sector_deg[s] = th;
        sum += th;
        nv++;
    }
    out->n_valid = nv;
    if (nv == 0) { out->status = -6; return -6; }
    out->mean_deg = sum / nv;
    /* advancing side: the one the tangential part of g points to */
    double gt[3], ga = dot3(c->p.g, a);
    for (int d = 0; d < 3; ++d) gt[d] = c->p.g[d] - ga * a[d];
    if (dot3(gt, gt) > 0) {
        int sa, sr;
        if (c->dim == 2) {
            sa = dot3(gt, b1) >= 0.0 ? 0 : 1;
            sr = 1 - sa;
        } else {
            double psi = atan2(dot3(gt, b2), dot3(gt, b1));
            sa = (int)floor((psi + M_PI) / (2.0 * M_PI) * n_sectors);
            if (sa >= n_sectors) sa -= n_sectors;
            if (sa < 0) sa = 0;
            sr = (sa + n_sectors / 2) % n_sectors;
        }
        out->adv_deg = out->sector_deg[sa];
        out->rec_deg = out->sector_deg[sr];
    }
    out->status = 0;
    return 0;
}

/* Unbalanced Young force at the contact lines (Sec. IV E, Eq. 17) with the
 * equilibrium angle of the modified Cassie-Baxter relation (Eq. 18).
 *
 * Reading: the isodensity lines of the diffuse interface end on the substrate
 * over a footprint; in each sector the footprint is the set of fluid nodes
 * next to the substrate (a lattice neighbour inside the primitive) whose
 * density lies between rho_g + band_lo (rho_l - rho_g) and rho_g + band_hi
 * (rho_l - rho_g).  phi_d is the share of those nodes over the mu_w surface
 * (stripe index even, or a uniform primitive), 1 - phi_d over the mu_w2
 * surface.  The angle and the sectors are those of the measurement made on
 * the same density. */
static int surface_kind(const ora_prim* pr, const double r[3]) {
    if (pr->wet_mode == 0) return 0;
    double rn = sqrt(dot3(r, r));
    double cosp = rn > 0 ? dot3(r, pr->pole) / rn : 1.0;
    if (cosp > 1) cosp = 1;
    if (cosp < -1) cosp = -1;
    long long stripe = (long long)floor(pr->r * acos(cosp) / pr->width);
    return (int)(stripe % 2);
}

int ora_young_force(ora_ctx* c, int solid, int n_sectors, double rho_m, double band_lo, double band_hi,
                    double gamma, double theta1_deg, double theta2_deg, double roughness,
                    ora_angle* angle, ora_young* out) {
    memset(out, 0, sizeof *out);
    for (int s = 0; s < 64; ++s) out->phi_d[s] = out->theta_eq_deg[s] = out->force[s] = NAN;
    int st = ora_measure(c, solid, n_sectors, rho_m, angle);
    out->step = angle->step;
    out->n_sectors = angle->n_sectors;
    out->status = st;
    if (st != 0) return st;
    const ora_prim* pr = &c->prim[solid];
    double b1[3], b2[3];
    frame_of(c->dim, angle->axis, b1, b2);
    const double lo = c->rho_g + band_lo * (c->rho_l - c->rho_g), hi = c->rho_g + band_hi * (c->rho_l - c->rho_g);
    const double* mf = c->p.model == 2 ? c->phi : c->rho;
    for (long long n = 0; n < c->N; ++n) {
        if (c->cls[n] != C_FLUID || !(mf[n] >= lo && mf[n] <= hi)) continue;
        int x = (int)(n % c->nx), y = (int)((n / c->nx) % c->ny), z = (int)(n / ((long long)c->nx * c->ny));
        int touches = 0;
        for (int i = 1; i < c->Q && !touches; ++i) {
            int X = x + c->e[i][0], Y = y + c->e[i][1], Z = z + c->e[i][2];
            X = (X + c->nx) % c->nx;
            Y = (Y + c->ny) % c->ny;
            Z = (Z + c->nz) % c->nz;
            touches = inside_prim(pr, X, Y, Z);
        }
        if (!touches) continue;
        double r[3] = {x - pr->c[0], y - pr->c[1], c->dim == 3 ? z - pr->c[2] : 0.0};
        out->count[sector_of(c->dim, r, b1, b2, angle->n_sectors)][surface_kind(pr, r)]++;
    }
    const double c1 = cos(theta1_deg * M_PI / 180.0), c2 = cos(theta2_deg * M_PI / 180.0);
    for (int s = 0; s < angle->n_sectors; ++s) {
        int tot = out->count[s][0] + out->count[s][1];
        if (tot == 0) continue;
        double phi = (double)out->count[s][0] / tot;
        double ce = roughness * phi * c1 + (1.0 - phi) * c2;
        if (ce > 1) ce = 1;
        if (ce < -1) ce = -1;
        out->phi_d[s] = phi;
        out->theta_eq_deg[s] = acos(ce) * 180.0 / M_PI;
        if (!isnan(angle->sector_deg[s]))
            out->force[s] = gamma * (cos(angle->sector_deg[s] * M_PI / 180.0) - ce);
    }
    return 0;
}
