/*
 * lbm_oracle.h -- plain FP64 CPU reference of the multiphase lattice Boltzmann
 * step with a curved wetting solid and the two-point contact-angle measurement
 * (Liu, Yao, Li, Wen, "Contact angle measurement on curved wetting surface in
 * multiphase lattice Boltzmann method", arXiv:2202.06516).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness oracle for the
 * GPU library.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never calls it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Everything is double precision, no FMA contraction (-ffp-contract=off),
 * one plain loop per step of the method, in the order the paper gives.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int dim;            /* 2 (D2Q9) or 3 (D3Q19) */
    int n[3];           /* lattice size; n[2] = 1 in 2-D */
    int wall[3];        /* 1: two solid layers at both ends of this axis; 0: periodic */
    int bgk;            /* 1: single relaxation time 1/tau on every moment */
    int bc_mode;        /* 0: halfway bounce-back; 1: linear interpolated bounce-back + mass correction */
    double tau, s_e, s_eps, s_q, s_pi, s_m;   /* MRT rates (s_v = 1/tau) */
    double Tr, a, b, R, omega;                /* Peng-Robinson parameters */
    double k, kappa;                          /* mesh-space scaling k and kappa-hat */
    double g[3];                              /* body acceleration (lattice units) */
    long long g_start;                        /* first step at which g acts */
    double rho_l, rho_g;                      /* <= 0: Maxwell coexistence */
    double wall_mu;                           /* outer-wall chemical potential; NaN: k^2 mu_sat */
    int model;          /* 0: chemical potential (Sec. II B); 1: pseudopotential (Shan-Chen); 2: phase field */
    double sc_G;        /* pseudopotential interaction strength (model 1) */
    /* phase-field model (model 2): order parameter phi in [-1, 1] carried by a
     * second population set g, free energy A/4 (phi^2 - 1)^2 + kappa/2 |grad phi|^2,
     * mobility M = gamma (tau_g - 1/2), fluid density rho0 in both phases */
    double pf_A, pf_kappa, pf_gamma, pf_tau, pf_rho0;
} ora_params;

typedef struct {
    long long step;
    int status;                 /* 0 ok, -6 no contact line */
    int n_sectors, n_valid;
    double mean_deg, adv_deg, rec_deg;
    double axis[3];             /* unit vector from substrate centre to liquid centroid */
    double sector_deg[64];
    double contact[64][3];      /* three-phase contact point per sector (lattice coords) */
    double p1[64][3], p2[64][3];/* selected interface points near 1 and 2 lu */
    unsigned long long key1[64], key2[64];  /* selection keys (float32 bits of |d-k| << 32 | link id) */
} ora_angle;

typedef struct ora_ctx ora_ctx;

/* thermodynamics (Eq. 10, Eq. 11 without the gradient term, Maxwell) */
double ora_pr_alpha(double Tr, double omega);
double ora_pr_p0(double rho, double T, double a, double b, double R, double alpha);
double ora_pr_mu(double rho, double T, double a, double b, double R, double alpha);
int    ora_pr_critical(double a, double b, double R, double* Tc, double* rhoc, double* pc);
int    ora_maxwell(double T, double a, double b, double R, double alpha,
                   double* rho_g, double* rho_l, double* p_sat, double* mu_sat);

/* lattice tables and the MRT transform, exposed for the pins */
int  ora_lattice(int dim, int* Q, int* e /*[Q*3]*/, double* w /*[Q]*/);
void ora_mrt_matrix(int dim, double* M /*[Q*Q], row = moment*/);
void ora_feq(int dim, double rho, const double u[3], double* feq /*[Q]*/);
/* one collision of a single node: f[Q] in, post-collision out, force F (3) */
void ora_collide_node(const ora_params* p, const double* f, const double F[3], double* fout);

ora_ctx* ora_create(const ora_params* p);
void     ora_destroy(ora_ctx* c);
/* convex sphere (circle in 2-D); wet_mode 0 uniform mu_w, 1 latitude stripes */
int  ora_add_sphere(ora_ctx* c, const double centre[3], double radius, int wet_mode,
                    double mu_w, double mu_w2, double stripe_width, const double pole[3]);
/* concave cavity: solid wherever |x - centre| >= radius; same wetting modes */
int  ora_add_cavity(ora_ctx* c, const double centre[3], double radius, int wet_mode,
                    double mu_w, double mu_w2, double stripe_width, const double pole[3]);
int  ora_set_muw_map(ora_ctx* c, const double* map /*[N] or NULL*/);
int  ora_build(ora_ctx* c);                       /* classify nodes; call after adding solids */
int  ora_init_drops(ora_ctx* c, const double* centres /*[n*3]*/, const double* radii, int n, double W);
int  ora_set_rho(ora_ctx* c, const double* rho);  /* state = f_eq(rho, 0) at fluid nodes */
int  ora_step(ora_ctx* c, long long nsteps);
int  ora_step_measured(ora_ctx* c, long long nsteps, int every, int solid, int n_sectors,
                       double rho_m, ora_angle* series, int cap, int* n_written);
int  ora_measure(ora_ctx* c, int solid, int n_sectors, double rho_m, ora_angle* out);

/* Unbalanced Young force per sector (Sec. IV E, Eq. 17) with the equilibrium
 * angle of Eq. 18, on a measurement made here on the same density (written to
 * *angle).  The footprint of a sector: fluid nodes with a lattice neighbour
 * inside the primitive and a density in [rho_g + band_lo (rho_l - rho_g),
 * rho_g + band_hi (rho_l - rho_g)]; count[s][0] on the mu_w surface (even
 * stripe or uniform), count[s][1] on mu_w2; phi_d = count[s][0] / total. */
typedef struct {
    long long step;
    int status, n_sectors;
    int count[64][2];
    double phi_d[64];           /* NaN without footprint */
    double theta_eq_deg[64];    /* Eq. 18 */
    double force[64];           /* Eq. 17; NaN where the sector has no angle */
} ora_young;
int  ora_young_force(ora_ctx* c, int solid, int n_sectors, double rho_m, double band_lo, double band_hi,
                     double gamma, double theta1_deg, double theta2_deg, double roughness,
                     ora_angle* angle, ora_young* out);

/* fields: 0 f (state, [Q][N]), 1 rho, 2 mu, 3 force ([3][N]), 4 class (uchar), 5 fpost;
 * phase-field model: 6 phi, 7 g (state of the order parameter, [Q][N]) */
void* ora_field(ora_ctx* c, int which);
int   ora_update_derived(ora_ctx* c);   /* rho, fill, mu, force of the current state */
void  ora_velocity(ora_ctx* c, double* v /*[3][N]*/);
double ora_mass(ora_ctx* c);
long long ora_get_step(ora_ctx* c);
void ora_get_info(ora_ctx* c, double* out /*[8]: Tc, T, alpha, rho_g, rho_l, mu_sat, p_sat, wall_mu*/);

/* individual step phases (used by the pins) */
void ora_phase_density(ora_ctx* c);
void ora_phase_fill(ora_ctx* c);
void ora_phase_mu(ora_ctx* c);
void ora_phase_force(ora_ctx* c);
void ora_phase_collide(ora_ctx* c);
void ora_phase_stream(ora_ctx* c);

/* q of the link from fluid node x along e_dir to a solid node; -1 if not cut */
double ora_link_q(ora_ctx* c, int x, int y, int z, int dir);

#ifdef __cplusplus
}
#endif
#endif
