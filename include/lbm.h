/*
 * lbm.h -- C ABI of the MI355X (gfx950) multiphase lattice Boltzmann library.
 *
 * The library advances the multiphase lattice Boltzmann equation of
 * Liu, Yao, Li & Wen, "Contact angle measurement on curved wetting surface in
 * multiphase lattice Boltzmann method" (arXiv:2202.06516) on one GPU, and
 * measures the contact angle of a drop on a curved wetting solid inside the
 * time step.  Every entry point takes plain pointers and sizes; no C++ or
 * framework types cross this boundary.
 *
 * Method (paper sections and equations):
 *   - MRT lattice Boltzmann equation, Eq. 1, rates S of Sec. II A; the BGK
 *     collision of Eq. 3 is available as the case of equal rates;
 *   - second-order equilibrium, Eq. 2; streaming, Eq. 4;
 *   - chemical potential of the Peng-Robinson fluid, Eq. 10-12, gradients by
 *     fourth-order central differences (Sec. II B);
 *   - non-ideal force F = -rho grad(mu) + cs^2 grad(rho), Eq. 7, applied by
 *     the exact-difference method, Eq. 13; optional body force rho g (Sec. IV);
 *   - wetting: a prescribed chemical potential on two solid layers, whose
 *     densities follow Eq. 14 (Sec. III A);
 *   - streaming at the curved wall: halfway bounce-back, or linear
 *     interpolated bounce-back with an exact mass correction (Sec. III A),
 *     whose q < 1/2 branch interpolates only with a partner population within
 *     a factor of two of the node's own (else halfway: no interpolation across
 *     the liquid-gas jump at a contact line);
 *   - contact angle: isodensity crossings on liquid-gas links (Eq. 15), the
 *     crossings nearest 1 and 2 lattice units from the substrate, their secant
 *     meets the substrate at the contact point, angle to the substrate tangent
 *     through the liquid (Sec. III B, Fig. 1).
 *
 * Conventions shared by all entry points:
 *   - every call returns lbm_status; 0 is success; a call never aborts;
 *   - on failure, lbm_last_error() describes the error; the string is owned
 *     by the context and stays valid until the next call on that context;
 *   - the context owns every buffer it allocates; caller buffers stay the
 *     caller's and are only read or written during the call (or, for device
 *     pointers, by work the call enqueues on the context's stream);
 *   - arrays are x-fastest: index = (z * ny + y) * nx + x; populations are
 *     structure-of-arrays [Q][nz][ny][nx];
 *   - direction order D2Q9:  0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1)
 *                            5 (1,1) 6 (-1,1) 7 (-1,-1) 8 (1,-1);
 *     D3Q19: 0 (0,0,0) 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1)
 *            6 (0,0,-1) 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0)
 *            11 (1,0,1) 12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1)
 *            16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1);
 *   - the state of a context is the pre-collision populations S_t after
 *     streaming; the step counter t counts completed steps;
 *   - work is enqueued on the context's stream (the one in lbm_config, else
 *     one the context creates); calls that return host data synchronise it;
 *   - a context is not thread-safe: one thread at a time per context.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,             /* invalid argument or configuration */
    LBM_E_NOMEM = -2,           /* host or device allocation failed */
    LBM_E_DEVICE = -3,          /* a HIP call failed */
    LBM_E_STATE = -4,           /* call out of order (e.g. step before init) */
    LBM_E_NONFINITE = -5,       /* a density became non-finite, <= 0, or >= 1/b */
    LBM_E_NO_CONTACT_LINE = -6, /* no sector holds both selected crossings */
    LBM_E_UNSUPPORTED = -7      /* valid request the library does not implement */
} lbm_status;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
enum { LBM_F32 = 0, LBM_F64 = 1, LBM_F32_MIXED = 2 };
enum { LBM_PERIODIC = 0, LBM_WALL = 1 };
enum { LBM_MRT = 0, LBM_BGK = 1 };
enum { LBM_BC_HALFWAY = 0, LBM_BC_BOUZIDI_MC = 1 };
/* Force model of the step.  The paper's own is the chemical-potential model
 * (Sec. II B).  Sec. V states that the measurement serves other multiphase
 * models as well, such as the pseudopotential ones.  LBM_MODEL_PSEUDOPOTENTIAL
 * is the Shan-Chen model: psi(rho) = 1 - exp(-rho) and
 * F = -G psi(x) sum_i w_i psi(x + e_i) e_i (+ rho g), with the same collision,
 * streaming and measurement.  Wetting uses a wall density: every mu_w (of a
 * primitive, a stripe, the map or the outer walls) is read as a density rho_w,
 * and both solid layers carry psi(rho_w).  Its coexistence densities depend on
 * the forcing scheme, so rho_l and rho_g must be given. */
/* LBM_MODEL_PHASE_FIELD is a phase-field model, the other family Sec. V names:
 * an order parameter phi (liquid +1, gas -1) carried by a second population
 * set g, free energy A/4 (phi^2 - 1)^2 + kappa/2 |grad phi|^2 (pf_A, pf_kappa),
 * mu = A (phi^3 - phi) - kappa lap(phi), capillary force mu grad(phi) (+ rho g)
 * on the fluid populations, g relaxed with 1/pf_tau toward the equilibrium of
 * the Cahn-Hilliard equation with mobility pf_gamma (pf_tau - 1/2), g streamed
 * with halfway bounce-back at every wall.  Wetting uses a wall order parameter:
 * every mu_w is read as phi_w, held by both solid layers (NaN wall_mu: 0).  The
 * measurement reads phi at the isolevel 0 (rho_l = 1 and rho_g = -1 stand for
 * the two bulk values); lbm_init_drops profiles phi by Eq. 16 with the fluid
 * density pf_rho0 everywhere.  On one lattice it runs the split step (the
 * one-pass step is not built for it); the batched solver runs it on every
 * case, the in-step and on-demand Young force included. */
enum { LBM_MODEL_CHEMICAL_POTENTIAL = 0, LBM_MODEL_PSEUDOPOTENTIAL = 1, LBM_MODEL_PHASE_FIELD = 2 };
enum { LBM_STEP_AUTO = 0, LBM_STEP_SPLIT = 1 };

#define LBM_MAX_SECTORS 64
#define LBM_MAX_SOLIDS 16

/* Configuration of one lattice.  lbm_config_default() fills every field. */
typedef struct {
    int lattice;          /* LBM_D2Q9 or LBM_D3Q19 */
    int precision;        /* LBM_F32 / LBM_F64: storage and arithmetic of the step;
                             LBM_F32_MIXED: FP32 storage, FP64 arithmetic */
    int n[3];             /* lattice size; n[2] must be 1 for D2Q9 */
    int axis_bc[3];       /* per axis LBM_PERIODIC, or LBM_WALL = two solid layers at both ends */
    int collision;        /* LBM_MRT (Eq. 1) or LBM_BGK (Eq. 3) */
    int bc_mode;          /* LBM_BC_HALFWAY or LBM_BC_BOUZIDI_MC at solid walls */
    double tau;           /* relaxation time; s_v = 1/tau (Sec. II A) */
    double s_e, s_eps, s_q;  /* MRT rates of Sec. II A (defaults 1.64, 1.54, 1.9) */
    double s_pi, s_m;     /* D3Q19 rates of the 4th-order (pi) and 3rd-order (m) moments */
    double Tr;            /* reduced temperature T/Tc (Sec. II B) */
    double pr_a, pr_b, pr_R, pr_omega;  /* Peng-Robinson a, b, R, acentric factor (Eq. 10) */
    double k;             /* mesh-space scaling of Eq. 12 */
    double kappa;         /* gradient coefficient kappa-hat of Eq. 12 */
    double g[3];          /* body acceleration in lattice units; force rho g on fluid nodes */
    int64_t g_start_step; /* first step t at which g acts */
    double rho_l, rho_g;  /* coexistence densities; <= 0 selects the Maxwell construction */
    double wall_mu;       /* chemical potential of outer walls; NaN selects k^2 mu_sat
                             (pseudopotential model: wall density, NaN selects (rho_l + rho_g) / 2) */
    void* stream;         /* hipStream_t to enqueue on, or NULL for a context-owned stream */
    int model;            /* LBM_MODEL_CHEMICAL_POTENTIAL (default), LBM_MODEL_PSEUDOPOTENTIAL or
                             LBM_MODEL_PHASE_FIELD; the pseudopotential model needs rho_l > rho_g > 0 and
                             ignores Tr, pr_*, k, kappa (the batched solver takes any of the three for all its
                             cases); the phase-field model ignores Tr, pr_*, k, kappa, rho_l, rho_g */
    double sc_G;          /* pseudopotential interaction strength G (default -6) */
    int step_kernel;      /* LBM_STEP_AUTO (default): D3Q19 lattices (either wall scheme; not the phase-field
                             model) with nx a multiple of 64 (at most 1024), ny a multiple of 4 and nz even
                             take one pass over the populations per step (the
                             collision also sums the next step's density); LBM_STEP_SPLIT: a density pass,
                             then the collision.  Both compute the same step; the density sums differ in
                             order, so the fields agree to rounding. */
    double pf_A, pf_kappa;  /* phase-field model: free-energy coefficients (default 0.01, 0.02) */
    double pf_gamma;        /* mobility coefficient: M = pf_gamma (pf_tau - 1/2) (default 1) */
    double pf_tau;          /* relaxation time of the order-parameter populations, > 1/2 (default 1) */
    double pf_rho0;         /* fluid density of the initial state (default 1) */
} lbm_config;

/* Fill *cfg with the library defaults for the given lattice. */
void lbm_config_default(lbm_config* cfg, int lattice);

/* Substrate shapes of Fig. 2: a convex circle (2-D) or sphere (3-D), and the
 * concave cavity, whose inside is fluid and outside solid. */
enum { LBM_SOLID_SPHERE = 0, LBM_SOLID_CAVITY = 1 };
enum { LBM_WET_UNIFORM = 0, LBM_WET_STRIPES = 1 };

/* A solid primitive.  LBM_SOLID_SPHERE: a node is solid iff
 * |x - center| <= radius; LBM_SOLID_CAVITY: iff |x - center| >= radius.  The
 * contact-angle measurement takes the substrate normal into the fluid (outward
 * for a sphere, toward the centre for a cavity); everything else treats both
 * kinds alike.  Any other kind is rejected with LBM_E_ARG.
 * Wettability (Sec. III A): mu_w on its solid nodes, or with LBM_WET_STRIPES
 * alternating mu_w / mu_w2 in latitude stripes of arc length stripe_width,
 * stripe = floor(radius * polar_angle / stripe_width), polar angle from pole. */
typedef struct {
    int kind;            /* LBM_SOLID_SPHERE or LBM_SOLID_CAVITY */
    int wet_mode;        /* LBM_WET_UNIFORM or LBM_WET_STRIPES */
    double center[3];
    double radius;
    double mu_w, mu_w2;
    double stripe_width;
    double pole[3];      /* stripe pole direction; zero vector selects +y (2-D) or +z (3-D) */
} lbm_solid;

/* A drop for the initial density field of Eq. 16. */
typedef struct {
    double center[3];
    double radius;
} lbm_drop;

/* Which solid and how many azimuthal sectors the measurement uses. */
typedef struct {
    int solid_index;     /* index into the array given to lbm_set_solid */
    int n_sectors;       /* 3-D: 1..64 azimuthal sectors about the drop axis; ignored in 2-D (2 sides) */
    double rho_m;        /* isodensity level; <= 0 selects (rho_l + rho_g) / 2 */
} lbm_measure_opts;

/* One contact-angle measurement.  Angles in degrees; NaN where invalid.
 *
 * 3-D sectors: a is the axis below; b1 is the lattice axis least aligned
 * with a (|a_k| compared after rounding to multiples of 1/1024, ties to the
 * lower axis) with its a-component removed and normalised, and b2 = a x b1.
 * A point r (relative to the substrate centre) has azimuth
 * psi = atan2(r.b2, r.b1) in [-pi, pi], and sector s holds
 * -pi + 2 pi s / n_sectors <= psi < -pi + 2 pi (s + 1) / n_sectors.
 * adv_deg is the sector holding the azimuth of g's part normal to a, rec_deg
 * the sector n_sectors / 2 further on (2-D: side 0 holds r.b1 >= 0). */
typedef struct {
    int64_t step;        /* t of the density field measured */
    int32_t status;      /* LBM_OK or LBM_E_NO_CONTACT_LINE */
    int32_t n_sectors;
    int32_t n_valid;
    int32_t pad_;
    double mean_deg;     /* mean over valid sectors */
    double adv_deg;      /* sector the tangential part of g points to (NaN if g has none) */
    double rec_deg;      /* the opposite sector */
    double axis[3];      /* unit vector from the substrate centre to the liquid centroid */
    double sector_deg[LBM_MAX_SECTORS];
    double contact[LBM_MAX_SECTORS][3];  /* contact point per sector, lattice coordinates */
} lbm_angle;

typedef struct {
    double Tc, T, alpha;          /* critical temperature, temperature, alpha(T) */
    double rho_g, rho_l;          /* coexistence densities in use */
    double mu_sat, p_sat;         /* psi'(rho) and p0 at coexistence (C = 0 in Eq. 9) */
    double wall_mu;               /* outer-wall chemical potential in use */
    double rho_m;                 /* default isodensity level */
    int32_t Q;
    int32_t precision;
    int64_t N;                    /* nodes */
    int64_t step;                 /* completed steps */
    int64_t n_fluid, n_layer1, n_layer2, n_boundary;
} lbm_info;

enum {
    LBM_FIELD_RHO = 0,   /* [N] density of S_t (fluid), Eq. 14 fill on the two solid layers */
    LBM_FIELD_F = 1,     /* [Q][N] populations S_t */
    LBM_FIELD_VEL = 2,   /* [3][N] v = u + F / (2 rho), Sec. II B */
    LBM_FIELD_MU = 3,    /* [N] chemical potential of Eq. 12; wall value on the solid layers
                            (pseudopotential model: psi, and psi(rho_w) on the layers) */
    LBM_FIELD_CLASS = 4, /* [N] uint8: 0 fluid, 1 first solid layer, 2 second, 3 deeper solid */
    LBM_FIELD_MASS = 5,  /* one double: sum of S_t over fluid nodes */
    LBM_FIELD_PHI = 6,   /* phase-field model: [N] order parameter sum_i g_i (fluid), phi_w on the solid layers */
    LBM_FIELD_G = 7      /* phase-field model: [Q][N] order-parameter populations (state, as F) */
};

typedef struct lbm_ctx lbm_ctx;

/* Create a context: validates cfg, computes the coexistence densities,
 * allocates the lattice on the current HIP device.  Errors: LBM_E_ARG,
 * LBM_E_NOMEM, LBM_E_DEVICE.  *out is NULL on failure. */
lbm_status lbm_create(const lbm_config* cfg, lbm_ctx** out);

/* Free a context and everything it owns.  NULL is accepted. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Set the solids (Sec. III A): classify nodes into fluid / first layer /
 * second layer / deeper solid, compute the wall fraction q of every cut link
 * and the wall chemical potential of every solid-layer node.  mu_w_map, if
 * not NULL, is a host array of N doubles that overrides the primitives'
 * wettability node by node.  Invalidates the state: call lbm_init_drops or
 * lbm_write next.  Errors: LBM_E_ARG (n > LBM_MAX_SOLIDS, bad primitive). */
lbm_status lbm_set_solid(lbm_ctx* ctx, const lbm_solid* prims, int n, const double* mu_w_map);

/* Initial density by Eq. 16 (tanh profile of width W around each drop;
 * where drops overlap the larger density wins); state = f_eq(rho, 0) on fluid
 * nodes; t = 0. */
lbm_status lbm_init_drops(lbm_ctx* ctx, const lbm_drop* drops, int n, double W);

/* Advance nsteps steps.  If measure_every > 0, the contact angle of
 * lbm_set_measure's options is measured inside the step, on the density of
 * every step t with t % measure_every == 0.  If series is not NULL, up to cap
 * measurements are copied to it and *n_written is set (this synchronises);
 * otherwise the call only enqueues work.  Errors: LBM_E_STATE before any
 * initial state, LBM_E_NONFINITE if a density went bad (checked when the
 * call synchronises). */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps, int measure_every,
                    lbm_angle* series, int cap, int* n_written);

/* Measurement options used by lbm_step's in-step measurement. */
lbm_status lbm_set_measure(lbm_ctx* ctx, const lbm_measure_opts* opts);

/* Measure the contact angle of the current state (synchronises).
 * Returns LBM_E_NO_CONTACT_LINE (out->mean_deg = NaN) if no sector is valid. */
lbm_status lbm_measure_angle(lbm_ctx* ctx, const lbm_measure_opts* opts, lbm_angle* out);

/* Copy a field of the current state to dst (host memory unless
 * dst_on_device).  bytes must equal the field size: N * elem for RHO, MU and PHI,
 * Q * N * elem for F and G, 3 * N * elem for VEL (elem = 4 for LBM_F32 and
 * LBM_F32_MIXED, 8 for LBM_F64), N for CLASS, 8 for MASS (always double).  PHI
 * and G exist in the phase-field model only (LBM_E_ARG otherwise).  Synchronises. */
lbm_status lbm_read(lbm_ctx* ctx, int field, void* dst, size_t bytes, int dst_on_device);

/* Replace the state.  LBM_FIELD_F: populations S_t (checkpoint restore);
 * LBM_FIELD_RHO: density, state = f_eq(rho, 0) on fluid nodes.  Phase-field
 * model: LBM_FIELD_PHI: order parameter on fluid nodes, state = f_eq(pf_rho0, 0)
 * and g at rest (g_0 = phi); LBM_FIELD_F and LBM_FIELD_G replace one
 * population set each (a checkpoint restore writes both); LBM_FIELD_RHO is
 * refused.  Sizes as for lbm_read.  Does not change t. */
lbm_status lbm_write(lbm_ctx* ctx, int field, const void* src, size_t bytes, int src_on_device);

/* Wait for enqueued work; LBM_E_NONFINITE if a density went bad. */
lbm_status lbm_sync(lbm_ctx* ctx);

lbm_status lbm_get_info(lbm_ctx* ctx, lbm_info* info);

/* Unbalanced Young force at the contact lines (Sec. IV E, Eq. 17) with the
 * equilibrium angle of the modified Cassie-Baxter relation (Eq. 18).  The
 * footprint of a sector is the set of fluid nodes with a lattice neighbour
 * inside the measured substrate whose density lies between rho_g + band_lo
 * (rho_l - rho_g) and rho_g + band_hi (rho_l - rho_g): where the diffuse
 * interface's isodensity lines end on the substrate.  phi_d is the share of
 * the footprint over the substrate's mu_w surface (a uniform substrate, or its
 * even latitude stripes), 1 - phi_d over its mu_w2 stripes. */
typedef struct {
    double gamma;        /* liquid-gas surface tension, lattice units */
    double theta1_deg;   /* equilibrium angle of the mu_w surface */
    double theta2_deg;   /* equilibrium angle of the mu_w2 stripes (unused on a uniform substrate) */
    double roughness;    /* r of Eq. 18 (1: smooth); > 0 */
    double band_lo, band_hi;  /* footprint band in (0, 1); 0 and 0 select 0.1 and 0.9 */
} lbm_young_opts;

typedef struct {
    int64_t step;        /* t of the density used */
    int32_t status;      /* LBM_OK or LBM_E_NO_CONTACT_LINE */
    int32_t n_sectors;
    int32_t count[LBM_MAX_SECTORS][2];     /* footprint nodes on the mu_w / mu_w2 surface */
    double phi_d[LBM_MAX_SECTORS];         /* count[s][0] / (count[s][0] + count[s][1]); NaN without footprint */
    double theta_eq_deg[LBM_MAX_SECTORS];  /* Eq. 18; NaN without footprint */
    double force[LBM_MAX_SECTORS];         /* Eq. 17: gamma (cos theta_s - cos theta_eq); NaN where either is */
} lbm_young;

/* Measure now (as lbm_measure_angle with the options of lbm_set_measure; the
 * angle is written to *angle) and compute, on the same density, the footprint
 * counts, phi_d, theta_eq and the unbalanced Young force per sector into *out.
 * Synchronises.  Errors: LBM_E_ARG (null pointer, gamma not finite,
 * roughness <= 0, band outside 0 < band_lo < band_hi < 1), LBM_E_STATE,
 * LBM_E_NO_CONTACT_LINE (out->status set, every value NaN), LBM_E_DEVICE. */
lbm_status lbm_young_force(lbm_ctx* ctx, const lbm_young_opts* opts, lbm_angle* angle, lbm_young* out);

/* Take the unbalanced Young force (Eq. 17-18) at every in-step measurement of
 * the following lbm_step calls, with these options (NULL turns it off).  Each
 * measurement then counts the footprint in the same frame and sectors, and
 * applies Eq. 18 and Eq. 17 on the device, in FP64, to the angles it has just
 * measured.  lbm_young_series returns those records.  Synchronises.  Errors:
 * LBM_E_ARG (options as for lbm_young_force), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_set_young(lbm_ctx* ctx, const lbm_young_opts* opts);

/* The Young-force records of the last lbm_step call that wrote an angle
 * series: out[i] belongs to series[i] of that call (min(cap, that count)
 * records, *n_written).  Synchronises.  Errors: LBM_E_ARG, LBM_E_STATE (off). */
lbm_status lbm_young_series(lbm_ctx* ctx, lbm_young* out, int cap, int* n_written);

/* Step the lattice nsteps times (no measurement) with a HIP event pair
 * around every kernel launch, and report the mean duration in milliseconds of
 * each kernel kind: names[i] (static strings) and ms[i] for i < *n_kinds
 * (cap entries at most).  Synchronises. */
lbm_status lbm_profile_step(lbm_ctx* ctx, int64_t nsteps, const char** names, double* ms,
                            int cap, int* n_kinds);

/* The message of the last error on ctx; with ctx NULL, that of the last call
 * without a context (lbm_measure_field) on this thread. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Contact angle of a density field the caller holds, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It is lbm_measure_angle without a context:
 * the same kernels (liquid centroid, crossing search, finalising block) run on
 * rho and cls as given, and the one record is written to out in device memory.
 * The call allocates nothing and does not synchronise: it enqueues five small
 * launches on stream (NULL: the null stream) and returns.
 *   rho  device, [N] of the element type of precision (FP32 for LBM_F32 and
 *        LBM_F32_MIXED, FP64 for LBM_F64), x fastest; only fluid nodes are read
 *        as densities;
 *   cls  device, [N] uint8 classes as lbm_read(LBM_FIELD_CLASS) writes them
 *        (0 fluid; bits 0-1 are read);
 *   solid  the substrate measured (host);  n_sectors  3-D: 1..64 (2-D: 2 sides);
 *   rho_m  the isodensity level, > 0;  g  body acceleration for the advancing /
 *        receding sectors (host, nullable = none);
 *   out  device, one lbm_angle; out->step is 0.
 * Scratch: the reduction slots live in a static device array of 2 KiB that
 * each GPU holds for the life of the process; the call clears them before use.
 * Calls on one GPU share it, so calls whose work overlaps in time on one GPU
 * (different streams without ordering) race: order them.  Limits, rejected
 * with LBM_E_ARG before anything is enqueued: n_sectors above 64 (the slots
 * hold 64 sectors), N * Q >= 2^32 (32-bit link ids), n outside 5..2^20 per
 * axis, n[2] != 1 for D2Q9, rho_m not positive, a bad primitive, a null
 * pointer.  LBM_E_DEVICE if no device is current or a launch fails.  The
 * message is lbm_last_error(NULL). */
lbm_status lbm_measure_field(int lattice, int precision, const int n[3], const void* rho, const uint8_t* cls,
                             const lbm_solid* solid, int n_sectors, double rho_m, const double g[3], lbm_angle* out,
                             void* stream);

/* ------------------------------------------------------------------------
 * Batched solver: many independent lattices advanced together.
 *
 * Each case has its own lattice size, one solid primitive (wettability as in
 * lbm_solid) and one drop (Eq. 16, W = 10); all cases share the fluid, the
 * collision and the boundary settings of the base configuration.  Cases are
 * packed in one allocation; every phase of a step is one persistent launch
 * over a work list of (case, tile) items, and step loops are captured in a
 * hipGraph.  A case advanced in a batch equals the same case advanced alone
 * with lbm_step, bit for bit.  The contact angle of every case is measured in
 * the step (2 sides in 2-D, 16 sectors in 3-D).
 *
 * Models: the chemical-potential model, the pseudopotential model and the
 * phase-field model (LBM_MODEL_PHASE_FIELD, as for one lattice: mu_w of each
 * solid and wall_mu are wall order parameters, the drop is the order
 * parameter of Eq. 16 with W = 2 sqrt(2 pf_kappa / pf_A), the flat-interface
 * width, and the measurement reads phi at the isolevel 0).
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

typedef struct {
    int n[3];            /* lattice size of the case; n[2] = 1 for D2Q9 */
    lbm_solid solid;
    lbm_drop drop;
} lbm_case;

typedef struct {
    int autotune;        /* 1: time candidate tile widths / workgroups per CU and keep the fastest */
    int tile_w;          /* 64, 128 or 256 nodes per tile row (tile = 256 nodes) when not tuning */
    int blocks_per_cu;   /* persistent workgroups per compute unit when not tuning (1..32) */
    const char* cache_path; /* JSON file of tuned choices keyed by the case table, or NULL */
} lbm_batch_opts;

typedef struct {
    int64_t total_nodes, fluid_nodes;  /* lattice nodes of all cases (each row is padded to a multiple of
                                          64 nodes in device memory), fluid nodes among them */
    int32_t ncases, tile_w, blocks_per_cu, n_items;
    double tune_ms_per_step;  /* time per step of the chosen launch shape (0 if not tuned) */
    int64_t step;
    double rho_g, rho_l;
} lbm_batch_info;

/* Create a batch (host geometry of every case, packed device arrays, initial
 * state of Eq. 16), optionally autotune.  Errors: LBM_E_ARG (bad case, or the
 * packed lattice exceeds 2^32 / Q nodes), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_batch_create(const lbm_config* base, const lbm_case* cases, int ncases, const lbm_batch_opts* opts,
                            lbm_batch** out);
lbm_status lbm_batch_destroy(lbm_batch* b);
/* Advance every case nsteps steps; measure every measure_every steps (0: never).  Enqueues only. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps, int measure_every);
/* Wait; LBM_E_NONFINITE if a density of any case went bad. */
lbm_status lbm_batch_sync(lbm_batch* b);
/* Latest in-step measurement of cases 0..n-1 (synchronises). */
lbm_status lbm_batch_angles(lbm_batch* b, lbm_angle* out, int n);
/* Measure every case now and return cases 0..n-1 (synchronises). */
lbm_status lbm_batch_measure(lbm_batch* b, lbm_angle* out, int n);
/* Unbalanced Young force of every case (Sec. IV E, Eq. 17-18), as
 * lbm_young_force computes it for one lattice: a measurement of every case now
 * (written to angles[0..n), sectors as lbm_batch_measure), the footprint counts
 * of each case on the density that measurement derived, then Eq. 18 and Eq. 17
 * in FP64 into out[0..n).  A case without a contact line gets out[c].status =
 * LBM_E_NO_CONTACT_LINE and NaN values; the call itself still succeeds.  n must
 * equal the number of cases.  Synchronises.  Errors: LBM_E_ARG (null pointer,
 * n, or options as for lbm_young_force), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_batch_young_force(lbm_batch* b, const lbm_young_opts* opts, lbm_angle* angles, lbm_young* out, int n);

/* Take the unbalanced Young force at every in-step measurement of every case
 * (as lbm_set_young does for one lattice; NULL turns it off), and read the
 * latest record of cases 0..n-1 (status LBM_E_NO_CONTACT_LINE and NaN values
 * before the first measurement or without a contact line).  Both synchronise.
 * Errors: LBM_E_ARG, LBM_E_STATE (off, for the read), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_batch_set_young(lbm_batch* b, const lbm_young_opts* opts);
lbm_status lbm_batch_young_last(lbm_batch* b, lbm_young* out, int n);

/* Fields of one case: RHO (n*elem bytes), F (Q*n*elem, [Q][n]), CLASS (n bytes);
 * the phase-field model also PHI (n*elem) and G (Q*n*elem).  Synchronises. */
lbm_status lbm_batch_read(lbm_batch* b, int case_index, int field, void* dst, size_t bytes, int dst_on_device);
/* Replace one case's state by f_eq(rho, 0) (LBM_FIELD_RHO; a warm start), or
 * for the phase-field model by the state at rest of an order-parameter field
 * (LBM_FIELD_PHI: phi on fluid nodes, rho = pf_rho0, g at rest).  Every other
 * case keeps its state (both population sets are brought to the same form
 * first).  Synchronises.  LBM_E_ARG for another field or a wrong size. */
lbm_status lbm_batch_write(lbm_batch* b, int case_index, int field, const void* src, size_t bytes, int src_on_device);
lbm_status lbm_batch_get_info(lbm_batch* b, lbm_batch_info* info);
/* Re-run the autotuner (the state is unchanged). */
lbm_status lbm_batch_tune(lbm_batch* b, const char* cache_path);
/* Advance every case nsteps steps (no measurement) with a HIP event pair
 * around each launch of kb_density, kb_mu and kb_collide (kb_pf_density,
 * kb_pf_mu and kb_pf_collide for the phase-field model), and report their
 * mean duration in milliseconds: names[i] (static strings) and ms[i] for
 * i < *n_kinds (cap entries at most).  Synchronises.  Errors: LBM_E_ARG,
 * LBM_E_STATE before any initial state, LBM_E_DEVICE, LBM_E_NONFINITE. */
lbm_status lbm_batch_profile_step(lbm_batch* b, int64_t nsteps, const char** names, double* ms, int cap,
                                  int* n_kinds);
const char* lbm_batch_last_error(const lbm_batch* b);

/* ------------------------------------------------------------------------
 * Learned warm start
 *
 * A convolutional U-Net maps planes of a 2-D lattice (channel 0: 1 on solid
 * nodes; channel 1: a value on solid nodes, the scaled wall chemical
 * potential; channel 2: a constant, the scaled drop volume; channel 3: phi of
 * the cold initial state of Eq. 16) to phi = (rho - rho_g) / (rho_l - rho_g)
 * of the equilibrated drop.  Its output,
 * made mass-exact by lbm_unet_warm_rho, replaces the initial density of
 * Eq. 16 through lbm_write / lbm_batch_write (RHO).  This is an extension:
 * the paper initialises every run with Eq. 16 (Sec. IV).
 *
 * Architecture: levels l = 0..L-1 with C_l = base_channels * 2^l channels;
 * per level two 3x3 convolutions (zero padding 1) each followed by ReLU; 2x2
 * max pooling between encoder levels; per decoder level a 2x2 stride-2
 * transposed convolution from C_{l+1} to C_l channels, concatenation
 * [upsampled | encoder output of level l], two 3x3 convolutions with ReLU; a
 * 1x1 head to one channel, no activation.  Products run on BF16 MFMA tiles
 * with FP32 accumulation; activations and their gradients are BF16;
 * weights, gradients and Adam moments are FP32.
 *
 * Tensors crossing this interface are FP32 device arrays, NHWC:
 * inputs x [n][H][W][in_channels], outputs and targets [n][H][W]
 * (the lattice's x is W, its y is H).
 *
 * Parameters form one FP32 vector in this order:
 *   for l = 0..L-1:  conv W [C_l][3][3][C_in(l)], b [C_l];  conv W [C_l][3][3][C_l], b [C_l]
 *                    (C_in(0) = in_channels, C_in(l) = C_{l-1});
 *   for l = L-2..0:  up W [2][2][C_l][C_{l+1}] (row (2a + b) C_l + co: output pixel
 *                    (2h + a, 2w + b) from input pixel (h, w)), b [C_l];
 *                    conv W [C_l][3][3][2 C_l] (input channels: upsampled first), b [C_l];
 *                    conv W [C_l][3][3][C_l], b [C_l];
 *   head w [C_0], b [1].
 * A 3x3 weight W[co][dy + 1][dx + 1][ci] multiplies input pixel (h + dy, w + dx).
 * The loss is the mean squared error over the n H W outputs.
 * ------------------------------------------------------------------------ */
typedef struct lbm_unet lbm_unet;

typedef struct {
    int H, W;            /* lattice rows and columns; divisible by 2^(levels-1) */
    int batch;           /* largest n of a call */
    int in_channels;     /* 1..8 (3 for the warm start) */
    int base_channels;   /* C_0: a multiple of 8 that divides 256 (8..128) */
    int levels;          /* L: 1..6 */
    double lr, beta1, beta2, eps;  /* Adam */
    void* stream;        /* hipStream_t or NULL (the network creates one) */
} lbm_unet_config;

enum { LBM_UNET_WEIGHTS = 0, LBM_UNET_GRADS = 1 };

/* H = W = 256, batch 8, 3 inputs, C_0 = 32, L = 4, Adam 1e-3 / 0.9 / 0.999 / 1e-8. */
void lbm_unet_config_default(lbm_unet_config* cfg);
/* Allocate the network (weights zero; set them with lbm_unet_set_params).
 * Errors: LBM_E_ARG (a field out of range), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_unet_create(const lbm_unet_config* cfg, lbm_unet** out);
lbm_status lbm_unet_destroy(lbm_unet* u);
int64_t lbm_unet_param_count(const lbm_unet* u);
/* Replace the weights (n = lbm_unet_param_count) and reset the Adam state. */
lbm_status lbm_unet_set_params(lbm_unet* u, const float* p, int64_t n, int src_on_device);
/* Copy out the weights (LBM_UNET_WEIGHTS) or the gradients of the last backward pass (LBM_UNET_GRADS). */
lbm_status lbm_unet_get_params(lbm_unet* u, float* p, int64_t n, int which, int dst_on_device);
/* y = network(x) for n samples (1 <= n <= batch); x, y on the device.  Synchronises. */
lbm_status lbm_unet_forward(lbm_unet* u, const float* x, float* y, int n);
/* Forward and the loss against target (device) only; loss (host). */
lbm_status lbm_unet_loss(lbm_unet* u, const float* x, const float* target, int n, double* loss);
/* Forward, loss against target (device), and gradients of every parameter; loss (host, nullable). */
lbm_status lbm_unet_backward(lbm_unet* u, const float* x, const float* target, int n, double* loss);
/* lbm_unet_backward, then one Adam step with bias correction. */
lbm_status lbm_unet_train_step(lbm_unet* u, const float* x, const float* target, int n, double* loss);
lbm_status lbm_unet_set_lr(lbm_unet* u, double lr);
/* Checkpoint: write the weights, the Adam moments and the Adam step to path
 * ("LBMUNET1", int32 {in_channels, base_channels, levels, 0}, int64 {parameter
 * count, step}, FP32 weights, first moments, second moments; host byte
 * order).  Synchronises.  LBM_E_ARG if the file cannot be written. */
lbm_status lbm_unet_save(lbm_unet* u, const char* path);
/* Restore a checkpoint written by lbm_unet_save for the same architecture
 * (in_channels, base_channels, levels; H, W and batch may differ).
 * LBM_E_ARG if the file is missing, truncated or of another architecture. */
lbm_status lbm_unet_load(lbm_unet* u, const char* path);

/* Input planes from a lattice's CLASS field (device, [n] uint8): x[i] =
 * {solid, solid ? solid_value : 0, plane} (x device FP32 [n][3]), and with
 * phi0 (device [n], nullable; the phi of the cold initial state) a fourth
 * channel phi0[i] (x [n][4]).  Enqueues on stream. */
lbm_status lbm_unet_encode(const uint8_t* cls, const float* phi0, int64_t n, double solid_value, double plane,
                           float* x, void* stream);
/* Training target from a density field (device, elem of precision): phi =
 * (rho - rho_g) / (rho_l - rho_g) on fluid nodes, 0 on solid nodes.  Enqueues on stream. */
lbm_status lbm_unet_target(const void* rho, int precision, const uint8_t* cls, int64_t n, double rho_g, double rho_l,
                           float* phi, void* stream);
/* Density for a warm start from a predicted phi (device [ny][nx]) of a 2-D
 * lattice: with smooth = r > 0, phi is first replaced, on fluid nodes, by its
 * mean over the fluid nodes of the (2r + 1)^2 window around each (periodic
 * images; r = 2 removes the one-node artefacts a prediction can carry, which
 * the fourth-order force would otherwise amplify; needs nx ny <= H W).  Fluid
 * nodes then get rho_g + (rho_l - rho_g) s clamp((phi + delta - cut) /
 * (1 - 2 cut), 0, 1), with delta (bisection) and s (close to 1) chosen so that
 * the fluid mass equals that of rho_ref (the cold initial state), solid nodes
 * 0; rho_out has the element type of precision.  cut in [0, 0.25) sends
 * predictions within cut of pure gas or liquid to exactly rho_g or rho_l (the
 * gas density is 1/37 of the liquid's at Tr = 0.8 and 1/850 at Tr = 0.6, so
 * small errors in phi would otherwise move it by multiples of itself).  info
 * (host, nullable, 5 doubles) = {reference mass, written mass, delta, s, fluid
 * nodes}.  Runs on the network's stream; synchronises.  LBM_E_ARG if cut or
 * smooth (0..8) is out of range, or the reference mass is not strictly
 * between n_fluid rho_g and n_fluid rho_l. */
lbm_status lbm_unet_warm_rho(lbm_unet* u, const float* phi, const void* rho_ref, const uint8_t* cls, int nx, int ny,
                             int precision, double rho_g, double rho_l, double cut, int smooth, void* rho_out,
                             double* info);
const char* lbm_unet_last_error(const lbm_unet* u);

#ifdef __cplusplus
}
#endif
#endif
