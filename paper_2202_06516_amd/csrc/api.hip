// api.hip -- the C ABI of lbm.h: contexts, launches, hipGraph step loops.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "host.hpp"
#include "kernels.hpp"
#include "fused.hpp"
#include "phasefield.hpp"
#include "young.hpp"

using namespace lbm;

namespace {

constexpr int kGraphSteps = 32;  // steps per captured graph (even: buffer parity is preserved)
constexpr int kFusedTY = 4;      // rows per workgroup of the one-pass step
constexpr int kMassBlocks = 1024;

// Device memory of lbm_measure_field, the entry point that allocates nothing:
// the control word and reduction slots (centroid sums, per-sector keys) of one
// measurement.  Each GPU holds its own copy for the life of the process.  In
// host code the name stands for no device address: kernels and copies get the
// address hipGetSymbolAddress returns for the current device (scratch_ptr).
constexpr size_t kScratchBytes = 2048;
static_assert(sizeof(DevCtl) <= kScratchBytes, "the measurement's slots must fit the static scratch");
static_assert(sizeof(AngleRec) == sizeof(lbm_angle), "AngleRec is written where lbm_angle is read");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local std::string g_free_err;  // last error of a call without a context (lbm_last_error(NULL))

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// address of this device's scratch, looked up once per device
lbm_status scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        g_free_err = "measure_field: no current HIP device";
        return LBM_E_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            g_free_err = std::string("measure_field: hipGetSymbolAddress: ") + hipGetErrorString(e);
            return LBM_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

struct lbm_ctx {
    lbm_config cfg{};
    std::string err;
    PRState pr{};
    double wall_mu = 0, rho_m = 0;
    double mu_ref = 0;  // stored mu is mu - mu_ref (k^2 mu_sat)
    int dim = 2, Q = 9;
    bool f64 = false;
    size_t elem = 4;
    Dims d{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;        // populations of the current state are in f[cur]
    bool fstar = false;  // f[cur] holds post-collision populations (pull form), else S_t
    void *rho = nullptr, *mu = nullptr;  // rho: the current density buffer, rhob[rcur]
    void* rhob[2] = {nullptr, nullptr};  // the one-pass step writes rho_{t+1} into the other one
    int rcur = 0;
    void *gy = nullptr, *gz = nullptr, *gyz = nullptr;  // its ghost sums
    void* force = nullptr;   // [3][N] force of the current state, read by the one-pass step
    void* sink = nullptr;    // [19][1024] slots the one-pass step's lanes without a fluid node read and write
    bool fused = false;      // the one-pass step k_step (D3Q19 lattices of whole-row tiles)
    int fzc = 0;             // planes per k_step workgroup
    bool rho_valid = false;  // rho (fluid + solid layers) and mu hold the fields of the current state
    uint8_t* cls = nullptr;
    uint32_t* nbmask = nullptr;
    int* bidx = nullptr;
    long long *l1_node = nullptr, *l2_node = nullptr, *b_node = nullptr;
    uint32_t *l1_mask = nullptr, *l2_mask = nullptr, *b_mask = nullptr;
    int* curved = nullptr;  // boundary-list indices of nodes with a cut link of q other than 1/2
    int n_curved = 0;       // their number when the one-pass step runs the interpolated wall, else 0
    void *l1_inv = nullptr, *l2_inv = nullptr, *b_q = nullptr;
    int n_l1 = 0, n_l2 = 0, n_b = 0;
    long long n_fluid = 0;
    DevCtl* ctl = nullptr;
    AngleRec* last = nullptr;
    AngleRec* series = nullptr;
    int series_capacity = 0;
    double* mass_part = nullptr;
    double* mass_out = nullptr;
    unsigned* young_counts = nullptr;  // [LBM_MAX_SECTORS][2] footprint counts of lbm_young_force
    bool young_on = false;             // the Young force at every in-step measurement (lbm_set_young)
    lbm_young_opts yopts{};
    YoungRec* ylast = nullptr;         // its latest record
    unsigned* ystep_counts = nullptr;  // its footprint counts, zero between measurements
    YoungRec* yseries = nullptr;       // its series, alongside the angle series
    int yseries_capacity = 0;
    int series_written = 0;            // records of the last lbm_step series
    bool have_geometry = false, have_state = false;
    std::vector<Solid> solids;
    lbm_measure_opts mopts{0, 32, 0.0};
    long long t = 0;  // host mirror of the step counter
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // phase-field model: the order-parameter populations (same form and
    // buffer parity as f) and the order parameter, whose solid layers hold phi_w
    bool pf = false;
    void* g[2] = {nullptr, nullptr};
    void* phi = nullptr;
};

namespace {

// the field whose isolevel is the interface: phi in the phase-field model, else rho
inline void* mfield(const lbm_ctx* c) { return c->pf ? c->phi : c->rho; }

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

template <typename T>
lbm_status dalloc(lbm_ctx* c, T** p, size_t bytes) {
    dfree(*p);
    *p = nullptr;
    if (bytes == 0) return LBM_OK;
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, LBM_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return LBM_OK;
}

void drop_graphs(lbm_ctx* c) {
    for (auto& g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

MeasureParams measure_params(const lbm_ctx* c, const lbm_measure_opts& o) {
    MeasureParams mp{};
    const Solid& s = c->solids[o.solid_index];
    for (int k = 0; k < 3; ++k) {
        mp.c[k] = k < c->dim ? s.c[k] : 0.0;
        mp.g[k] = k < c->dim ? c->cfg.g[k] : 0.0;
    }
    mp.R = s.r;
    mp.concave = s.concave;
    mp.rho_m = o.rho_m > 0 ? o.rho_m : c->rho_m;
    mp.n_sectors = c->dim == 2 ? 2 : o.n_sectors;
    mp.dim = c->dim;
    return mp;
}

lbm_status check_measure_opts(lbm_ctx* c, const lbm_measure_opts& o) {
    if (o.solid_index < 0 || o.solid_index >= (int)c->solids.size())
        return fail(c, LBM_E_ARG, "measure: solid_index out of range (set solids first)");
    if (c->dim == 3 && (o.n_sectors < 1 || o.n_sectors > LBM_MAX_SECTORS))
        return fail(c, LBM_E_ARG, "measure: n_sectors must lie in 1..64");
    return LBM_OK;
}

// Tile shape and launch counts of a lattice whose nx, ny, nz are set.
void tile_dims(Dims& d, int dim) {
    {
        // tile width: the widest of 256, 128, 64 nodes that the row fills (wide rows
        // straddle fewer cache lines in the x-shifted gathers); LBM_TILE_W overrides
        const char* e = std::getenv("LBM_TILE_W");
        const int tw = e ? std::atoi(e) : (d.nx >= 256 ? 256 : d.nx >= 128 ? 128 : 64);
        d.tws = tw == 256 ? 8 : tw == 128 ? 7 : 6;
    }
    d.tx = (d.nx + (1 << d.tws) - 1) >> d.tws;
    d.ty = (d.ny + (256 >> d.tws) - 1) / (256 >> d.tws);
    d.nblocks = (unsigned)d.tx * (unsigned)d.ty * (unsigned)d.nz;
    {
        // planes per workgroup of the chemical-potential kernel (3-D): 8 took it from 0.080 to 0.067 ms
        // at 256^3; LBM_ZCHUNK overrides
        const char* e = std::getenv("LBM_ZCHUNK");
        const int zc = dim == 3 ? (e ? std::atoi(e) : 8) : 1;
        d.zc = zc < 1 ? 1 : zc;
        d.nblocks_zc = (unsigned)d.tx * (unsigned)d.ty * (unsigned)((d.nz + d.zc - 1) / d.zc);
    }
    {
        const char* e = std::getenv("LBM_XCD_REMAP");
        d.xcd_remap = e ? std::atoi(e) != 0 : 1;
    }
}

// ---------------------------------------------------------------------------
// typed launcher
// ---------------------------------------------------------------------------
template <class L, typename R, typename C = R>
struct Run {
    static Thermo thermo(const lbm_ctx* c) {
        const double k2 = c->cfg.k * c->cfg.k;
        const PRState& p = c->pr;
        Thermo th;
        th.k2RT = k2 * p.R * p.T;
        th.k2A = k2 * p.a * p.alpha / (2.0 * std::sqrt(2.0) * p.b);
        th.k2aal = k2 * p.a * p.alpha;
        th.b = p.b;
        th.s2m1 = std::sqrt(2.0) - 1.0;
        th.s2p1 = std::sqrt(2.0) + 1.0;
        th.mu_ref = c->mu_ref;
        th.kappa = c->cfg.kappa;
        return th;
    }
    static Collision<C> collision(const lbm_ctx* c) {
        Collision<C> cp{};
        const lbm_config& g = c->cfg;
        cp.bgk = g.collision == LBM_BGK;
        cp.omega = (C)(1.0 / g.tau);
        const double sv = 1.0 / g.tau;
        for (int k = 0; k < 19; ++k) cp.rate[k] = C(0);
        for (int k = 0; k < L::Q; ++k) {
            double s = 0;
            switch (L::kind(k)) {
                case 1: s = g.s_e; break;
                case 2: s = g.s_eps; break;
                case 3: s = g.s_q; break;
                case 4: s = sv; break;
                case 5: s = g.s_pi; break;
                case 6: s = g.s_m; break;
                default: s = 0; break;
            }
            cp.rate[k] = (C)(s / row_norm2<L>(k));
        }
        for (int k = 0; k < 3; ++k) cp.g[k] = k < c->dim ? g.g[k] : 0.0;
        cp.g_start = g.g_start_step;
        cp.sc_G = g.sc_G;
        return cp;
    }
    static dim3 grid(const lbm_ctx* c) { return dim3(c->d.nblocks, 1, 1); }
    // the z-chunked chemical-potential kernel
    static dim3 zgrid(const lbm_ctx* c) { return dim3(c->d.zc > 1 ? c->d.nblocks_zc : c->d.nblocks, 1, 1); }
    // the crossing search walks the tiles in a grid-stride loop
    static dim3 cross_grid(const lbm_ctx* c) { return dim3(c->d.nblocks < 2048u ? c->d.nblocks : 2048u, 1, 1); }

    // The wall condition of a gather of the stored state.  On the one-pass path
    // the interpolated wall is already in the slots the pull reads
    // (k_interp_wall after each step), so its gathers take halfway bounce-back.
    static WallBC wall(const lbm_ctx* c) {
        WallBC bc;
        bc.nbmask = c->nbmask;
        bc.bidx = c->bidx;
        bc.q = c->b_q;
        bc.bouzidi = c->cfg.bc_mode == LBM_BC_BOUZIDI_MC && !c->fused;
        return bc;
    }
    static void density(lbm_ctx* c, const R* f, bool pull, double rho_m) {
        const dim3 blk(256, 1, 1), grd = grid(c);
        const R inv_b = (R)(1.0 / c->pr.b);
        if (pull)
            k_density<L, R, C, true><<<grd, blk, 0, c->stream>>>(f, (R*)c->rho, c->cls, c->d, wall(c), c->ctl, rho_m, inv_b);
        else
            k_density<L, R, C, false><<<grd, blk, 0, c->stream>>>(f, (R*)c->rho, c->cls, c->d, wall(c), c->ctl, rho_m, inv_b);
    }
    static void fills(lbm_ctx* c, hipEvent_t* ev, int* kinds, int& k) { fills_on(c, (R*)c->rho, ev, kinds, k); }
    static void fills_on(lbm_ctx* c, R* rho, hipEvent_t* ev, int* kinds, int& k) {
        if (c->n_l1) {
            if (ev) (void)hipEventRecord(ev[2 * k], c->stream);
            k_fill<L, R, C><<<(c->n_l1 + 255) / 256, 256, 0, c->stream>>>(c->l1_node, c->l1_mask, (const R*)c->l1_inv,
                                                                           c->n_l1, rho, c->d);
            if (ev) { (void)hipEventRecord(ev[2 * k + 1], c->stream); kinds[k++] = 1; }
        }
        if (c->n_l2) {
            if (ev) (void)hipEventRecord(ev[2 * k], c->stream);
            k_fill<L, R, C><<<(c->n_l2 + 255) / 256, 256, 0, c->stream>>>(c->l2_node, c->l2_mask, (const R*)c->l2_inv,
                                                                           c->n_l2, rho, c->d);
            if (ev) { (void)hipEventRecord(ev[2 * k + 1], c->stream); kinds[k++] = 2; }
        }
    }

    // the in-step Young force: counting parameters (the drop axis comes from
    // the measurement's own centroid on the device) and the Eq. 17-18 options
    static YoungParams young_step_params(const lbm_ctx* c, const MeasureParams& mp) {
        double lo, hi;
        young_band(c->yopts, lo, hi);
        lbm_angle a{};
        a.n_sectors = mp.n_sectors;
        return young_params(c->solids[c->mopts.solid_index], a, c->dim, c->pr.rho_g, c->pr.rho_l, lo, hi);
    }
    static YoungStep young_step(const lbm_ctx* c, const MeasureParams&) {
        YoungStep ys{};
        ys.on = 1;
        ys.gamma = c->yopts.gamma;
        ys.c1 = std::cos(c->yopts.theta1_deg * M_PI / 180.0);
        ys.c2 = std::cos(c->yopts.theta2_deg * M_PI / 180.0);
        ys.roughness = c->yopts.roughness;
        ys.counts = c->ystep_counts;
        ys.last = c->ylast;
        return ys;
    }

    // chemical potential, or psi of the pseudopotential model, on fluid nodes
    static void launch_mu(lbm_ctx* c, R* rho, R* mu) {
        const dim3 blk(256, 1, 1);
        const bool sc = c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL, zch = c->d.zc > 1;
        if (sc && zch) k_mu<L, R, C, true, true><<<zgrid(c), blk, 0, c->stream>>>(rho, mu, c->cls, c->d, thermo(c));
        else if (sc) k_mu<L, R, C, true><<<grid(c), blk, 0, c->stream>>>(rho, mu, c->cls, c->d, thermo(c));
        else if (zch) k_mu<L, R, C, false, true><<<zgrid(c), blk, 0, c->stream>>>(rho, mu, c->cls, c->d, thermo(c));
        else k_mu<L, R, C><<<grid(c), blk, 0, c->stream>>>(rho, mu, c->cls, c->d, thermo(c));
    }

    template <bool PULL, bool MRT>
    static void launch_collide(lbm_ctx* c, const R* fin, R* fout, R* rho, R* mu, const WallBC& bc,
                               const Collision<C>& cp) {
        const dim3 blk(256, 1, 1), grd = grid(c);
        if (c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL)
            k_collide<L, R, C, PULL, MRT, true><<<grd, blk, 0, c->stream>>>(fin, fout, rho, mu, c->cls, c->d, bc, cp, c->ctl);
        else
            k_collide<L, R, C, PULL, MRT><<<grd, blk, 0, c->stream>>>(fin, fout, rho, mu, c->cls, c->d, bc, cp, c->ctl);
    }

    // the launches of one step, reading f[src] and writing f[1-src]; pull
    // selects the form of f[src] (post-collision populations, else S_t)
    static void step_launches(lbm_ctx* c, int src, bool pull, const MeasureParams& mp, hipEvent_t* ev, int* kinds) {
        if (c->pf) {
            pf_step_launches(c, src, pull, mp, ev, kinds);
            return;
        }
        const dim3 blk(256, 1, 1), grd = grid(c);
        const R* fin = (const R*)c->f[src];
        R* fout = (R*)c->f[1 - src];
        R* rho = (R*)c->rho;
        R* mu = (R*)c->mu;
        int k = 0;
        auto start = [&]() { if (ev) (void)hipEventRecord(ev[2 * k], c->stream); };
        auto mark = [&](int kind) { if (ev) { (void)hipEventRecord(ev[2 * k + 1], c->stream); kinds[k++] = kind; } };
        start();
        density(c, fin, pull, mp.rho_m);
        mark(0);
        fills(c, ev, kinds, k);
        start();
        launch_mu(c, rho, mu);
        mark(3);
        start();
        k_cross<L, R><<<cross_grid(c), blk, 0, c->stream>>>(rho, c->cls, c->d, c->ctl, mp);
        YoungStep ys{};
        if (c->young_on) {
            ys = young_step(c, mp);
            k_young_step<L, R><<<cross_grid(c), blk, 0, c->stream>>>(rho, c->cls, c->d, young_step_params(c, mp), mp,
                                                                    c->ctl, c->ystep_counts);
        }
        mark(5);
        start();
        const WallBC bc = wall(c);
        const Collision<C> cp = collision(c);
        const bool mrt = c->cfg.collision == LBM_MRT;
        if (pull) {
            if (mrt) launch_collide<true, true>(c, fin, fout, rho, mu, bc, cp);
            else launch_collide<true, false>(c, fin, fout, rho, mu, bc, cp);
        } else {
            if (mrt) launch_collide<false, true>(c, fin, fout, rho, mu, bc, cp);
            else launch_collide<false, false>(c, fin, fout, rho, mu, bc, cp);
        }
        mark(4);
        start();
        k_finalize<L, R><<<1, 64, 0, c->stream>>>(rho, c->ctl, c->d, mp, c->series, c->last, 1, ys, c->yseries);
        mark(6);
        if (kinds) kinds[k] = -1;
    }

    // phase-field model (the split step): parameters, density, mu, collision
    static PhaseField phase_field(const lbm_ctx* c) {
        PhaseField pf;
        pf.A = c->cfg.pf_A;
        pf.kappa = c->cfg.pf_kappa;
        pf.gamma = c->cfg.pf_gamma;
        pf.omega = 1.0 / c->cfg.pf_tau;
        pf.rho0 = c->cfg.pf_rho0;
        return pf;
    }
    static WallBC halfway(const lbm_ctx* c) {
        WallBC bc = wall(c);
        bc.bouzidi = 0;
        return bc;
    }
    // phi of the state in f[src] / g[src]; with_rho: rho as well (the fields a
    // read or a measurement returns; the step's collision forms rho itself)
    static void pf_density(lbm_ctx* c, int src, bool pull, double phi_m, bool with_rho) {
        const R* f = (const R*)c->f[src];
        const R* g = (const R*)c->g[src];
        const dim3 grd = grid(c), blk(256, 1, 1);
#define LBM_PF_DENSITY(P, W) \
    k_pf_density<L, R, C, P, W><<<grd, blk, 0, c->stream>>>(f, g, (R*)c->rho, (R*)c->phi, c->cls, c->d, wall(c), \
                                                            c->ctl, phi_m)
        if (pull) {
            if (with_rho) LBM_PF_DENSITY(true, true);
            else LBM_PF_DENSITY(true, false);
        } else {
            if (with_rho) LBM_PF_DENSITY(false, true);
            else LBM_PF_DENSITY(false, false);
        }
#undef LBM_PF_DENSITY
    }
    static void pf_mu(lbm_ctx* c) {
        if (c->d.zc > 1)
            k_pf_mu<L, R, true><<<zgrid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->phi, (R*)c->mu, c->cls, c->d,
                                                                             phase_field(c));
        else
            k_pf_mu<L, R, false><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->phi, (R*)c->mu, c->cls, c->d,
                                                                             phase_field(c));
    }
    template <bool PULL, bool MRT>
    static void pf_collide(lbm_ctx* c, int src, const WallBC& bc, const Collision<C>& cp) {
        k_pf_collide<L, R, C, PULL, MRT><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>(
            (const R*)c->f[src], (R*)c->f[1 - src], (const R*)c->g[src], (R*)c->g[1 - src], (const R*)c->phi,
            (const R*)c->mu, c->cls, c->d, bc, cp, phase_field(c), c->ctl);
    }
    static void pf_step_launches(lbm_ctx* c, int src, bool pull, const MeasureParams& mp, hipEvent_t* ev,
                                 int* kinds) {
        const dim3 blk(256, 1, 1);
        const R* phi = (const R*)c->phi;
        int k = 0;
        auto start = [&]() { if (ev) (void)hipEventRecord(ev[2 * k], c->stream); };
        auto mark = [&](int kind) { if (ev) { (void)hipEventRecord(ev[2 * k + 1], c->stream); kinds[k++] = kind; } };
        start();
        pf_density(c, src, pull, mp.rho_m, false);
        mark(0);
        start();
        pf_mu(c);
        mark(3);
        start();
        k_cross<L, R><<<cross_grid(c), blk, 0, c->stream>>>(phi, c->cls, c->d, c->ctl, mp);
        YoungStep ys{};
        if (c->young_on) {
            ys = young_step(c, mp);
            k_young_step<L, R><<<cross_grid(c), blk, 0, c->stream>>>(phi, c->cls, c->d, young_step_params(c, mp), mp,
                                                                    c->ctl, c->ystep_counts);
        }
        mark(5);
        start();
        const WallBC bc = wall(c);
        const Collision<C> cp = collision(c);
        const bool mrt = c->cfg.collision == LBM_MRT;
        if (pull) {
            if (mrt) pf_collide<true, true>(c, src, bc, cp);
            else pf_collide<true, false>(c, src, bc, cp);
        } else {
            if (mrt) pf_collide<false, true>(c, src, bc, cp);
            else pf_collide<false, false>(c, src, bc, cp);
        }
        mark(4);
        start();
        k_finalize<L, R><<<1, 64, 0, c->stream>>>(phi, c->ctl, c->d, mp, c->series, c->last, 1, ys, c->yseries);
        mark(6);
        if (kinds) kinds[k] = -1;
    }
    // S_t of the order-parameter populations into g[1 - cur]
    static R* materialize_g(lbm_ctx* c) {
        R* out = (R*)c->g[1 - c->cur];
        if (c->fstar)
            k_materialize<L, R, C, true><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->g[c->cur], out, c->cls,
                                                                                    c->d, halfway(c));
        else
            k_materialize<L, R, C, false><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->g[c->cur], out,
                                                                                     c->cls, c->d, halfway(c));
        return out;
    }
    // the state of an order-parameter field (device array of N values)
    static void pf_init(lbm_ctx* c, const void* src) {
        k_pf_init<L, R><<<2048, 256, 0, c->stream>>>((const R*)src, (R*)c->phi, (R*)c->rho, (R*)c->f[c->cur],
                                                     (R*)c->g[c->cur], c->cls, c->d.N, c->cfg.pf_rho0, 0, c->d.N);
    }

    // One step on the one-pass path, reading f[src] and rhob[rsrc] (rho_t, with
    // mu_t in mu) and writing f[1-src] and rhob[1-rsrc] (rho_{t+1}, mu_{t+1}).
    template <bool PULL, bool MRT, bool SC>
    static void launch_step(lbm_ctx* c, const R* fin, R* fout, const R* rho, R* rnext, const WallBC& bc,
                            const Collision<C>& cp) {
        const dim3 grd((unsigned)((c->d.ny / kFusedTY) * (c->d.nz / c->fzc)), 1, 1), blk((unsigned)c->d.nx, 1, 1);
        // workgroup = one row of nx threads; the launch bound follows it
        if (c->d.nx <= 256)
            k_step<R, C, PULL, MRT, SC, kFusedTY, 256><<<grd, blk, 0, c->stream>>>(
                fin, fout, rho, (const R*)c->mu, (const R*)c->force, rnext, (R*)c->gy, (R*)c->gz, (R*)c->gyz, c->cls,
                c->d, bc, cp, c->ctl, c->fzc, (R*)c->sink);
        else
            k_step<R, C, PULL, MRT, SC, kFusedTY, 1024><<<grd, blk, 0, c->stream>>>(
                fin, fout, rho, (const R*)c->mu, (const R*)c->force, rnext, (R*)c->gy, (R*)c->gz, (R*)c->gyz, c->cls,
                c->d, bc, cp, c->ctl, c->fzc, (R*)c->sink);
    }
    // the force of the current state (rho, mu) into c->force
    static void launch_force(lbm_ctx* c, const R* rho) {
        const dim3 blk(256, 1, 1);
        if (c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL)
            k_force<L, R, C, true><<<zgrid(c), blk, 0, c->stream>>>(rho, (const R*)c->mu, c->cls, c->d, collision(c),
                                                                    c->ctl, (R*)c->force);
        else
            k_force<L, R, C, false><<<zgrid(c), blk, 0, c->stream>>>(rho, (const R*)c->mu, c->cls, c->d, collision(c),
                                                                     c->ctl, (R*)c->force);
    }
    // quiet: a step known on the host to measure nothing (t % every != 0); it
    // leaves out k_cross, k_young_step and k_finalize, which return at once on
    // such steps, and k_ghost counts the step instead of k_finalize
    static void fused_step_launches(lbm_ctx* c, int src, bool pull, int rsrc, const MeasureParams& mp, hipEvent_t* ev,
                                    int* kinds, bool quiet = false) {
        if constexpr (L::D == 3) {
            const dim3 blk(256, 1, 1);
            const R* fin = (const R*)c->f[src];
            R* fout = (R*)c->f[1 - src];
            R* rho = (R*)c->rhob[rsrc];
            R* rnext = (R*)c->rhob[1 - rsrc];
            int k = 0;
            auto start = [&]() { if (ev) (void)hipEventRecord(ev[2 * k], c->stream); };
            auto mark = [&](int kind) { if (ev) { (void)hipEventRecord(ev[2 * k + 1], c->stream); kinds[k++] = kind; } };
            YoungStep ys{};
            if (!quiet) {
                start();
                k_cross<L, R><<<cross_grid(c), blk, 0, c->stream>>>(rho, c->cls, c->d, c->ctl, mp);
                if (c->young_on) {
                    ys = young_step(c, mp);
                    k_young_step<L, R><<<cross_grid(c), blk, 0, c->stream>>>(rho, c->cls, c->d,
                                                                            young_step_params(c, mp), mp, c->ctl,
                                                                            c->ystep_counts);
                }
                mark(5);
            }
            start();
            const WallBC bc = wall(c);
            const Collision<C> cp = collision(c);
            const bool mrt = c->cfg.collision == LBM_MRT, sc = c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL;
            if (sc) {
                if (pull) { if (mrt) launch_step<true, true, true>(c, fin, fout, rho, rnext, bc, cp);
                            else launch_step<true, false, true>(c, fin, fout, rho, rnext, bc, cp); }
                else { if (mrt) launch_step<false, true, true>(c, fin, fout, rho, rnext, bc, cp);
                       else launch_step<false, false, true>(c, fin, fout, rho, rnext, bc, cp); }
            } else {
                if (pull) { if (mrt) launch_step<true, true, false>(c, fin, fout, rho, rnext, bc, cp);
                            else launch_step<true, false, false>(c, fin, fout, rho, rnext, bc, cp); }
                else { if (mrt) launch_step<false, true, false>(c, fin, fout, rho, rnext, bc, cp);
                       else launch_step<false, false, false>(c, fin, fout, rho, rnext, bc, cp); }
            }
            mark(7);
            if (c->n_curved) {
                // the interpolated wall into the slots the next pull reads
                start();
                k_interp_wall<L, R, C><<<(c->n_curved + 255) / 256, blk, 0, c->stream>>>(
                    c->curved, c->n_curved, c->b_node, c->b_mask, fout, c->d, bc);
                mark(10);
            }
            if (!quiet) {
                start();
                k_finalize<L, R><<<1, 64, 0, c->stream>>>(rho, c->ctl, c->d, mp, c->series, c->last, 1, ys,
                                                          c->yseries);
                mark(6);
            }
            start();
            {
                const int ein = 2 * (c->d.ny / kFusedTY);
                const long long rows = (long long)(c->d.nz / c->fzc) * (2LL * c->d.ny + (long long)(c->fzc - 2) * ein);
                const long long thr = rows * (c->d.nx / 4);
                k_ghost<R, kFusedTY><<<(unsigned)((thr + 255) / 256), 256, 0, c->stream>>>(
                    rnext, (const R*)c->gy, (const R*)c->gz, (const R*)c->gyz, c->d, c->fzc, rows,
                    quiet ? c->ctl : nullptr);
            }
            mark(8);
            fills_on(c, rnext, ev, kinds, k);
            start();
            const R inv_b = (R)(1.0 / c->pr.b);
            if (sc)
                k_mu_step<L, R, C, true><<<zgrid(c), blk, 0, c->stream>>>(rnext, (R*)c->mu, c->cls, c->d, thermo(c),
                                                                         c->ctl, mp.rho_m, inv_b, (R*)c->sink);
            else
                k_mu_step<L, R, C, false><<<zgrid(c), blk, 0, c->stream>>>(rnext, (R*)c->mu, c->cls, c->d, thermo(c),
                                                                          c->ctl, mp.rho_m, inv_b, (R*)c->sink);
            mark(3);
            if (sc) {
                // the pseudopotential force for the next step (k_step forms Eq. 7 itself)
                start();
                launch_force(c, rnext);
                mark(9);
            }
            if (kinds) kinds[k] = -1;
        }
    }

    // liquid centroid sums of the current density (a measurement of step t
    // whose density the previous one-pass step already completed)
    static void centroid(lbm_ctx* c, double rho_m) {
        k_centroid<L, R><<<cross_grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->rho, c->cls, c->d, rho_m, &c->ctl->m);
    }

    // S_t of the current state into f[1 - cur] (free between steps)
    static R* materialize(lbm_ctx* c) {
        R* out = (R*)c->f[1 - c->cur];
        if (c->fstar)
            k_materialize<L, R, C, true><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->f[c->cur], out, c->cls, c->d, wall(c));
        else
            k_materialize<L, R, C, false><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->f[c->cur], out, c->cls, c->d, wall(c));
        return out;
    }

    // density, solid fill and mu of the current state (no measurement)
    static void derive(lbm_ctx* c, bool with_mu) {
        if (c->pf) {
            pf_density(c, c->cur, c->fstar, c->rho_m, true);
            if (with_mu) pf_mu(c);
            return;
        }
        if (c->fused && c->rho_valid) return;  // the one-pass step keeps them current
        if (c->fused) with_mu = true;
        MeasureParams mp{};
        mp.rho_m = c->rho_m;
        mp.n_sectors = 2;
        mp.dim = c->dim;
        density(c, (const R*)c->f[c->cur], c->fstar, mp.rho_m);
        int k = 0;
        fills(c, nullptr, nullptr, k);
        if (with_mu) launch_mu(c, (R*)c->rho, (R*)c->mu);
        if (c->fused) {
            if constexpr (L::D == 3)
                if (c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL) launch_force(c, (const R*)c->rho);
            c->rho_valid = true;
        }
    }

    static void velocity(lbm_ctx* c, void* out) {
        derive(c, true);
        const R* S = materialize(c);
        if (c->pf)
            k_pf_velocity<L, R, C><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>(
                S, (const R*)c->phi, (const R*)c->mu, c->cls, c->d, collision(c), c->t, (R*)out);
        else if (c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL)
            k_velocity<L, R, C, true><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>(
                S, (const R*)c->rho, (const R*)c->mu, c->cls, c->d, collision(c), c->t, (R*)out);
        else
            k_velocity<L, R, C><<<grid(c), dim3(256, 1, 1), 0, c->stream>>>(
                S, (const R*)c->rho, (const R*)c->mu, c->cls, c->d, collision(c), c->t, (R*)out);
    }

    static void measure_now(lbm_ctx* c, const MeasureParams& mp) {
        if (c->pf) {
            pf_density(c, c->cur, c->fstar, mp.rho_m, true);
            k_cross<L, R><<<cross_grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->phi, c->cls, c->d, c->ctl, mp);
            k_finalize<L, R><<<1, 64, 0, c->stream>>>((const R*)c->phi, c->ctl, c->d, mp, nullptr, c->last, 0);
            return;
        }
        if (c->fused && c->rho_valid) {
            centroid(c, mp.rho_m);
        } else {
            density(c, (const R*)c->f[c->cur], c->fstar, mp.rho_m);
            int k = 0;
            fills(c, nullptr, nullptr, k);
            launch_mu(c, (R*)c->rho, (R*)c->mu);
            if (c->fused) {
                if constexpr (L::D == 3)
                    if (c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL) launch_force(c, (const R*)c->rho);
                c->rho_valid = true;
            }
        }
        k_cross<L, R><<<cross_grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)c->rho, c->cls, c->d, c->ctl, mp);
        k_finalize<L, R><<<1, 64, 0, c->stream>>>((const R*)c->rho, c->ctl, c->d, mp, nullptr, c->last, 0);
    }

    static void young_count(lbm_ctx* c, const YoungParams& yp) {
        k_young_count<L, R><<<cross_grid(c), dim3(256, 1, 1), 0, c->stream>>>((const R*)mfield(c), c->cls, c->d, yp,
                                                                            c->young_counts);
    }

    static void init_feq(lbm_ctx* c) {
        k_init_feq<L, R><<<2048, 256, 0, c->stream>>>((const R*)c->rho, (R*)c->f[c->cur], c->cls, c->d.N, 0, c->d.N);
    }

    static void mass(lbm_ctx* c) {
        const R* S = materialize(c);
        k_mass_partial<L, R><<<kMassBlocks, 256, 0, c->stream>>>(S, c->cls, c->d.N, c->mass_part);
        k_mass_final<<<1, 64, 0, c->stream>>>(c->mass_part, kMassBlocks, c->mass_out);
    }

};

// dispatch on (lattice, storage precision, arithmetic precision)
template <template <class, typename, typename> class Op, typename... Args>
void dispatch(lbm_ctx* c, Args&&... args) {
    const int p = c->cfg.precision;
    if (c->dim == 2) {
        if (p == LBM_F64) Op<D2Q9, double, double>::go(c, args...);
        else if (p == LBM_F32_MIXED) Op<D2Q9, float, double>::go(c, args...);
        else Op<D2Q9, float, float>::go(c, args...);
    } else {
        if (p == LBM_F64) Op<D3Q19, double, double>::go(c, args...);
        else if (p == LBM_F32_MIXED) Op<D3Q19, float, double>::go(c, args...);
        else Op<D3Q19, float, float>::go(c, args...);
    }
}

template <class L, typename R, typename C>
struct OpStep {
    static void go(lbm_ctx* c, int src, bool pull, const MeasureParams* mp, hipEvent_t* ev, int* kinds) {
        Run<L, R, C>::step_launches(c, src, pull, *mp, ev, kinds);
    }
};
template <class L, typename R, typename C>
struct OpFusedStep {
    static void go(lbm_ctx* c, int src, bool pull, int rsrc, const MeasureParams* mp, hipEvent_t* ev, int* kinds,
                   bool quiet = false) {
        Run<L, R, C>::fused_step_launches(c, src, pull, rsrc, *mp, ev, kinds, quiet);
    }
};
template <class L, typename R, typename C>
struct OpCentroid {
    static void go(lbm_ctx* c, double rho_m) { Run<L, R, C>::centroid(c, rho_m); }
};
template <class L, typename R, typename C>
struct OpDerive {
    static void go(lbm_ctx* c, bool with_mu) { Run<L, R, C>::derive(c, with_mu); }
};
template <class L, typename R, typename C>
struct OpVel {
    static void go(lbm_ctx* c, void* out) { Run<L, R, C>::velocity(c, out); }
};
template <class L, typename R, typename C>
struct OpMeasure {
    static void go(lbm_ctx* c, const MeasureParams* mp) { Run<L, R, C>::measure_now(c, *mp); }
};
template <class L, typename R, typename C>
struct OpYoung {
    static void go(lbm_ctx* c, const YoungParams* yp) { Run<L, R, C>::young_count(c, *yp); }
};
template <class L, typename R, typename C>
struct OpInit {
    static void go(lbm_ctx* c) { Run<L, R, C>::init_feq(c); }
};
template <class L, typename R, typename C>
struct OpMaterialize {
    static void go(lbm_ctx* c, void** out) { *out = Run<L, R, C>::materialize(c); }
};
template <class L, typename R, typename C>
struct OpMaterializeG {
    static void go(lbm_ctx* c, void** out) { *out = Run<L, R, C>::materialize_g(c); }
};
template <class L, typename R, typename C>
struct OpPfInit {
    static void go(lbm_ctx* c, const void* src) { Run<L, R, C>::pf_init(c, src); }
};
template <class L, typename R, typename C>
struct OpMass {
    static void go(lbm_ctx* c) { Run<L, R, C>::mass(c); }
};

// the measurement of lbm_measure_field on a caller's density field; the
// slots live in the static scratch at ctl
template <class L, typename R, typename C>
struct OpMeasureField {
    static void go(const Dims& d, const void* rho, const uint8_t* cls, DevCtl* ctl, const MeasureParams& mp,
                   AngleRec* out, hipStream_t st) {
        const R* r = (const R*)rho;
        k_ctl_set<<<1, 64, 0, st>>>(ctl, 0, 0, 1, 0, 1);
        k_ctl_reset<<<1, 64, 0, st>>>(ctl, 0, 1, 0);
        k_centroid<L, R><<<d.nblocks < 2048u ? d.nblocks : 2048u, 256, 0, st>>>(r, cls, d, mp.rho_m, &ctl->m);
        k_cross<L, R><<<d.nblocks < 2048u ? d.nblocks : 2048u, 256, 0, st>>>(r, cls, d, ctl, mp);
        k_finalize<L, R><<<1, 64, 0, st>>>(r, ctl, d, mp, nullptr, out, 0);
    }
};

// copy a host double array into a device array of the context precision
lbm_status upload_real(lbm_ctx* c, void** dst, const std::vector<double>& v) {
    lbm_status s = dalloc(c, (char**)dst, v.size() * c->elem);
    if (s != LBM_OK || v.empty()) return s;
    if (c->f64) {
        HIPCHK(c, hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> t(v.begin(), v.end());
        HIPCHK(c, hipMemcpy(*dst, t.data(), t.size() * 4, hipMemcpyHostToDevice));
    }
    return LBM_OK;
}

template <typename T>
lbm_status upload(lbm_ctx* c, T** dst, const std::vector<T>& v) {
    lbm_status s = dalloc(c, dst, v.size() * sizeof(T));
    if (s != LBM_OK || v.empty()) return s;
    HIPCHK(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return LBM_OK;
}

lbm_status ctl_reset(lbm_ctx* c, int every, int force, int cap) {
    k_ctl_reset<<<1, 64, 0, c->stream>>>(c->ctl, every, force, cap);
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status check_status(lbm_ctx* c) {
    DevCtl h;
    HIPCHK(c, hipMemcpyAsync(&h, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.status & 1) return fail(c, LBM_E_NONFINITE, "a density became non-finite, non-positive or >= 1/b");
    return LBM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void lbm_config_default(lbm_config* cfg, int lattice) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->lattice = lattice;
    cfg->precision = lattice == LBM_D2Q9 ? LBM_F64 : LBM_F32;
    cfg->n[0] = cfg->n[1] = 128;
    cfg->n[2] = lattice == LBM_D2Q9 ? 1 : 128;
    cfg->axis_bc[0] = cfg->axis_bc[1] = cfg->axis_bc[2] = LBM_PERIODIC;
    cfg->collision = lattice == LBM_D2Q9 ? LBM_MRT : LBM_BGK;
    cfg->bc_mode = LBM_BC_HALFWAY;
    cfg->tau = 1.0;
    cfg->s_e = 1.64;
    cfg->s_eps = 1.54;
    cfg->s_q = 1.9;
    cfg->s_pi = 1.54;
    cfg->s_m = 1.9;
    cfg->Tr = 0.6;
    cfg->pr_a = 2.0 / 49.0;
    cfg->pr_b = 2.0 / 21.0;
    cfg->pr_R = 1.0;
    cfg->pr_omega = 0.344;
    cfg->k = 0.28;
    cfg->kappa = 0.01;
    cfg->g_start_step = 0;
    cfg->rho_l = cfg->rho_g = 0.0;
    cfg->wall_mu = NAN;
    cfg->stream = nullptr;
    cfg->model = LBM_MODEL_CHEMICAL_POTENTIAL;
    cfg->sc_G = -6.0;
    cfg->step_kernel = LBM_STEP_AUTO;
    cfg->pf_A = 0.01;
    cfg->pf_kappa = 0.02;
    cfg->pf_gamma = 1.0;
    cfg->pf_tau = 1.0;
    cfg->pf_rho0 = 1.0;
}

const char* lbm_last_error(const lbm_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    return g_free_err.empty() ? "null context" : g_free_err.c_str();
}

lbm_status lbm_create(const lbm_config* cfg, lbm_ctx** out) {
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    if (!cfg) return LBM_E_ARG;
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_E_NOMEM;
    c->cfg = *cfg;
    auto bad = [&](const std::string& m) {
        delete c;
        return LBM_E_ARG;
        (void)m;
    };
    if (cfg->lattice != LBM_D2Q9 && cfg->lattice != LBM_D3Q19) return bad("lattice");
    if (cfg->precision != LBM_F32 && cfg->precision != LBM_F64 && cfg->precision != LBM_F32_MIXED)
        return bad("precision");
    c->dim = cfg->lattice == LBM_D2Q9 ? 2 : 3;
    c->Q = c->dim == 2 ? 9 : 19;
    c->f64 = cfg->precision == LBM_F64;
    c->elem = c->f64 ? 8 : 4;
    if (c->dim == 2 && cfg->n[2] != 1) return bad("n[2] must be 1 for D2Q9");
    for (int k = 0; k < c->dim; ++k) {
        if (cfg->n[k] < 5 || cfg->n[k] > (1 << 20)) return bad("n out of range");
        if (cfg->axis_bc[k] != LBM_PERIODIC && cfg->axis_bc[k] != LBM_WALL) return bad("axis_bc");
        if (cfg->axis_bc[k] == LBM_WALL && cfg->n[k] < 8) return bad("wall axis needs n >= 8");
    }
    const long long N = (long long)cfg->n[0] * cfg->n[1] * (c->dim == 3 ? cfg->n[2] : 1);
    if ((unsigned long long)N * (unsigned long long)c->Q >= (1ull << 32)) return bad("N * Q must stay below 2^32");
    if (!(cfg->tau > 0.5)) return bad("tau must exceed 1/2");
    if (cfg->collision != LBM_MRT && cfg->collision != LBM_BGK) return bad("collision");
    if (cfg->bc_mode != LBM_BC_HALFWAY && cfg->bc_mode != LBM_BC_BOUZIDI_MC) return bad("bc_mode");
    if (!(cfg->k > 0) || !(cfg->kappa >= 0) || !(cfg->pr_a > 0) || !(cfg->pr_b > 0) || !(cfg->pr_R > 0))
        return bad("thermodynamic parameters");
    if (cfg->model != LBM_MODEL_CHEMICAL_POTENTIAL && cfg->model != LBM_MODEL_PSEUDOPOTENTIAL &&
        cfg->model != LBM_MODEL_PHASE_FIELD)
        return bad("model");
    if (cfg->model == LBM_MODEL_PHASE_FIELD &&
        (!(cfg->pf_A > 0) || !(cfg->pf_kappa > 0) || !(cfg->pf_gamma > 0) || !(cfg->pf_tau > 0.5) ||
         !(cfg->pf_rho0 > 0) || !std::isfinite(cfg->pf_A + cfg->pf_kappa + cfg->pf_gamma + cfg->pf_tau + cfg->pf_rho0)))
        return bad("the phase-field model needs pf_A, pf_kappa, pf_gamma, pf_rho0 > 0 and pf_tau > 1/2");
    c->pf = cfg->model == LBM_MODEL_PHASE_FIELD;
    if (cfg->model == LBM_MODEL_PSEUDOPOTENTIAL &&
        (!(cfg->rho_g > 0) || !(cfg->rho_l > cfg->rho_g) || !std::isfinite(cfg->sc_G)))
        return bad("the pseudopotential model needs rho_l > rho_g > 0 and a finite sc_G");
    c->d.nx = cfg->n[0];
    c->d.px = cfg->n[0];
    c->d.ny = cfg->n[1];
    c->d.nz = c->dim == 3 ? cfg->n[2] : 1;
    c->d.N = N;
    c->d.off = 0;
    tile_dims(c->d, c->dim);
    if (cfg->step_kernel != LBM_STEP_AUTO && cfg->step_kernel != LBM_STEP_SPLIT) return bad("step_kernel");
    {
        // the one-pass step: D3Q19 (either wall scheme), whole rows of
        // 64..1024 nodes per workgroup, 4 rows, zc planes: 32, halved until it
        // divides nz, and by default halved down to 8 while the grid would hold
        // fewer than 512 workgroups (two per compute unit of a 256-CU device);
        // LBM_FUSED_ZC sets the starting value.  Interleaved on one device at
        // 256^3 (with the stencil ring), the walk over 8, 16, 32 planes took
        // 0.574, 0.584, 0.570 ms and the ghost sums 0.025, 0.022, 0.020 ms;
        // without the ring 64 planes (one workgroup per CU) took 0.729 ms, and
        // at 512^3 16 and 32 planes 4.61 and 4.59 ms
        const char* e = std::getenv("LBM_FUSED_ZC");
        int zc = e ? std::atoi(e) : 32;
        while (zc > 2 && c->d.nz % zc) zc >>= 1;
        if (!e)
            while (zc > 8 && (long long)(c->d.ny / kFusedTY) * (c->d.nz / zc) < 512) zc >>= 1;
        c->fzc = zc;
        // (its node indices and the byte offsets of its population accesses, up to
        // five arrays from one base, are 32-bit)
        const size_t elem = cfg->precision == LBM_F64 ? 8 : 4;
        c->fused = cfg->step_kernel == LBM_STEP_AUTO && !c->pf && c->dim == 3 &&
                   c->d.nx % 64 == 0 && c->d.nx <= 1024 && c->d.ny % kFusedTY == 0 && zc >= 2 && c->d.nz % zc == 0 &&
                   5ull * (unsigned long long)N * elem < (1ull << 32);
    }
    c->pr.a = cfg->pr_a;
    c->pr.b = cfg->pr_b;
    c->pr.R = cfg->pr_R;
    c->pr.omega = cfg->pr_omega;
    c->pr.Tr = cfg->Tr;
    std::string err;
    if (!pr_solve(c->pr, err)) return bad(err);
    if (cfg->rho_l > 0) c->pr.rho_l = cfg->rho_l;
    if (cfg->rho_g > 0) c->pr.rho_g = cfg->rho_g;
    c->rho_m = 0.5 * (c->pr.rho_l + c->pr.rho_g);
    c->wall_mu = std::isnan(cfg->wall_mu) ? cfg->k * cfg->k * c->pr.mu_sat : cfg->wall_mu;
    c->mu_ref = cfg->k * cfg->k * c->pr.mu_sat;
    if (cfg->model == LBM_MODEL_PSEUDOPOTENTIAL) {
        // wall values are densities; psi is stored unshifted
        c->wall_mu = std::isnan(cfg->wall_mu) ? c->rho_m : cfg->wall_mu;
        c->mu_ref = 0.0;
    }
    if (c->pf) {
        // bulk values of the order parameter; the wall values are order parameters
        c->pr.rho_l = 1.0;
        c->pr.rho_g = -1.0;
        c->rho_m = 0.0;
        c->wall_mu = std::isnan(cfg->wall_mu) ? 0.0 : cfg->wall_mu;
        c->mu_ref = 0.0;
    }

    lbm_status s = LBM_OK;
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LBM_E_DEVICE;
        }
        c->own_stream = true;
    }
    const size_t fbytes = (size_t)c->Q * N * c->elem;
    if ((s = dalloc(c, (char**)&c->f[0], fbytes)) || (s = dalloc(c, (char**)&c->f[1], fbytes)) ||
        (s = dalloc(c, (char**)&c->rhob[0], N * c->elem)) || (s = dalloc(c, (char**)&c->mu, N * c->elem)) ||
        (c->fused && ((s = dalloc(c, (char**)&c->rhob[1], N * c->elem)) || (s = dalloc(c, (char**)&c->gy, N * c->elem)) ||
                      (s = dalloc(c, (char**)&c->gz, N * c->elem)) || (s = dalloc(c, (char**)&c->gyz, N * c->elem)) ||
                      (s = dalloc(c, (char**)&c->force, 3 * N * c->elem)) ||
                      (s = dalloc(c, (char**)&c->sink, 19 * 1024 * c->elem)))) ||
        (s = dalloc(c, &c->cls, (size_t)N)) || (s = dalloc(c, &c->nbmask, (size_t)N * 4)) ||
        (s = dalloc(c, &c->bidx, (size_t)N * 4)) ||
        (s = dalloc(c, &c->ctl, sizeof(DevCtl))) || (s = dalloc(c, &c->last, sizeof(AngleRec))) ||
        (s = dalloc(c, &c->mass_part, kMassBlocks * sizeof(double))) || (s = dalloc(c, &c->mass_out, sizeof(double))) ||
        (s = dalloc(c, &c->young_counts, 2 * LBM_MAX_SECTORS * sizeof(unsigned))) ||
        (c->pf && ((s = dalloc(c, (char**)&c->g[0], fbytes)) || (s = dalloc(c, (char**)&c->g[1], fbytes)) ||
                   (s = dalloc(c, (char**)&c->phi, N * c->elem))))) {
        lbm_destroy(c);
        return s;
    }
    c->rho = c->rhob[0];
    DevCtl h{};
    for (auto& k : h.m.keys) k[0] = k[1] = ~0ull;
    if (hipMemcpy(c->ctl, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
        lbm_destroy(c);
        return LBM_E_DEVICE;
    }
    // a lattice with no solid
    if (lbm_set_solid(c, nullptr, 0, nullptr) != LBM_OK) {
        lbm_destroy(c);
        return LBM_E_DEVICE;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    void* ps[] = {c->f[0], c->f[1], c->rhob[0], c->rhob[1], c->gy, c->gz, c->gyz, c->force, c->sink, c->mu, c->cls, c->nbmask, c->bidx, c->l1_node, c->l2_node, c->b_node,
                  c->l1_mask, c->l2_mask, c->b_mask, c->l1_inv, c->l2_inv, c->b_q, c->ctl, c->last, c->series,
                  c->mass_part, c->mass_out, c->young_counts, c->ylast, c->yseries, c->ystep_counts,
                  c->g[0], c->g[1], c->phi, c->curved};
    for (void* p : ps) dfree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LBM_OK;
}

lbm_status lbm_set_solid(lbm_ctx* c, const lbm_solid* prims, int n, const double* mu_w_map) {
    if (!c) return LBM_E_ARG;
    if (n < 0 || n > LBM_MAX_SOLIDS || (n > 0 && !prims)) return fail(c, LBM_E_ARG, "set_solid: bad primitive count");
    std::vector<Solid> ss;
    for (int i = 0; i < n; ++i) {
        const lbm_solid& p = prims[i];
        if ((p.kind != LBM_SOLID_SPHERE && p.kind != LBM_SOLID_CAVITY) || !(p.radius > 0))
            return fail(c, LBM_E_ARG, "set_solid: bad primitive");
        if (p.wet_mode != LBM_WET_UNIFORM && p.wet_mode != LBM_WET_STRIPES)
            return fail(c, LBM_E_ARG, "set_solid: bad wet_mode");
        if (p.wet_mode == LBM_WET_STRIPES && !(p.stripe_width > 0))
            return fail(c, LBM_E_ARG, "set_solid: stripe_width must be positive");
        Solid s{};
        for (int k = 0; k < 3; ++k) s.c[k] = k < c->dim ? p.center[k] : 0.0;
        s.r = p.radius;
        s.concave = p.kind == LBM_SOLID_CAVITY;
        s.wet_mode = p.wet_mode;
        s.mu1 = p.mu_w;
        s.mu2 = p.mu_w2;
        s.width = p.stripe_width;
        double pl[3] = {p.pole[0], p.pole[1], c->dim == 3 ? p.pole[2] : 0.0};
        double pn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        if (pn == 0) {
            pl[0] = 0; pl[1] = c->dim == 2 ? 1 : 0; pl[2] = c->dim == 2 ? 0 : 1;
            pn = 1;
        }
        for (int k = 0; k < 3; ++k) s.pole[k] = pl[k] / pn;
        ss.push_back(s);
    }
    Geometry g;
    std::string err;
    const int wall[3] = {c->cfg.axis_bc[0] == LBM_WALL, c->cfg.axis_bc[1] == LBM_WALL,
                         c->dim == 3 && c->cfg.axis_bc[2] == LBM_WALL};
    if (!build_geometry(g, c->dim, c->cfg.n, wall, ss, mu_w_map, c->wall_mu, err)) return fail(c, LBM_E_ARG, err);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->solids = ss;
    lbm_status s;
    HIPCHK(c, hipMemcpy(c->cls, g.cls.data(), g.N, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->nbmask, g.nbmask.data(), g.N * 4, hipMemcpyHostToDevice));
    {
        std::vector<int> bi((size_t)g.N, -1);
        for (size_t k = 0; k < g.b_node.size(); ++k) bi[g.b_node[k]] = (int)k;
        HIPCHK(c, hipMemcpy(c->bidx, bi.data(), g.N * 4, hipMemcpyHostToDevice));
    }
    if ((s = upload(c, &c->l1_node, g.l1_node)) || (s = upload(c, &c->l2_node, g.l2_node)) ||
        (s = upload(c, &c->b_node, g.b_node)) || (s = upload(c, &c->l1_mask, g.l1_mask)) ||
        (s = upload(c, &c->l2_mask, g.l2_mask)) || (s = upload(c, &c->b_mask, g.b_mask)) ||
        (s = upload_real(c, &c->l1_inv, g.l1_inv)) || (s = upload_real(c, &c->l2_inv, g.l2_inv)) ||
        (s = upload_real(c, &c->b_q, g.b_q)))
        return s;
    c->n_l1 = (int)g.l1_node.size();
    c->n_l2 = (int)g.l2_node.size();
    c->n_b = (int)g.b_node.size();
    {
        std::vector<int> cv;
        if (c->fused && c->cfg.bc_mode == LBM_BC_BOUZIDI_MC)
            for (size_t k = 0; k < g.b_node.size(); ++k)
                if (g.cls[g.b_node[k]] & CLS_CURVED_) cv.push_back((int)k);
        if ((s = upload(c, &c->curved, cv))) return s;
        c->n_curved = (int)cv.size();
    }
    c->n_fluid = g.n_fluid;
    // static wall chemical potential on the two solid layers; zero elsewhere
    {
        std::vector<double> muh((size_t)g.N, 0.0);
        // the layers' wall value: mu_w (stored shifted), or for the
        // pseudopotential model psi of the wall density
        // (phase-field model: the wall order parameter, into phi; mu stays zero there)
        const bool sc = c->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL;
        auto wall = [&](double v) { return sc ? 1.0 - std::exp(-v) : v - c->mu_ref; };
        for (size_t i = 0; i < g.l1_node.size(); ++i) muh[g.l1_node[i]] = wall(g.l1_mu[i]);
        for (size_t i = 0; i < g.l2_node.size(); ++i) muh[g.l2_node[i]] = wall(g.l2_mu[i]);
        std::vector<char> zero((size_t)g.N * c->elem, 0);
        void* dst = c->pf ? c->phi : c->mu;
        if (c->f64) {
            HIPCHK(c, hipMemcpy(dst, muh.data(), g.N * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> t(muh.begin(), muh.end());
            HIPCHK(c, hipMemcpy(dst, t.data(), g.N * 4, hipMemcpyHostToDevice));
        }
        if (c->pf) HIPCHK(c, hipMemcpy(c->mu, zero.data(), zero.size(), hipMemcpyHostToDevice));
        for (void* rb : c->rhob)
            if (rb) HIPCHK(c, hipMemcpy(rb, zero.data(), zero.size(), hipMemcpyHostToDevice));
        c->rcur = 0;
        c->rho = c->rhob[0];
        c->rho_valid = false;
    }
    c->have_geometry = true;
    c->have_state = false;
    c->series_written = 0;
    if (!c->solids.empty() && c->mopts.solid_index >= (int)c->solids.size()) c->mopts.solid_index = 0;
    return LBM_OK;
}

lbm_status lbm_init_drops(lbm_ctx* c, const lbm_drop* drops, int n, double W) {
    if (!c) return LBM_E_ARG;
    if (n < 1 || !drops || !(W > 0)) return fail(c, LBM_E_ARG, "init_drops: need n >= 1 drops and W > 0");
    const Dims& d = c->d;
    std::vector<uint8_t> cls(d.N);
    HIPCHK(c, hipMemcpy(cls.data(), c->cls, d.N, hipMemcpyDeviceToHost));
    std::vector<double> rho(d.N, 0.0);
    const double rg = c->pr.rho_g, rl = c->pr.rho_l;
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < d.N; ++i) {
        if ((cls[i] & 3) != 0) continue;
        const int x = (int)(i % d.nx), y = (int)((i / d.nx) % d.ny), z = (int)(i / ((long long)d.nx * d.ny));
        double best = -1e300;
        for (int k = 0; k < n; ++k) {
            const double dx = x - drops[k].center[0], dy = y - drops[k].center[1];
            const double dz = c->dim == 3 ? z - drops[k].center[2] : 0.0;
            const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            // Eq. 16
            const double v = 0.5 * (rg + rl) + 0.5 * (rg - rl) * std::tanh(2.0 * (r - drops[k].radius) / W);
            if (v > best) best = v;
        }
        rho[i] = best;
    }
    lbm_status s;
    // (phase-field model: the profile is the order parameter's, rho_l = 1, rho_g = -1)
    const int field = c->pf ? LBM_FIELD_PHI : LBM_FIELD_RHO;
    if (c->f64) {
        s = lbm_write(c, field, rho.data(), rho.size() * 8, 0);
    } else {
        std::vector<float> fr(rho.begin(), rho.end());
        s = lbm_write(c, field, fr.data(), fr.size() * 4, 0);
    }
    if (s != LBM_OK) return s;
    c->t = 0;
    k_ctl_set<<<1, 64, 0, c->stream>>>(c->ctl, 0, 0, 0, 0, 1);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// lbm_write of the phase-field model: PHI (state at rest around it), or one
// population set of a checkpoint (F or G)
static lbm_status pf_write(lbm_ctx* c, int field, const void* src, size_t bytes, hipMemcpyKind kind) {
    const size_t N = (size_t)c->d.N, fb = (size_t)c->Q * N * c->elem;
    auto zero = [&](void* p, size_t nbytes) {
        if (c->f64) k_fill_value<double><<<2048, 256, 0, c->stream>>>((double*)p, nbytes / 8, 0.0);
        else k_fill_value<float><<<2048, 256, 0, c->stream>>>((float*)p, nbytes / 4, 0.0f);
    };
    if (field == LBM_FIELD_PHI) {
        if (bytes != N * c->elem) return fail(c, LBM_E_ARG, "write PHI: bytes must be N * elem");
        // the source is staged in g[1 - cur] (free between steps), stream-ordered,
        // and both spare buffers are cleared afterwards
        HIPCHK(c, hipMemcpyAsync(c->g[1 - c->cur], src, bytes, kind, c->stream));
        dispatch<OpPfInit>(c, (const void*)c->g[1 - c->cur]);
        zero(c->f[1 - c->cur], fb);
        zero(c->g[1 - c->cur], fb);
    } else if (field == LBM_FIELD_F || field == LBM_FIELD_G) {
        if (bytes != fb) return fail(c, LBM_E_ARG, "write F/G: bytes must be Q * N * elem");
        if (!c->have_state) {
            // a fresh state: the set not written starts at zero
            zero(c->f[c->cur], fb);
            zero(c->g[c->cur], fb);
        } else if (c->fstar) {
            // both sets to S_t first, so that the two stay in one form
            void* S = nullptr;
            dispatch<OpMaterialize>(c, &S);
            dispatch<OpMaterializeG>(c, &S);
            c->cur ^= 1;
        }
        HIPCHK(c, hipMemcpyAsync(field == LBM_FIELD_F ? c->f[c->cur] : c->g[c->cur], src, bytes, kind, c->stream));
    } else {
        return fail(c, LBM_E_ARG, "write: the phase-field model takes PHI, F or G");
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->rho_valid = false;
    c->fstar = false;
    c->have_state = true;
    c->series_written = 0;
    return LBM_OK;
}

lbm_status lbm_write(lbm_ctx* c, int field, const void* src, size_t bytes, int src_on_device) {
    if (!c) return LBM_E_ARG;
    if (!src) return fail(c, LBM_E_ARG, "write: null source");
    if (!c->have_geometry) return fail(c, LBM_E_STATE, "write: no geometry");
    const size_t N = (size_t)c->d.N;
    const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (c->pf) return pf_write(c, field, src, bytes, kind);
    if (field == LBM_FIELD_RHO) {
        if (bytes != N * c->elem) return fail(c, LBM_E_ARG, "write RHO: bytes must be N * elem");
        // stream-ordered: a device-to-device copy may otherwise still be in
        // flight when the kernels below (or the caller's next writes to src) run
        c->rho_valid = false;
        HIPCHK(c, hipMemcpyAsync(c->rho, src, bytes, kind, c->stream));
        // zero both population buffers, then f = f_eq(rho, 0)
        const size_t fb = (size_t)c->Q * N * c->elem;
        if (c->f64) {
            k_fill_value<double><<<2048, 256, 0, c->stream>>>((double*)c->f[0], fb / 8, 0.0);
            k_fill_value<double><<<2048, 256, 0, c->stream>>>((double*)c->f[1], fb / 8, 0.0);
        } else {
            k_fill_value<float><<<2048, 256, 0, c->stream>>>((float*)c->f[0], fb / 4, 0.0f);
            k_fill_value<float><<<2048, 256, 0, c->stream>>>((float*)c->f[1], fb / 4, 0.0f);
        }
        dispatch<OpInit>(c);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->fstar = false;
        c->have_state = true;
        c->series_written = 0;
        return LBM_OK;
    }
    if (field == LBM_FIELD_F) {
        const size_t fb = (size_t)c->Q * N * c->elem;
        if (bytes != fb) return fail(c, LBM_E_ARG, "write F: bytes must be Q * N * elem");
        c->rho_valid = false;
        HIPCHK(c, hipMemcpyAsync(c->f[c->cur], src, bytes, kind, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->fstar = false;
        c->have_state = true;
        c->series_written = 0;
        return LBM_OK;
    }
    return fail(c, LBM_E_ARG, "write: field must be RHO or F");
}

lbm_status lbm_set_measure(lbm_ctx* c, const lbm_measure_opts* o) {
    if (!c || !o) return LBM_E_ARG;
    lbm_status s = check_measure_opts(c, *o);
    if (s) return s;
    c->mopts = *o;
    drop_graphs(c);
    return LBM_OK;
}

static lbm_status ensure_series(lbm_ctx* c, int cap) {
    if (cap <= c->series_capacity) return LBM_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    lbm_status s = dalloc(c, &c->series, (size_t)cap * sizeof(AngleRec));
    if (!s) s = dalloc(c, &c->yseries, (size_t)cap * sizeof(YoungRec));
    if (s) {
        c->series_capacity = 0;
        return s;
    }
    c->series_capacity = cap;
    return LBM_OK;
}

lbm_status lbm_set_young(lbm_ctx* c, const lbm_young_opts* yo) {
    if (!c) return LBM_E_ARG;
    if (yo && !young_opts_ok(*yo))
        return fail(c, LBM_E_ARG, "set_young: gamma finite, roughness > 0, 0 < band_lo < band_hi < 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    // off until both buffers are allocated and cleared: the step launches the
    // in-step kernels only when it is on
    c->young_on = false;
    c->series_written = 0;  // records of earlier options are not returned
    if (!yo) return LBM_OK;
    c->yopts = *yo;
    lbm_status s = LBM_OK;
    if (!c->ylast) s = dalloc(c, &c->ylast, sizeof(YoungRec));
    if (!s && !c->ystep_counts) s = dalloc(c, &c->ystep_counts, 2 * LBM_MAX_SECTORS * sizeof(unsigned));
    if (s) return s;
    // the counts start at zero; every in-step measurement clears them after use
    HIPCHK(c, hipMemset(c->ystep_counts, 0, 2 * LBM_MAX_SECTORS * sizeof(unsigned)));
    c->young_on = true;
    return LBM_OK;
}

lbm_status lbm_young_series(lbm_ctx* c, lbm_young* out, int cap, int* n_written) {
    if (!c || !out || cap < 0 || !n_written) return LBM_E_ARG;
    *n_written = 0;
    if (!c->young_on) return fail(c, LBM_E_STATE, "young_series: the in-step Young force is off (lbm_set_young)");
    const int n = c->series_written < cap ? c->series_written : cap;
    if (n > 0) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(out, c->yseries, (size_t)n * sizeof(YoungRec), hipMemcpyDeviceToHost));
    }
    *n_written = n;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps, int measure_every, lbm_angle* series, int cap, int* n_written) {
    if (!c) return LBM_E_ARG;
    if (n_written) *n_written = 0;
    if (!c->have_state) return fail(c, LBM_E_STATE, "step: no initial state (call lbm_init_drops or lbm_write)");
    if (nsteps < 0 || measure_every < 0 || cap < 0) return fail(c, LBM_E_ARG, "step: negative argument");
    if (measure_every > 0 && c->solids.empty()) return fail(c, LBM_E_ARG, "step: measurement needs a solid");
    if (c->young_on && c->solids.empty()) return fail(c, LBM_E_STATE, "step: the Young force needs a solid");
    c->series_written = 0;
    if (series && cap > 0) {
        lbm_status s = ensure_series(c, cap);
        if (s) return s;
    } else if (c->series_capacity == 0) {
        lbm_status s = ensure_series(c, 1);
        if (s) return s;
    }
    MeasureParams mp{};
    if (!c->solids.empty()) {
        lbm_status s = check_measure_opts(c, c->mopts);
        if (s) return s;
        mp = measure_params(c, c->mopts);
    } else {
        mp.rho_m = c->rho_m;
        mp.n_sectors = 2;
        mp.dim = c->dim;
    }
    lbm_status s = ctl_reset(c, measure_every, 0, series ? cap : 0);
    if (s) return s;
    int64_t done = 0;
    const bool fused = c->fused;
    if (fused) {
        // the one-pass step needs rho_t (with the solid layers) and mu_t, and on
        // a measure step the liquid centroid sums of rho_t
        if (!c->rho_valid) dispatch<OpDerive>(c, true);
        else if (measure_every > 0 && c->t % measure_every == 0) dispatch<OpCentroid>(c, mp.rho_m);
    }
    auto launch_one = [&](int src, bool pull, int rsrc, bool quiet) {
        if (fused) dispatch<OpFusedStep>(c, src, pull, rsrc, &mp, (hipEvent_t*)nullptr, (int*)nullptr, quiet);
        else dispatch<OpStep>(c, src, pull, &mp, (hipEvent_t*)nullptr, (int*)nullptr);
    };
    auto advance = [&]() {
        c->cur ^= 1;
        c->fstar = true;
        if (fused) {
            c->rcur ^= 1;
            c->rho = c->rhob[c->rcur];
        }
    };
    auto eager = [&]() {
        launch_one(c->cur, c->fstar, c->rcur, false);
        advance();
        ++done;
        ++c->t;
    };
    // eager steps until the populations are in pull form in buffer 0 (and the
    // density in buffer 0), then whole captured graphs (an even number of
    // steps keeps the parity), then the rest.  The one-pass step has two
    // graphs: graph[0] of full steps, and graph[1] of quiet steps for windows
    // of kGraphSteps steps of which none is a measure step (t % every != 0).
    auto quiet_window = [&](int64_t t0) {
        if (!fused) return false;
        if (measure_every <= 0) return true;
        const int64_t r = t0 % measure_every;
        return r != 0 && measure_every - r >= kGraphSteps;
    };
    while (done < nsteps && (!c->fstar || c->cur != 0 || c->rcur != 0 || nsteps - done < kGraphSteps)) eager();
    while (nsteps - done >= kGraphSteps) {
        const int gi = quiet_window(c->t) ? 1 : 0;
        if (!c->graph[gi]) {
            hipGraph_t g;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < kGraphSteps; ++k) launch_one(k & 1, true, k & 1, gi == 1);
            HIPCHK(c, hipStreamEndCapture(c->stream, &g));
            hipError_t e = hipGraphInstantiate(&c->graph[gi], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->graph[gi] = nullptr;
                return fail(c, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        HIPCHK(c, hipGraphLaunch(c->graph[gi], c->stream));
        done += kGraphSteps;
        c->t += kGraphSteps;
    }
    while (done < nsteps) eager();
    HIPCHK(c, hipGetLastError());
    if (series && cap > 0) {
        DevCtl h;
        HIPCHK(c, hipMemcpyAsync(&h, c->ctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int nw = h.series_count < cap ? h.series_count : cap;
        if (nw > 0) HIPCHK(c, hipMemcpy(series, c->series, (size_t)nw * sizeof(AngleRec), hipMemcpyDeviceToHost));
        if (n_written) *n_written = nw;
        c->series_written = nw;
        if (h.status & 1) return fail(c, LBM_E_NONFINITE, "a density became non-finite, non-positive or >= 1/b");
    }
    return LBM_OK;
}

lbm_status lbm_measure_angle(lbm_ctx* c, const lbm_measure_opts* o, lbm_angle* out) {
    if (!c || !o || !out) return LBM_E_ARG;
    if (!c->have_state) return fail(c, LBM_E_STATE, "measure: no state");
    lbm_status s = check_measure_opts(c, *o);
    if (s) return s;
    const MeasureParams mp = measure_params(c, *o);
    if ((s = ctl_reset(c, 0, 1, 0))) return s;
    dispatch<OpMeasure>(c, &mp);
    if ((s = ctl_reset(c, 0, 0, 0))) return s;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out, c->last, sizeof(AngleRec), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out->step = c->t;
    if (out->status != 0) return fail(c, LBM_E_NO_CONTACT_LINE, "no sector holds both selected crossings");
    return LBM_OK;
}

lbm_status lbm_young_force(lbm_ctx* c, const lbm_young_opts* yo, lbm_angle* angle, lbm_young* out) {
    if (!c || !yo || !angle || !out) return LBM_E_ARG;
    if (!young_opts_ok(*yo)) return fail(c, LBM_E_ARG, "young: gamma finite, roughness > 0, 0 < band_lo < band_hi < 1");
    double lo, hi;
    young_band(*yo, lo, hi);
    std::memset(angle, 0, sizeof *angle);
    const lbm_status ms = lbm_measure_angle(c, &c->mopts, angle);
    young_clear(*angle, ms, out);
    if (ms != LBM_OK) return ms;
    // footprint counts on the density the measurement derived
    YoungParams yp = young_params(c->solids[c->mopts.solid_index], *angle, c->dim, c->pr.rho_g, c->pr.rho_l, lo, hi);
    HIPCHK(c, hipMemsetAsync(c->young_counts, 0, 2 * LBM_MAX_SECTORS * sizeof(unsigned), c->stream));
    dispatch<OpYoung>(c, &yp);
    HIPCHK(c, hipGetLastError());
    unsigned h[2 * LBM_MAX_SECTORS];
    HIPCHK(c, hipMemcpyAsync(h, c->young_counts, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    young_from_counts(*yo, *angle, h, out);
    return LBM_OK;
}

lbm_status lbm_read(lbm_ctx* c, int field, void* dst, size_t bytes, int dst_on_device) {
    if (!c || !dst) return c ? fail(c, LBM_E_ARG, "read: null destination") : LBM_E_ARG;
    if (!c->have_state && field != LBM_FIELD_CLASS) return fail(c, LBM_E_STATE, "read: no state");
    const size_t N = (size_t)c->d.N;
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    lbm_status s;
    switch (field) {
        case LBM_FIELD_RHO:
        case LBM_FIELD_MU:
            if (bytes != N * c->elem) return fail(c, LBM_E_ARG, "read: bytes must be N * elem");
            if ((s = ctl_reset(c, 0, 0, 0))) return s;
            dispatch<OpDerive>(c, field == LBM_FIELD_MU);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipMemcpyAsync(dst, field == LBM_FIELD_RHO ? c->rho : c->mu, bytes, kind, c->stream));
            if (field == LBM_FIELD_MU) {
                // undo the stored shift on fluid and solid-layer nodes (deeper solid reads mu_ref)
                if (dst_on_device) {
                    if (c->f64) k_add_value<double><<<1024, 256, 0, c->stream>>>((double*)dst, N, c->mu_ref);
                    else k_add_value<float><<<1024, 256, 0, c->stream>>>((float*)dst, N, (float)c->mu_ref);
                    HIPCHK(c, hipGetLastError());
                } else {
                    HIPCHK(c, hipStreamSynchronize(c->stream));
                    if (c->f64) for (size_t i = 0; i < N; ++i) ((double*)dst)[i] += c->mu_ref;
                    else for (size_t i = 0; i < N; ++i) ((float*)dst)[i] = (float)((double)((float*)dst)[i] + c->mu_ref);
                }
            }
            break;
        case LBM_FIELD_F:
            if (bytes != (size_t)c->Q * N * c->elem) return fail(c, LBM_E_ARG, "read F: bytes must be Q * N * elem");
            {
                void* S = nullptr;
                dispatch<OpMaterialize>(c, &S);
                HIPCHK(c, hipGetLastError());
                HIPCHK(c, hipMemcpyAsync(dst, S, bytes, kind, c->stream));
            }
            break;
        case LBM_FIELD_VEL: {
            if (bytes != 3 * N * c->elem) return fail(c, LBM_E_ARG, "read VEL: bytes must be 3 * N * elem");
            if ((s = ctl_reset(c, 0, 0, 0))) return s;
            void* tmp = nullptr;
            if (dst_on_device) tmp = dst;
            else if ((s = dalloc(c, (char**)&tmp, bytes))) return s;
            dispatch<OpVel>(c, tmp);
            HIPCHK(c, hipGetLastError());
            if (!dst_on_device) {
                HIPCHK(c, hipMemcpyAsync(dst, tmp, bytes, hipMemcpyDeviceToHost, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                dfree(tmp);
            }
            break;
        }
        case LBM_FIELD_CLASS: {
            if (bytes != N) return fail(c, LBM_E_ARG, "read CLASS: bytes must be N");
            std::vector<uint8_t> h(N);
            HIPCHK(c, hipStreamSynchronize(c->stream));
            HIPCHK(c, hipMemcpy(h.data(), c->cls, N, hipMemcpyDeviceToHost));
            for (auto& v : h) v &= 3;
            if (dst_on_device) HIPCHK(c, hipMemcpyAsync(dst, h.data(), N, hipMemcpyHostToDevice, c->stream));
            else std::memcpy(dst, h.data(), N);
            break;
        }
        case LBM_FIELD_PHI:
            if (!c->pf) return fail(c, LBM_E_ARG, "read PHI: a field of the phase-field model");
            if (bytes != N * c->elem) return fail(c, LBM_E_ARG, "read PHI: bytes must be N * elem");
            if ((s = ctl_reset(c, 0, 0, 0))) return s;
            dispatch<OpDerive>(c, false);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipMemcpyAsync(dst, c->phi, bytes, kind, c->stream));
            break;
        case LBM_FIELD_G:
            if (!c->pf) return fail(c, LBM_E_ARG, "read G: a field of the phase-field model");
            if (bytes != (size_t)c->Q * N * c->elem) return fail(c, LBM_E_ARG, "read G: bytes must be Q * N * elem");
            {
                void* S = nullptr;
                dispatch<OpMaterializeG>(c, &S);
                HIPCHK(c, hipGetLastError());
                HIPCHK(c, hipMemcpyAsync(dst, S, bytes, kind, c->stream));
            }
            break;
        case LBM_FIELD_MASS:
            if (bytes != 8) return fail(c, LBM_E_ARG, "read MASS: bytes must be 8");
            dispatch<OpMass>(c);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipMemcpyAsync(dst, c->mass_out, 8, kind, c->stream));
            break;
        default:
            return fail(c, LBM_E_ARG, "read: unknown field");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
    if (!c) return LBM_E_ARG;
    return check_status(c);
}

lbm_status lbm_get_info(lbm_ctx* c, lbm_info* info) {
    if (!c || !info) return LBM_E_ARG;
    std::memset(info, 0, sizeof *info);
    info->Tc = c->pr.Tc;
    info->T = c->pr.T;
    info->alpha = c->pr.alpha;
    info->rho_g = c->pr.rho_g;
    info->rho_l = c->pr.rho_l;
    info->mu_sat = c->pr.mu_sat;
    info->p_sat = c->pr.p_sat;
    info->wall_mu = c->wall_mu;
    info->rho_m = c->rho_m;
    info->Q = c->Q;
    info->precision = c->cfg.precision;
    info->N = c->d.N;
    info->step = c->t;
    info->n_fluid = c->n_fluid;
    info->n_layer1 = c->n_l1;
    info->n_layer2 = c->n_l2;
    info->n_boundary = c->n_b;
    return LBM_OK;
}

lbm_status lbm_profile_step(lbm_ctx* c, int64_t nsteps, const char** names, double* ms, int cap, int* n_kinds) {
    static const char* kNames[11] = {"k_density", "k_fill_layer1", "k_fill_layer2", "k_mu",    "k_collide",
                                     "k_cross",   "k_finalize",    "k_step",        "k_ghost", "k_force",
                                     "k_interp_wall"};
    if (!c || !names || !ms || !n_kinds) return LBM_E_ARG;
    if (!c->have_state) return fail(c, LBM_E_STATE, "profile: no state");
    if (nsteps < 1) return fail(c, LBM_E_ARG, "profile: nsteps >= 1");
    MeasureParams mp{};
    if (!c->solids.empty()) mp = measure_params(c, c->mopts);
    else { mp.rho_m = c->rho_m; mp.n_sectors = 2; mp.dim = c->dim; }
    lbm_status s = ctl_reset(c, 0, 0, 0);
    if (s) return s;
    if (c->fused && !c->rho_valid) dispatch<OpDerive>(c, true);
    hipEvent_t ev[24];
    for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
    double tot[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int cnt[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t t = 0; t < nsteps; ++t) {
        int kinds[12];
        if (c->fused) {
            dispatch<OpFusedStep>(c, c->cur, c->fstar, c->rcur, &mp, ev, kinds);
            c->rcur ^= 1;
            c->rho = c->rhob[c->rcur];
        } else {
            dispatch<OpStep>(c, c->cur, c->fstar, &mp, ev, kinds);
        }
        c->cur ^= 1;
        c->fstar = true;
        ++c->t;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int k = 0; k < 11 && kinds[k] >= 0; ++k) {
            float e = 0;
            HIPCHK(c, hipEventElapsedTime(&e, ev[2 * k], ev[2 * k + 1]));
            tot[kinds[k]] += e;
            cnt[kinds[k]] += 1;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    int n = 0;
    for (int k = 0; k < 11 && n < cap; ++k) {
        if (!cnt[k]) continue;
        names[n] = kNames[k];
        ms[n] = tot[k] / cnt[k];
        ++n;
    }
    *n_kinds = n;
    return check_status(c);
}

lbm_status lbm_measure_field(int lattice, int precision, const int n[3], const void* rho, const uint8_t* cls,
                             const lbm_solid* solid, int n_sectors, double rho_m, const double g[3], lbm_angle* out,
                             void* stream) {
    auto bad = [](const char* m) {
        g_free_err = std::string("measure_field: ") + m;
        return LBM_E_ARG;
    };
    g_free_err.clear();
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return bad("lattice must be LBM_D2Q9 or LBM_D3Q19");
    if (precision != LBM_F32 && precision != LBM_F64 && precision != LBM_F32_MIXED) return bad("precision");
    if (!n || !rho || !cls || !solid || !out) return bad("null pointer");
    const int dim = lattice == LBM_D2Q9 ? 2 : 3, Q = dim == 2 ? 9 : 19;
    if (dim == 2 && n[2] != 1) return bad("n[2] must be 1 for D2Q9");
    for (int k = 0; k < dim; ++k)
        if (n[k] < 5 || n[k] > (1 << 20)) return bad("n out of range (5 .. 2^20 per axis)");
    const long long N = (long long)n[0] * n[1] * (dim == 3 ? n[2] : 1);
    if ((unsigned long long)N * (unsigned long long)Q >= (1ull << 32))
        return bad("N * Q must stay below 2^32 (32-bit link ids of the selection keys)");
    if (dim == 3 && (n_sectors < 1 || n_sectors > LBM_MAX_SECTORS))
        return bad("n_sectors must lie in 1..64 (the static slots hold 64 sectors)");
    if (!(rho_m > 0) || !std::isfinite(rho_m)) return bad("rho_m must be positive and finite");
    if ((solid->kind != LBM_SOLID_SPHERE && solid->kind != LBM_SOLID_CAVITY) || !(solid->radius > 0))
        return bad("bad solid primitive");
    void* sp = nullptr;
    lbm_status s = scratch_ptr(&sp);
    if (s != LBM_OK) return s;
    Dims d{};
    d.nx = n[0];
    d.px = n[0];
    d.ny = n[1];
    d.nz = dim == 3 ? n[2] : 1;
    d.N = N;
    d.off = 0;
    tile_dims(d, dim);
    MeasureParams mp{};
    for (int k = 0; k < 3; ++k) {
        mp.c[k] = k < dim ? solid->center[k] : 0.0;
        mp.g[k] = g && k < dim ? g[k] : 0.0;
    }
    mp.R = solid->radius;
    mp.concave = solid->kind == LBM_SOLID_CAVITY;
    mp.rho_m = rho_m;
    mp.n_sectors = dim == 2 ? 2 : n_sectors;
    mp.dim = dim;
    const hipStream_t st = (hipStream_t)stream;
    DevCtl* ctl = (DevCtl*)sp;
    AngleRec* rec = (AngleRec*)out;
    if (dim == 2) {
        if (precision == LBM_F64) OpMeasureField<D2Q9, double, double>::go(d, rho, cls, ctl, mp, rec, st);
        else OpMeasureField<D2Q9, float, float>::go(d, rho, cls, ctl, mp, rec, st);
    } else {
        if (precision == LBM_F64) OpMeasureField<D3Q19, double, double>::go(d, rho, cls, ctl, mp, rec, st);
        else OpMeasureField<D3Q19, float, float>::go(d, rho, cls, ctl, mp, rec, st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_free_err = std::string("measure_field: launch: ") + hipGetErrorString(e);
        return LBM_E_DEVICE;
    }
    return LBM_OK;
}

}  // extern "C"
