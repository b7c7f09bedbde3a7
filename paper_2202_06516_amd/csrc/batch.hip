// batch.hip -- many independent lattices advanced together.
//
// Every case (its own lattice size, solid, wettability and drop) lives at an
// offset of one packed allocation.  Each phase of the step is one persistent
// launch: a fixed grid of workgroups walks a work list of (case, tile) items
// and runs the same per-node device bodies as the single-lattice kernels, so a
// case advanced in a batch is bitwise identical to the same case advanced
// alone.  The phase-field model runs on the same work list with its own
// density, mu and collision bodies.  Step loops are captured in a hipGraph.  The tile width and the
// number of workgroups per compute unit come from a small autotuner that times
// candidate launches on the batch itself and caches its choice in a JSON file.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"
#include "lbm.h"
#include "phasefield.hpp"
#include "young.hpp"

using namespace lbm;

namespace {

struct Item {
    int c;            // case
    int x0, y0, z0;   // first node of the tile
};

// tile_w is 64, 128 or 256: shifts, not divisions
__device__ __forceinline__ void item_node(const Item& it, int tile_w, int& x, int& y, int& z) {
    x = it.x0 + (int)(threadIdx.x & (unsigned)(tile_w - 1));
    y = it.y0 + (int)(threadIdx.x >> (__ffs(tile_w) - 1));
    z = it.z0;
}

// First work-list slot of this workgroup.  Workgroups are dealt to the 8 XCDs
// round-robin by id; the slots are permuted so that each XCD owns a
// contiguous run of gridDim.x / 8 consecutive items in every sweep (the
// neighbouring tiles of a case, and the stencil rows they share, meet in one
// L2).  A bijection of [0, gridDim.x); item k of sweep j is slot + j gridDim.x.
__device__ __forceinline__ int xcd_slot() {
    const unsigned g = gridDim.x, b = blockIdx.x, q = g >> 3, r = g & 7u, xcd = b & 7u, loc = b >> 3;
    return (int)((xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + loc);
}

template <class L, typename R, typename C, bool PULL>
__global__ void __launch_bounds__(256) kb_density(const Item* __restrict__ items, int nitems, const Dims* __restrict__ dims,
                                                  int tile_w, const R* __restrict__ f, R* __restrict__ rho,
                                                  const uint8_t* __restrict__ cls, WallBC bc, DevCtl* __restrict__ ctl,
                                                  MeasureSlots* __restrict__ slots, const MeasureParams* __restrict__ mp,
                                                  R inv_b) {
    const bool meas = measuring(ctl);
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        const bool liquid = density_node<L, R, C, PULL>(f, rho, cls, d, bc, x, y, z, x < d.nx && y < d.ny,
                                                        mp[it.c].rho_m, inv_b, &ctl->status);
        if (meas) centroid_reduce(liquid, x, y, z, &slots[it.c]);
    }
}

template <class L, typename R, typename C>
__global__ void __launch_bounds__(256) kb_fill(const long long* __restrict__ node, const uint32_t* __restrict__ mask,
                                               const R* __restrict__ inv_den, const int* __restrict__ ecase, int beg,
                                               int end, R* __restrict__ rho, const Dims* __restrict__ dims) {
    for (int k = beg + blockIdx.x * 256 + threadIdx.x; k < end; k += gridDim.x * 256)
        fill_entry<L, R, C>(node[k], mask[k], inv_den[k], rho, dims[ecase[k]]);
}

template <class L, typename R, typename C, bool SC = false>
__global__ void __launch_bounds__(256) kb_mu(const Item* __restrict__ items, int nitems, const Dims* __restrict__ dims,
                                             int tile_w, const R* __restrict__ rho, R* __restrict__ mu,
                                             const uint8_t* __restrict__ cls, Thermo th) {
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        R r0;
        (void)mu_node<L, R, C, SC>(rho, mu, cls, d, th, x, y, z, x < d.nx && y < d.ny, r0);
    }
}

// the crossing search of a measure step, its own launch (returns at once otherwise)
template <class L, typename R>
__global__ void __launch_bounds__(256) kb_cross(const Item* __restrict__ items, int nitems, const Dims* __restrict__ dims,
                                                int tile_w, const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                                const DevCtl* __restrict__ ctl, MeasureSlots* __restrict__ slots,
                                                const MeasureParams* __restrict__ mp) {
    if (!measuring(ctl)) return;
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        bool fluid = false;
        R r0 = R(0);
        if (x < d.nx && y < d.ny) {
            const long long idx = nid(d, x, y, z);
            fluid = (cls[idx] & CLS_MASK) == CLS_FLUID;
            if (fluid) r0 = rho[idx];
        }
        crossings_node<L, R>(rho, cls, d, x, y, z, fluid, r0, mp[it.c], &slots[it.c]);
    }
}

template <class L, typename R, typename C, bool PULL, bool MRT, bool SC = false>
__global__ void __launch_bounds__(256) kb_collide(const Item* __restrict__ items, int nitems,
                                                  const Dims* __restrict__ dims, int tile_w, const R* __restrict__ fin,
                                                  R* __restrict__ fout, const R* __restrict__ rho,
                                                  const R* __restrict__ mu, const uint8_t* __restrict__ cls, WallBC bc,
                                                  Collision<C> cp, const DevCtl* __restrict__ ctl) {
    const long long t = ctl->t;
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        collide_node<L, R, C, PULL, MRT, true, SC>(fin, fout, rho, mu, cls, d, bc, cp, t, x, y, z);
    }
}

// footprint counts of the unbalanced Young force, every case at once; a case
// whose measurement found no contact line has n_sectors = 0 and is skipped
template <class L, typename R>
__global__ void __launch_bounds__(256) kb_young_count(const Item* __restrict__ items, int nitems,
                                                      const Dims* __restrict__ dims, int tile_w,
                                                      const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                                      const YoungParams* __restrict__ yps,
                                                      unsigned* __restrict__ counts) {
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const YoungParams yp = yps[it.c];
        if (yp.n_sectors == 0) continue;
        const Dims d = dims[it.c];
        const Frame F = frame_from_axis(yp.axis, yp.dim);
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        young_node<L, R>(rho, cls, d, yp, F, x, y, z, counts + (size_t)it.c * 2 * LBM_MAX_SECTORS);
    }
}

// one workgroup of 64 per case
template <class L, typename R>
__global__ void __launch_bounds__(64) kb_finalize(const R* __restrict__ rho, const DevCtl* __restrict__ ctl,
                                                  const Dims* __restrict__ dims, const MeasureParams* __restrict__ mp,
                                                  MeasureSlots* __restrict__ slots, AngleRec* __restrict__ last,
                                                  YoungStep ys = YoungStep{}) {
    if (!measuring(ctl)) return;
    const int c = blockIdx.x;
    finalize_slots<L, R>(rho, dims[c], mp[c], &slots[c], ctl->t, &last[c], nullptr);
    if (ys.on) {
        // this case's counts and record
        __syncthreads();
        YoungStep yc = ys;
        yc.counts = ys.counts + (size_t)c * 2 * LBM_MAX_SECTORS;
        yc.last = ys.last + c;
        young_finish(yc, &last[c], nullptr);
    }
}

// the footprint counts of an in-step measurement of every case (returns at
// once on the other steps), each in its own measurement's frame
template <class L, typename R>
__global__ void __launch_bounds__(256) kb_young_step(const Item* __restrict__ items, int nitems,
                                                     const Dims* __restrict__ dims, int tile_w,
                                                     const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                                     const YoungParams* __restrict__ yps,
                                                     const MeasureParams* __restrict__ mp,
                                                     const MeasureSlots* __restrict__ slots, const DevCtl* __restrict__ ctl,
                                                     unsigned* __restrict__ counts) {
    if (!measuring(ctl)) return;
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Frame F = make_frame(&slots[it.c], mp[it.c]);
        if (!F.ok) continue;
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        young_node<L, R>(rho, cls, d, yps[it.c], F, x, y, z, counts + (size_t)it.c * 2 * LBM_MAX_SECTORS);
    }
}

// --- the phase-field model: phi (and with RHO rho) of every case, mu of phi, and
// the collision of both population sets; the crossing search and the finalize
// read phi at the isolevel mp.rho_m (0)
template <class L, typename R, typename C, bool PULL, bool RHO>
__global__ void __launch_bounds__(256) kb_pf_density(const Item* __restrict__ items, int nitems,
                                                     const Dims* __restrict__ dims, int tile_w, const R* __restrict__ f,
                                                     const R* __restrict__ g, R* __restrict__ rho, R* __restrict__ phi,
                                                     const uint8_t* __restrict__ cls, WallBC bc,
                                                     DevCtl* __restrict__ ctl, MeasureSlots* __restrict__ slots,
                                                     const MeasureParams* __restrict__ mp) {
    const bool meas = measuring(ctl);
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        const bool liquid = pf_density_node<L, R, C, PULL, RHO>(f, g, rho, phi, cls, d, bc, &ctl->status,
                                                                mp[it.c].rho_m, x, y, z);
        if (meas) centroid_reduce(liquid, x, y, z, &slots[it.c]);
    }
}

template <class L, typename R>
__global__ void __launch_bounds__(256) kb_pf_mu(const Item* __restrict__ items, int nitems,
                                                const Dims* __restrict__ dims, int tile_w, const R* __restrict__ phi,
                                                R* __restrict__ mu, const uint8_t* __restrict__ cls, PhaseField pf) {
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        if (x < d.nx && y < d.ny) pf_mu_node<L, R>(phi, mu, cls, d, pf, x, y, z);
    }
}

template <class L, typename R, typename C, bool PULL, bool MRT>
__global__ void __launch_bounds__(256) kb_pf_collide(const Item* __restrict__ items, int nitems,
                                                     const Dims* __restrict__ dims, int tile_w,
                                                     const R* __restrict__ fin, R* __restrict__ fout,
                                                     const R* __restrict__ gin, R* __restrict__ gout,
                                                     const R* __restrict__ phi, const R* __restrict__ mu,
                                                     const uint8_t* __restrict__ cls, WallBC bc, Collision<C> cp,
                                                     PhaseField pf, DevCtl* __restrict__ ctl) {
    const long long t = ctl->t;
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        pf_collide_node<L, R, C, PULL, MRT>(fin, fout, gin, gout, phi, mu, cls, d, bc, cp, pf, &ctl->status, t, x, y,
                                            z);
    }
}

__global__ void kb_tick(DevCtl* ctl) {
    if (threadIdx.x == 0) ctl->t += 1;
}

__global__ void kb_slots_reset(MeasureSlots* slots, int n) {
    const int c = blockIdx.x;
    if (c >= n) return;
    slots[c].keys[threadIdx.x][0] = ~0ull;
    slots[c].keys[threadIdx.x][1] = ~0ull;
    if (threadIdx.x == 0) slots[c].cnt = slots[c].sx = slots[c].sy = slots[c].sz = 0ull;
}

template <class L, typename R, typename C, bool PULL>
__global__ void __launch_bounds__(256) kb_materialize(const Item* __restrict__ items, int nitems,
                                                      const Dims* __restrict__ dims, int tile_w,
                                                      const R* __restrict__ f, R* __restrict__ out,
                                                      const uint8_t* __restrict__ cls, WallBC bc) {
    for (int k = xcd_slot(); k < nitems; k += gridDim.x) {
        const Item it = items[k];
        const Dims d = dims[it.c];
        int x, y, z;
        item_node(it, tile_w, x, y, z);
        if (x >= d.nx || y >= d.ny) continue;
        const long long idx = nid(d, x, y, z);
        const uint8_t c = cls[idx];
        R S[L::Q];
        if ((c & CLS_MASK) == CLS_FLUID) gather<L, R, C, PULL>(f, d, idx, x, y, z, c, bc, S);
        else
            for (int i = 0; i < L::Q; ++i) S[i] = R(0);
        for (int i = 0; i < L::Q; ++i) out[(size_t)i * d.N + idx] = S[i];
    }
}

constexpr int kBatchGraphSteps = 16;

}  // namespace

struct lbm_batch {
    lbm_config cfg{};
    std::string err;
    PRState pr{};
    double rho_m = 0, mu_ref = 0, wall_mu = 0;
    int dim = 2, Q = 9, ncases = 0, cus = 256;
    size_t elem = 4;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    long long Ntot = 0, n_fluid = 0;   // packed nodes (rows padded), fluid nodes
    long long n_nodes = 0;             // lattice nodes of all cases
    std::vector<Dims> dims_h;
    std::vector<MeasureParams> mp_h;
    std::vector<Solid> solids_h;       // the substrate of every case
    YoungParams* yparams = nullptr;    // Young-force counting parameters per case (allocated on first use)
    unsigned* ycounts = nullptr;       // footprint counts [case][sector][surface]
    bool young_on = false;             // the Young force at every in-step measurement
    lbm_young_opts yopts{};
    YoungParams* ystep_params = nullptr;  // its counting parameters per case
    unsigned* ystep_counts = nullptr;     // its counts [case][sector][surface], zero between measurements
    YoungRec* ylast = nullptr;            // its latest record per case
    Dims* dims = nullptr;
    MeasureParams* mp = nullptr;
    MeasureSlots* slots = nullptr;
    AngleRec* last = nullptr;
    DevCtl* ctl = nullptr;
    void* f[2] = {nullptr, nullptr};
    bool pf = false;                   // the phase-field model
    PhaseField pfp{};                  // its parameters
    void* g[2] = {nullptr, nullptr};   // its order-parameter populations
    void* phi = nullptr;               // its order parameter (wall values on the solid layers)
    int cur = 0;
    bool fstar = false, have_state = false;
    void *rho = nullptr, *mu = nullptr, *inv = nullptr, *bq = nullptr;
    uint8_t* cls = nullptr;
    uint32_t *nbmask = nullptr, *fmask = nullptr;
    int *bidx = nullptr, *fcase = nullptr;
    long long* fnode = nullptr;
    int n_l1 = 0, n_l2 = 0;
    Item* items = nullptr;
    int nitems = 0;
    int tile_w = 64, bpc = 4;
    double tune_ms = 0;
    hipGraphExec_t graph = nullptr;
    long long t = 0;
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status s, const std::string& m) {
    if (b) b->err = m;
    return s;
}

#define BCHK(b, call)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
lbm_status balloc(lbm_batch* b, T** p, size_t bytes) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (!bytes) return LBM_OK;
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return bfail(b, LBM_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return LBM_OK;
}

template <typename T>
lbm_status bupload(lbm_batch* b, T** p, const std::vector<T>& v) {
    lbm_status s = balloc(b, p, v.size() * sizeof(T));
    if (s || v.empty()) return s;
    BCHK(b, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return LBM_OK;
}

lbm_status bupload_real(lbm_batch* b, void** p, const std::vector<double>& v) {
    lbm_status s = balloc(b, (char**)p, v.size() * b->elem);
    if (s || v.empty()) return s;
    if (b->elem == 8) {
        BCHK(b, hipMemcpy(*p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> t(v.begin(), v.end());
        BCHK(b, hipMemcpy(*p, t.data(), t.size() * 4, hipMemcpyHostToDevice));
    }
    return LBM_OK;
}

void build_items(lbm_batch* b) {
    std::vector<Item> it;
    const int th = 256 / b->tile_w;
    for (int c = 0; c < b->ncases; ++c) {
        const Dims& d = b->dims_h[c];
        for (int z = 0; z < d.nz; ++z)
            for (int y0 = 0; y0 < d.ny; y0 += th)
                for (int x0 = 0; x0 < d.nx; x0 += b->tile_w) it.push_back(Item{c, x0, y0, z});
    }
    if (b->items) (void)hipFree(b->items);
    b->items = nullptr;
    b->nitems = (int)it.size();
    if (hipMalloc((void**)&b->items, it.size() * sizeof(Item)) == hipSuccess)
        (void)hipMemcpy(b->items, it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice);
}

template <class L, typename R, typename C>
struct BRun {
    static Thermo thermo(const lbm_batch* b) {
        const double k2 = b->cfg.k * b->cfg.k;
        const PRState& p = b->pr;
        Thermo th;
        th.k2RT = k2 * p.R * p.T;
        th.k2A = k2 * p.a * p.alpha / (2.0 * std::sqrt(2.0) * p.b);
        th.k2aal = k2 * p.a * p.alpha;
        th.b = p.b;
        th.s2m1 = std::sqrt(2.0) - 1.0;
        th.s2p1 = std::sqrt(2.0) + 1.0;
        th.mu_ref = b->mu_ref;
        th.kappa = b->cfg.kappa;
        return th;
    }
    static Collision<C> collision(const lbm_batch* b) {
        Collision<C> cp{};
        const lbm_config& g = b->cfg;
        cp.bgk = g.collision == LBM_BGK;
        cp.omega = (C)(1.0 / g.tau);
        const double sv = 1.0 / g.tau;
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
        for (int k = 0; k < 3; ++k) cp.g[k] = k < b->dim ? g.g[k] : 0.0;
        cp.g_start = g.g_start_step;
        cp.sc_G = b->cfg.sc_G;
        return cp;
    }
    static WallBC wall(const lbm_batch* b) {
        WallBC bc;
        bc.nbmask = b->nbmask;
        bc.bidx = b->bidx;
        bc.q = b->bq;
        bc.bouzidi = b->cfg.bc_mode == LBM_BC_BOUZIDI_MC;
        return bc;
    }
    // ev, if set, holds event pairs recorded around kb_density (0, 1), kb_mu
    // (2, 3) and kb_collide (4, 5) on the batch's stream
    static void density(lbm_batch* b, bool pull, int grid, hipEvent_t* ev = nullptr) {
        const R* f = (const R*)b->f[b->cur];
        const R inv_b = (R)(1.0 / b->pr.b);
        if (ev) (void)hipEventRecord(ev[0], b->stream);
        if (pull)
            kb_density<L, R, C, true><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, f, (R*)b->rho,
                                                                   b->cls, wall(b), b->ctl, b->slots, b->mp, inv_b);
        else
            kb_density<L, R, C, false><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, f, (R*)b->rho,
                                                                    b->cls, wall(b), b->ctl, b->slots, b->mp, inv_b);
        if (ev) (void)hipEventRecord(ev[1], b->stream);
        const int ng1 = (b->n_l1 + 255) / 256, ng2 = (b->n_l2 + 255) / 256;
        if (b->n_l1)
            kb_fill<L, R, C><<<ng1 < grid ? ng1 : grid, 256, 0, b->stream>>>(b->fnode, b->fmask, (const R*)b->inv, b->fcase,
                                                                             0, b->n_l1, (R*)b->rho, b->dims);
        if (b->n_l2)
            kb_fill<L, R, C><<<ng2 < grid ? ng2 : grid, 256, 0, b->stream>>>(
                b->fnode, b->fmask, (const R*)b->inv, b->fcase, b->n_l1, b->n_l1 + b->n_l2, (R*)b->rho, b->dims);
    }
    // phase-field model: phi of the state in f[src] / g[src] (with_rho: rho
    // as well, for reads; the collision forms rho itself)
    static void pf_density(lbm_batch* b, int src, bool pull, bool with_rho, int grid) {
        const R* f = (const R*)b->f[src];
        const R* g = (const R*)b->g[src];
#define KB_PF_DENSITY(P, W)                                                                                        \
    kb_pf_density<L, R, C, P, W><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, f, g,      \
                                                              (R*)b->rho, (R*)b->phi, b->cls, wall(b), b->ctl,   \
                                                              b->slots, b->mp)
        if (pull) {
            if (with_rho) KB_PF_DENSITY(true, true);
            else KB_PF_DENSITY(true, false);
        } else {
            if (with_rho) KB_PF_DENSITY(false, true);
            else KB_PF_DENSITY(false, false);
        }
#undef KB_PF_DENSITY
    }
    static void pf_mu(lbm_batch* b, int grid) {
        kb_pf_mu<L, R><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, (const R*)b->phi, (R*)b->mu,
                                                    b->cls, b->pfp);
    }
    // the field the measurement reads: phi of the phase-field model, else rho
    static const R* mfield(const lbm_batch* b) { return (const R*)(b->pf ? b->phi : b->rho); }

    // chemical potential, or psi of the pseudopotential model, on fluid nodes
    static void launch_mu(lbm_batch* b, int grid) {
        if (b->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL)
            kb_mu<L, R, C, true><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w,
                                                              (const R*)b->rho, (R*)b->mu, b->cls, thermo(b));
        else
            kb_mu<L, R, C><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, (const R*)b->rho,
                                                        (R*)b->mu, b->cls, thermo(b));
    }

    // one step from f[src] (pull form if pull) into f[1 - src]
    static void step(lbm_batch* b, int src, bool pull, int grid, hipEvent_t* ev = nullptr) {
        if (b->pf) {
            if (ev) (void)hipEventRecord(ev[0], b->stream);
            pf_density(b, src, pull, false, grid);
            if (ev) (void)hipEventRecord(ev[1], b->stream);
        } else {
            const int save = b->cur;
            b->cur = src;
            density(b, pull, grid, ev);
            b->cur = save;
        }
        if (ev) (void)hipEventRecord(ev[2], b->stream);
        if (b->pf) pf_mu(b, grid);
        else launch_mu(b, grid);
        if (ev) (void)hipEventRecord(ev[3], b->stream);
        const R* mf = mfield(b);
        kb_cross<L, R><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, mf, b->cls, b->ctl, b->slots,
                                                    b->mp);
        YoungStep ys{};
        if (b->young_on) {
            kb_young_step<L, R><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, mf, b->cls,
                                                             b->ystep_params, b->mp, b->slots, b->ctl,
                                                             b->ystep_counts);
            ys.on = 1;
            ys.gamma = b->yopts.gamma;
            ys.c1 = std::cos(b->yopts.theta1_deg * M_PI / 180.0);
            ys.c2 = std::cos(b->yopts.theta2_deg * M_PI / 180.0);
            ys.roughness = b->yopts.roughness;
            ys.counts = b->ystep_counts;
            ys.last = b->ylast;
        }
        const R* fin = (const R*)b->f[src];
        R* fout = (R*)b->f[1 - src];
        const WallBC bc = wall(b);
        const Collision<C> cp = collision(b);
        const bool mrt = b->cfg.collision == LBM_MRT;
#define KB_ARGS b->items, b->nitems, b->dims, b->tile_w, fin, fout, (const R*)b->rho, (const R*)b->mu, b->cls, bc, cp, b->ctl
        if (ev) (void)hipEventRecord(ev[4], b->stream);
        if (b->pf) {
#define KB_PF_ARGS                                                                                              \
    b->items, b->nitems, b->dims, b->tile_w, fin, fout, (const R*)b->g[src], (R*)b->g[1 - src], (const R*)b->phi, \
        (const R*)b->mu, b->cls, bc, cp, b->pfp, b->ctl
            if (pull) {
                if (mrt) kb_pf_collide<L, R, C, true, true><<<grid, 256, 0, b->stream>>>(KB_PF_ARGS);
                else kb_pf_collide<L, R, C, true, false><<<grid, 256, 0, b->stream>>>(KB_PF_ARGS);
            } else {
                if (mrt) kb_pf_collide<L, R, C, false, true><<<grid, 256, 0, b->stream>>>(KB_PF_ARGS);
                else kb_pf_collide<L, R, C, false, false><<<grid, 256, 0, b->stream>>>(KB_PF_ARGS);
            }
#undef KB_PF_ARGS
        } else if (b->cfg.model == LBM_MODEL_PSEUDOPOTENTIAL) {
            if (pull) {
                if (mrt) kb_collide<L, R, C, true, true, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
                else kb_collide<L, R, C, true, false, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
            } else {
                if (mrt) kb_collide<L, R, C, false, true, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
                else kb_collide<L, R, C, false, false, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
            }
        } else if (pull) {
            if (mrt) kb_collide<L, R, C, true, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
            else kb_collide<L, R, C, true, false><<<grid, 256, 0, b->stream>>>(KB_ARGS);
        } else {
            if (mrt) kb_collide<L, R, C, false, true><<<grid, 256, 0, b->stream>>>(KB_ARGS);
            else kb_collide<L, R, C, false, false><<<grid, 256, 0, b->stream>>>(KB_ARGS);
        }
#undef KB_ARGS
        if (ev) (void)hipEventRecord(ev[5], b->stream);
        kb_finalize<L, R><<<b->ncases, 64, 0, b->stream>>>(mf, b->ctl, b->dims, b->mp, b->slots, b->last, ys);
        kb_tick<<<1, 64, 0, b->stream>>>(b->ctl);
    }
    // S_t of the fluid populations (order: those of the phase-field model,
    // which stream with halfway bounce-back) into the spare buffer
    static R* materialize(lbm_batch* b, int grid, bool order = false) {
        void* const* set = order ? b->g : b->f;
        R* out = (R*)set[1 - b->cur];
        WallBC bc = wall(b);
        if (order) bc.bouzidi = 0;
        if (b->fstar)
            kb_materialize<L, R, C, true><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w,
                                                                       (const R*)set[b->cur], out, b->cls, bc);
        else
            kb_materialize<L, R, C, false><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w,
                                                                        (const R*)set[b->cur], out, b->cls, bc);
        return out;
    }
    // the state at rest of rho (f_eq(rho, 0)) or, for the phase-field model,
    // of the order parameter staged in src, on packed nodes [beg, end)
    static void init_state(lbm_batch* b, const void* src, long long beg, long long end) {
        if (b->pf)
            k_pf_init<L, R><<<2048, 256, 0, b->stream>>>((const R*)src, (R*)b->phi, (R*)b->rho, (R*)b->f[b->cur],
                                                         (R*)b->g[b->cur], b->cls, b->Ntot, b->pfp.rho0, beg, end);
        else
            k_init_feq<L, R><<<4096, 256, 0, b->stream>>>((const R*)b->rho, (R*)b->f[b->cur], b->cls, b->Ntot, beg, end);
    }
};

template <template <class, typename, typename> class Op, typename... Args>
void bdispatch(lbm_batch* b, Args&&... args) {
    const int p = b->cfg.precision;
    if (b->dim == 2) {
        if (p == LBM_F64) Op<D2Q9, double, double>::go(b, args...);
        else if (p == LBM_F32_MIXED) Op<D2Q9, float, double>::go(b, args...);
        else Op<D2Q9, float, float>::go(b, args...);
    } else {
        if (p == LBM_F64) Op<D3Q19, double, double>::go(b, args...);
        else if (p == LBM_F32_MIXED) Op<D3Q19, float, double>::go(b, args...);
        else Op<D3Q19, float, float>::go(b, args...);
    }
}

template <class L, typename R, typename C>
struct BStep {
    static void go(lbm_batch* b, int src, bool pull, int grid) { BRun<L, R, C>::step(b, src, pull, grid); }
};
template <class L, typename R, typename C>
struct BStepTimed {
    static void go(lbm_batch* b, int src, bool pull, int grid, hipEvent_t* ev) {
        BRun<L, R, C>::step(b, src, pull, grid, ev);
    }
};
// the fields of the current state: rho (with the solid fill), or for the
// phase-field model phi and rho
template <class L, typename R, typename C>
struct BDerive {
    static void go(lbm_batch* b, int grid) {
        if (b->pf) BRun<L, R, C>::pf_density(b, b->cur, b->fstar, true, grid);
        else BRun<L, R, C>::density(b, b->fstar, grid);
    }
};
template <class L, typename R, typename C>
struct BMaterialize {
    static void go(lbm_batch* b, int grid, void** out, bool order) {
        *out = BRun<L, R, C>::materialize(b, grid, order);
    }
};
template <class L, typename R, typename C>
struct BInit {
    static void go(lbm_batch* b, const void* src, long long beg, long long end) {
        BRun<L, R, C>::init_state(b, src, beg, end);
    }
};
template <class L, typename R, typename C>
struct BMeasure {
    static void go(lbm_batch* b, int grid) {
        if (b->pf) {
            BRun<L, R, C>::pf_density(b, b->cur, b->fstar, true, grid);
        } else {
            BRun<L, R, C>::density(b, b->fstar, grid);
            BRun<L, R, C>::launch_mu(b, grid);
        }
        const R* mf = BRun<L, R, C>::mfield(b);
        kb_cross<L, R><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w, mf, b->cls, b->ctl,
                                                    b->slots, b->mp);
        kb_finalize<L, R><<<b->ncases, 64, 0, b->stream>>>(mf, b->ctl, b->dims, b->mp, b->slots, b->last);
    }
};

template <class L, typename R, typename C>
struct BYoung {
    static void go(lbm_batch* b, int grid) {
        kb_young_count<L, R><<<grid, 256, 0, b->stream>>>(b->items, b->nitems, b->dims, b->tile_w,
                                                         BRun<L, R, C>::mfield(b), b->cls, b->yparams, b->ycounts);
    }
};

int grid_of(const lbm_batch* b) { return b->bpc * b->cus; }

void drop_graph(lbm_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

// --- autotuner: time candidate (tile width, workgroups per CU) pairs ---------
std::string tune_key(const lbm_batch* b) {
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) { h = (h ^ v) * 1099511628211ull; };
    mix((unsigned long long)b->dim);
    mix((unsigned long long)b->cfg.precision);
    mix((unsigned long long)b->cfg.collision);
    mix((unsigned long long)b->cfg.bc_mode);
    mix((unsigned long long)b->cfg.model);
    for (const Dims& d : b->dims_h) {
        mix((unsigned long long)d.nx);
        mix((unsigned long long)d.ny);
        mix((unsigned long long)d.nz);
    }
    char buf[32];
    std::snprintf(buf, sizeof buf, "%016llx", h);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, int& tw, int& bpc) {
    if (!path) return false;
    std::ifstream in(path);
    if (!in) return false;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string s = ss.str();
    const size_t p = s.find("\"" + key + "\"");
    if (p == std::string::npos) return false;
    const size_t q1 = s.find("\"tile_w\":", p), q2 = s.find("\"blocks_per_cu\":", p);
    if (q1 == std::string::npos || q2 == std::string::npos) return false;
    tw = std::atoi(s.c_str() + q1 + 9);
    bpc = std::atoi(s.c_str() + q2 + 16);
    return (tw == 64 || tw == 128 || tw == 256) && bpc >= 1 && bpc <= 32;
}

void cache_store(const char* path, const std::string& key, int tw, int bpc, double ms) {
    if (!path) return;
    std::string body;
    {
        std::ifstream in(path);
        if (in) {
            std::stringstream ss;
            ss << in.rdbuf();
            body = ss.str();
        }
    }
    // keep the other keys: the file is {"key": {...}, ...}; drop a stale entry of this key
    std::string entries;
    size_t pos = body.find('{');
    if (pos != std::string::npos) {
        const size_t end = body.rfind('}');
        entries = body.substr(pos + 1, end > pos ? end - pos - 1 : 0);
        const size_t k = entries.find("\"" + key + "\"");
        if (k != std::string::npos) {
            const size_t e = entries.find('}', k);
            size_t from = k, to = e + 1;
            if (to < entries.size() && entries[to] == ',') ++to;
            else if (from > 0 && entries[from - 1] == ',') --from;
            entries.erase(from, to - from);
        }
    }
    while (!entries.empty() && (entries.back() == '\n' || entries.back() == ' ' || entries.back() == ',')) entries.pop_back();
    char rec[256];
    std::snprintf(rec, sizeof rec, "\n  \"%s\": {\"tile_w\": %d, \"blocks_per_cu\": %d, \"ms_per_step\": %.6f}", key.c_str(),
                  tw, bpc, ms);
    std::ofstream out(path);
    out << "{" << entries << (entries.empty() ? "" : ",") << rec << "\n}\n";
}

lbm_status autotune(lbm_batch* b, const char* cache) {
    int tw, bpc;
    const std::string key = tune_key(b);
    if (cache_lookup(cache, key, tw, bpc)) {
        b->tile_w = tw;
        b->bpc = bpc;
        build_items(b);
        return LBM_OK;
    }
    // time a few steps per candidate on a copy of the state; restore afterwards
    const size_t fb = (size_t)b->Q * b->Ntot * b->elem;
    void* snap = nullptr;
    if (balloc(b, (char**)&snap, b->pf ? 2 * fb : fb)) return LBM_E_NOMEM;
    BCHK(b, hipMemcpyAsync(snap, b->f[b->cur], fb, hipMemcpyDeviceToDevice, b->stream));
    if (b->pf) BCHK(b, hipMemcpyAsync((char*)snap + fb, b->g[b->cur], fb, hipMemcpyDeviceToDevice, b->stream));
    const int cur0 = b->cur;
    const bool fstar0 = b->fstar;
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, 0, 0, 0, 0);
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    double best = 1e30;
    int btw = 64, bbpc = 4;
    const int tws[3] = {64, 128, 256}, bpcs[4] = {2, 4, 8, 16};
    for (int tw_ : tws)
        for (int bp : bpcs) {
            b->tile_w = tw_;
            b->bpc = bp;
            build_items(b);
            auto run = [&](int n) {
                for (int s = 0; s < n; ++s) {
                    bdispatch<BStep>(b, b->cur, b->fstar, grid_of(b));
                    b->cur ^= 1;
                    b->fstar = true;
                }
            };
            run(2);
            BCHK(b, hipEventRecord(e0, b->stream));
            run(4);
            BCHK(b, hipEventRecord(e1, b->stream));
            BCHK(b, hipEventSynchronize(e1));
            float ms = 0;
            BCHK(b, hipEventElapsedTime(&ms, e0, e1));
            if (ms / 4 < best) {
                best = ms / 4;
                btw = tw_;
                bbpc = bp;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cur = cur0;
    b->fstar = fstar0;
    BCHK(b, hipMemcpyAsync(b->f[b->cur], snap, fb, hipMemcpyDeviceToDevice, b->stream));
    if (b->pf) BCHK(b, hipMemcpyAsync(b->g[b->cur], (char*)snap + fb, fb, hipMemcpyDeviceToDevice, b->stream));
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, 0, 0, 0, 1);
    BCHK(b, hipStreamSynchronize(b->stream));
    (void)hipFree(snap);
    b->tile_w = btw;
    b->bpc = bbpc;
    b->tune_ms = best;
    build_items(b);
    cache_store(cache, key, btw, bbpc, best);
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

lbm_status lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    void* ps[] = {b->dims, b->mp,   b->slots, b->last, b->ctl,  b->f[0], b->f[1], b->rho,  b->mu,   b->inv,
                  b->bq,   b->cls,  b->nbmask, b->fmask, b->bidx, b->fcase, b->fnode, b->items,
                  b->yparams, b->ycounts, b->ystep_params, b->ystep_counts, b->ylast, b->g[0], b->g[1], b->phi};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_config* base, const lbm_case* cases, int ncases, const lbm_batch_opts* opts,
                            lbm_batch** out) {
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    if (!base || !cases || ncases < 1) return LBM_E_ARG;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_E_NOMEM;
    b->cfg = *base;
    auto bad = [&]() {
        delete b;
        return LBM_E_ARG;
    };
    if (base->lattice != LBM_D2Q9 && base->lattice != LBM_D3Q19) return bad();
    if (base->model != LBM_MODEL_CHEMICAL_POTENTIAL && base->model != LBM_MODEL_PSEUDOPOTENTIAL &&
        base->model != LBM_MODEL_PHASE_FIELD)
        return bad();
    if (base->model == LBM_MODEL_PHASE_FIELD &&
        (!(base->pf_A > 0) || !(base->pf_kappa > 0) || !(base->pf_gamma > 0) || !(base->pf_tau > 0.5) ||
         !(base->pf_rho0 > 0) ||
         !std::isfinite(base->pf_A + base->pf_kappa + base->pf_gamma + base->pf_tau + base->pf_rho0)))
        return bad();
    if (base->model == LBM_MODEL_PSEUDOPOTENTIAL &&
        (!(base->rho_g > 0) || !(base->rho_l > base->rho_g) || !std::isfinite(base->sc_G)))
        return bad();
    if (base->precision != LBM_F32 && base->precision != LBM_F64 && base->precision != LBM_F32_MIXED) return bad();
    if (!(base->tau > 0.5) || !(base->k > 0) || !(base->kappa >= 0)) return bad();
    b->dim = base->lattice == LBM_D2Q9 ? 2 : 3;
    b->Q = b->dim == 2 ? 9 : 19;
    b->elem = base->precision == LBM_F64 ? 8 : 4;
    b->ncases = ncases;
    b->pr.a = base->pr_a;
    b->pr.b = base->pr_b;
    b->pr.R = base->pr_R;
    b->pr.omega = base->pr_omega;
    b->pr.Tr = base->Tr;
    std::string err;
    if (!pr_solve(b->pr, err)) return bad();
    if (base->rho_l > 0) b->pr.rho_l = base->rho_l;
    if (base->rho_g > 0) b->pr.rho_g = base->rho_g;
    b->rho_m = 0.5 * (b->pr.rho_l + b->pr.rho_g);
    b->mu_ref = base->k * base->k * b->pr.mu_sat;
    b->wall_mu = std::isnan(base->wall_mu) ? b->mu_ref : base->wall_mu;
    if (base->model == LBM_MODEL_PSEUDOPOTENTIAL) {
        // wall values are densities; psi is stored unshifted
        b->mu_ref = 0.0;
        b->wall_mu = std::isnan(base->wall_mu) ? b->rho_m : base->wall_mu;
    }
    b->pf = base->model == LBM_MODEL_PHASE_FIELD;
    // initial interface width of Eq. 16
    double W = 10.0;
    if (b->pf) {
        // bulk order parameters +1 / -1, isolevel 0; wall values are order
        // parameters, written into phi; the drop takes the flat-interface
        // profile tanh(r / xi), xi = sqrt(2 kappa / A), i.e. Eq. 16 with W = 2 xi
        b->pr.rho_l = 1.0;
        b->pr.rho_g = -1.0;
        b->rho_m = 0.0;
        b->mu_ref = 0.0;
        b->wall_mu = std::isnan(base->wall_mu) ? 0.0 : base->wall_mu;
        b->pfp.A = base->pf_A;
        b->pfp.kappa = base->pf_kappa;
        b->pfp.gamma = base->pf_gamma;
        b->pfp.omega = 1.0 / base->pf_tau;
        b->pfp.rho0 = base->pf_rho0;
        W = 2.0 * std::sqrt(2.0 * base->pf_kappa / base->pf_A);
    }
    const bool sc = base->model == LBM_MODEL_PSEUDOPOTENTIAL;
    auto wall_value = [&](double v) { return sc ? 1.0 - std::exp(-v) : v - b->mu_ref; };
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (base->stream) {
        b->stream = (hipStream_t)base->stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return LBM_E_DEVICE;
        }
        b->own_stream = true;
    }

    // geometry of every case on the host, packed at increasing offsets
    const int wall[3] = {base->axis_bc[0] == LBM_WALL, base->axis_bc[1] == LBM_WALL,
                         b->dim == 3 && base->axis_bc[2] == LBM_WALL};
    std::vector<uint8_t> cls;
    std::vector<uint32_t> nbm, fmask;
    std::vector<int> bidx, fcase;
    std::vector<long long> fnode1, fnode2;
    std::vector<uint32_t> fmask1, fmask2;
    std::vector<double> inv1, inv2, bq, muh, rhoh;
    std::vector<int> fcase1, fcase2;
    long long off = 0;
    int nb_total = 0;
    for (int ci = 0; ci < ncases; ++ci) {
        const lbm_case& cs = cases[ci];
        int n[3] = {cs.n[0], cs.n[1], b->dim == 3 ? cs.n[2] : 1};
        if (n[0] < 5 || n[1] < 5 || n[2] < 1 || (b->dim == 3 && n[2] < 5)) {
            lbm_batch_destroy(b);
            return LBM_E_ARG;
        }
        if (cs.solid.kind != LBM_SOLID_SPHERE && cs.solid.kind != LBM_SOLID_CAVITY) {
            lbm_batch_destroy(b);
            return LBM_E_ARG;
        }
        Solid s{};
        for (int k = 0; k < 3; ++k) s.c[k] = k < b->dim ? cs.solid.center[k] : 0.0;
        s.r = cs.solid.radius;
        s.concave = cs.solid.kind == LBM_SOLID_CAVITY;
        s.wet_mode = cs.solid.wet_mode;
        s.mu1 = cs.solid.mu_w;
        s.mu2 = cs.solid.mu_w2;
        s.width = cs.solid.stripe_width > 0 ? cs.solid.stripe_width : 1.0;
        double pl[3] = {cs.solid.pole[0], cs.solid.pole[1], b->dim == 3 ? cs.solid.pole[2] : 0.0};
        double pn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        if (pn == 0) { pl[0] = 0; pl[1] = b->dim == 2 ? 1 : 0; pl[2] = b->dim == 2 ? 0 : 1; pn = 1; }
        for (int k = 0; k < 3; ++k) s.pole[k] = pl[k] / pn;
        if (!(s.r > 0)) {
            lbm_batch_destroy(b);
            return LBM_E_ARG;
        }
        Geometry g;
        if (!build_geometry(g, b->dim, n, wall, std::vector<Solid>{s}, nullptr, b->wall_mu, err)) {
            lbm_batch_destroy(b);
            return LBM_E_ARG;
        }
        // rows padded to a multiple of 64 nodes, so that every row of every
        // case starts on a 256-byte boundary (FP32) and the 64-wide tiles of
        // the work list are aligned; pad nodes are deep solid and never read
        const int px = (n[0] + 63) / 64 * 64;
        const long long Np = (long long)px * n[1] * n[2];
        auto at = [&](long long i) {  // unpadded node index of the case -> padded
            return (i / n[0]) * px + i % n[0];
        };
        Dims d{};
        d.nx = n[0];
        d.px = px;
        d.ny = n[1];
        d.nz = n[2];
        d.off = off;
        b->dims_h.push_back(d);
        b->solids_h.push_back(s);
        MeasureParams mp{};
        for (int k = 0; k < 3; ++k) {
            mp.c[k] = s.c[k];
            mp.g[k] = k < b->dim ? base->g[k] : 0.0;
        }
        mp.R = s.r;
        mp.concave = s.concave;
        mp.rho_m = b->rho_m;
        mp.n_sectors = b->dim == 2 ? 2 : 16;
        mp.dim = b->dim;
        b->mp_h.push_back(mp);
        const size_t base_at = cls.size();
        cls.resize(base_at + (size_t)Np, (uint8_t)3);
        nbm.resize(base_at + (size_t)Np, 0u);
        bidx.resize(base_at + (size_t)Np, -1);
        muh.resize(base_at + (size_t)Np, 0.0);
        rhoh.resize(base_at + (size_t)Np, 0.0);
        for (long long i = 0; i < g.N; ++i) {
            cls[base_at + at(i)] = g.cls[i];
            nbm[base_at + at(i)] = g.nbmask[i];
        }
        for (size_t k = 0; k < g.b_node.size(); ++k) bidx[base_at + at(g.b_node[k])] = nb_total + (int)k;
        bq.insert(bq.end(), g.b_q.begin(), g.b_q.end());
        nb_total += (int)g.b_node.size();
        for (size_t k = 0; k < g.l1_node.size(); ++k) {
            muh[base_at + at(g.l1_node[k])] = wall_value(g.l1_mu[k]);
            fnode1.push_back(off + at(g.l1_node[k]));
            fmask1.push_back(g.l1_mask[k]);
            inv1.push_back(g.l1_inv[k]);
            fcase1.push_back(ci);
        }
        for (size_t k = 0; k < g.l2_node.size(); ++k) {
            muh[base_at + at(g.l2_node[k])] = wall_value(g.l2_mu[k]);
            fnode2.push_back(off + at(g.l2_node[k]));
            fmask2.push_back(g.l2_mask[k]);
            inv2.push_back(g.l2_inv[k]);
            fcase2.push_back(ci);
        }
        // Eq. 16 around the case's drop
        const double rg = b->pr.rho_g, rl = b->pr.rho_l;
        for (long long i = 0; i < g.N; ++i) {
            if ((g.cls[i] & 3) != 0) continue;
            const int x = (int)(i % n[0]), y = (int)((i / n[0]) % n[1]), z = (int)(i / ((long long)n[0] * n[1]));
            const double dx = x - cs.drop.center[0], dy = y - cs.drop.center[1];
            const double dz = b->dim == 3 ? z - cs.drop.center[2] : 0.0;
            const double rr = std::sqrt(dx * dx + dy * dy + dz * dz);
            rhoh[base_at + at(i)] = 0.5 * (rg + rl) + 0.5 * (rg - rl) * std::tanh(2.0 * (rr - cs.drop.radius) / W);
        }
        b->n_fluid += g.n_fluid;
        b->n_nodes += g.N;
        off += Np;
    }
    b->Ntot = off;
    if ((unsigned long long)b->Ntot * (unsigned long long)b->Q >= (1ull << 32)) {
        lbm_batch_destroy(b);
        return LBM_E_ARG;
    }
    for (Dims& d : b->dims_h) d.N = b->Ntot;
    b->n_l1 = (int)fnode1.size();
    b->n_l2 = (int)fnode2.size();
    std::vector<long long> fnode(fnode1);
    fnode.insert(fnode.end(), fnode2.begin(), fnode2.end());
    fmask = fmask1;
    fmask.insert(fmask.end(), fmask2.begin(), fmask2.end());
    std::vector<double> inv(inv1);
    inv.insert(inv.end(), inv2.begin(), inv2.end());
    fcase = fcase1;
    fcase.insert(fcase.end(), fcase2.begin(), fcase2.end());

    lbm_status s;
    const size_t fb = (size_t)b->Q * b->Ntot * b->elem;
    if ((s = balloc(b, (char**)&b->f[0], fb)) || (s = balloc(b, (char**)&b->f[1], fb)) ||
        (s = bupload(b, &b->dims, b->dims_h)) || (s = bupload(b, &b->mp, b->mp_h)) ||
        (s = balloc(b, &b->slots, (size_t)ncases * sizeof(MeasureSlots))) ||
        (s = balloc(b, &b->last, (size_t)ncases * sizeof(AngleRec))) || (s = balloc(b, &b->ctl, sizeof(DevCtl))) ||
        (s = bupload(b, &b->cls, cls)) || (s = bupload(b, &b->nbmask, nbm)) || (s = bupload(b, &b->bidx, bidx)) ||
        (s = bupload_real(b, &b->bq, bq)) ||
        (s = bupload_real(b, b->pf ? &b->phi : &b->mu, muh)) ||
        (b->pf && ((s = balloc(b, (char**)&b->g[0], fb)) || (s = balloc(b, (char**)&b->g[1], fb)) ||
                   (s = bupload_real(b, &b->mu, std::vector<double>(muh.size(), 0.0))))) ||
        (s = bupload_real(b, &b->rho, rhoh)) ||
        (s = bupload(b, &b->fnode, fnode)) || (s = bupload(b, &b->fmask, fmask)) || (s = bupload_real(b, &b->inv, inv)) ||
        (s = bupload(b, &b->fcase, fcase))) {
        std::string e = b->err;
        lbm_batch_destroy(b);
        return s;
    }
    DevCtl h{};
    for (auto& k : h.m.keys) k[0] = k[1] = ~0ull;
    if (hipMemcpy(b->ctl, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
        lbm_batch_destroy(b);
        return LBM_E_DEVICE;
    }
    kb_slots_reset<<<ncases, 64, 0, b->stream>>>(b->slots, ncases);
    // state = f_eq(rho, 0) with rho of Eq. 16; phase-field model: the order
    // parameter of Eq. 16 (staged in rho) at rest, rho = rho0
    auto zero = [&](void* p) {
        if (b->elem == 8) k_fill_value<double><<<2048, 256, 0, b->stream>>>((double*)p, fb / 8, 0.0);
        else k_fill_value<float><<<2048, 256, 0, b->stream>>>((float*)p, fb / 4, 0.0f);
    };
    zero(b->f[1]);
    if (b->pf) {
        zero(b->g[1]);
        if (hipMemcpyAsync(b->g[1], b->rho, (size_t)b->Ntot * b->elem, hipMemcpyDeviceToDevice, b->stream) !=
            hipSuccess) {
            lbm_batch_destroy(b);
            return LBM_E_DEVICE;
        }
    }
    bdispatch<BInit>(b, b->pf ? (const void*)b->g[1] : nullptr, 0ll, b->Ntot);
    if (b->pf) zero(b->g[1]);
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        lbm_batch_destroy(b);
        return LBM_E_DEVICE;
    }
    b->have_state = true;
    b->tile_w = opts && (opts->tile_w == 64 || opts->tile_w == 128 || opts->tile_w == 256) ? opts->tile_w : 64;
    b->bpc = opts && opts->blocks_per_cu >= 1 && opts->blocks_per_cu <= 32 ? opts->blocks_per_cu : 4;
    build_items(b);
    if (!b->items) {
        lbm_batch_destroy(b);
        return LBM_E_NOMEM;
    }
    if (opts && opts->autotune) {
        if ((s = autotune(b, opts->cache_path))) {
            lbm_batch_destroy(b);
            return s;
        }
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps, int measure_every) {
    if (!b) return LBM_E_ARG;
    if (nsteps < 0 || measure_every < 0) return bfail(b, LBM_E_ARG, "batch step: negative argument");
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, measure_every, 0, 0, 0);
    BCHK(b, hipGetLastError());
    int64_t done = 0;
    auto eager = [&]() {
        bdispatch<BStep>(b, b->cur, b->fstar, grid_of(b));
        b->cur ^= 1;
        b->fstar = true;
        ++done;
        ++b->t;
    };
    while (done < nsteps && (!b->fstar || b->cur != 0 || nsteps - done < kBatchGraphSteps)) eager();
    if (nsteps - done >= kBatchGraphSteps) {
        if (!b->graph) {
            hipGraph_t g;
            BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < kBatchGraphSteps; ++k) bdispatch<BStep>(b, k & 1, true, grid_of(b));
            BCHK(b, hipStreamEndCapture(b->stream, &g));
            const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->graph = nullptr;
                return bfail(b, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        while (nsteps - done >= kBatchGraphSteps) {
            BCHK(b, hipGraphLaunch(b->graph, b->stream));
            done += kBatchGraphSteps;
            b->t += kBatchGraphSteps;
        }
    }
    while (done < nsteps) eager();
    BCHK(b, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_batch_profile_step(lbm_batch* b, int64_t nsteps, const char** names, double* ms, int cap,
                                  int* n_kinds) {
    static const char* kNames[3] = {"kb_density", "kb_mu", "kb_collide"};
    static const char* kPfNames[3] = {"kb_pf_density", "kb_pf_mu", "kb_pf_collide"};
    if (!b || !names || !ms || !n_kinds || cap < 0) return LBM_E_ARG;
    if (!b->have_state) return bfail(b, LBM_E_STATE, "batch profile: no state");
    if (nsteps < 1) return bfail(b, LBM_E_ARG, "batch profile: nsteps >= 1");
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, 0, 0, 0, 0);
    BCHK(b, hipGetLastError());
    hipEvent_t ev[6];
    int made = 0;
    for (auto& e : ev) {
        if (hipEventCreate(&e) != hipSuccess) break;
        ++made;
    }
    if (made < 6) {
        for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
        return bfail(b, LBM_E_DEVICE, "batch profile: hipEventCreate failed");
    }
    double tot[3] = {0, 0, 0};
    hipError_t err = hipSuccess;
    for (int64_t t = 0; t < nsteps && err == hipSuccess; ++t) {
        bdispatch<BStepTimed>(b, b->cur, b->fstar, grid_of(b), ev);
        b->cur ^= 1;
        b->fstar = true;
        ++b->t;
        err = hipStreamSynchronize(b->stream);
        for (int k = 0; k < 3 && err == hipSuccess; ++k) {
            float e = 0;
            err = hipEventElapsedTime(&e, ev[2 * k], ev[2 * k + 1]);
            tot[k] += e;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch profile: ") + hipGetErrorString(err));
    int n = 0;
    for (int k = 0; k < 3 && n < cap; ++k, ++n) {
        names[n] = b->pf ? kPfNames[k] : kNames[k];
        ms[n] = tot[k] / (double)nsteps;
    }
    *n_kinds = n;
    return lbm_batch_sync(b);
}

lbm_status lbm_batch_sync(lbm_batch* b) {
    if (!b) return LBM_E_ARG;
    DevCtl h;
    BCHK(b, hipMemcpyAsync(&h, b->ctl, sizeof h, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    if (h.status & 1) return bfail(b, LBM_E_NONFINITE, "a density became non-finite, non-positive or >= 1/b");
    return LBM_OK;
}

lbm_status lbm_batch_angles(lbm_batch* b, lbm_angle* out, int n) {
    if (!b || !out || n < 1 || n > b->ncases) return b ? bfail(b, LBM_E_ARG, "batch angles: bad count") : LBM_E_ARG;
    BCHK(b, hipStreamSynchronize(b->stream));
    BCHK(b, hipMemcpy(out, b->last, (size_t)n * sizeof(AngleRec), hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status lbm_batch_measure(lbm_batch* b, lbm_angle* out, int n) {
    if (!b || !out || n < 1 || n > b->ncases) return b ? bfail(b, LBM_E_ARG, "batch measure: bad count") : LBM_E_ARG;
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, 0, 1, 0, 0);
    kb_slots_reset<<<b->ncases, 64, 0, b->stream>>>(b->slots, b->ncases);
    bdispatch<BMeasure>(b, grid_of(b));
    k_ctl_set<<<1, 64, 0, b->stream>>>(b->ctl, b->t, 0, 0, 0, 0);
    BCHK(b, hipGetLastError());
    return lbm_batch_angles(b, out, n);
}

lbm_status lbm_batch_young_force(lbm_batch* b, const lbm_young_opts* yo, lbm_angle* angles, lbm_young* out, int n) {
    if (!b) return LBM_E_ARG;
    if (!yo || !angles || !out || n != b->ncases)
        return bfail(b, LBM_E_ARG, "batch young: null pointer, or n is not the number of cases");
    if (!young_opts_ok(*yo))
        return bfail(b, LBM_E_ARG, "batch young: gamma finite, roughness > 0, 0 < band_lo < band_hi < 1");
    double lo, hi;
    young_band(*yo, lo, hi);
    lbm_status st = lbm_batch_measure(b, angles, n);
    if (st != LBM_OK) return st;
    const size_t cbytes = (size_t)n * 2 * LBM_MAX_SECTORS * sizeof(unsigned);
    if (!b->yparams) {
        if (hipMalloc((void**)&b->yparams, (size_t)n * sizeof(YoungParams)) != hipSuccess ||
            hipMalloc((void**)&b->ycounts, cbytes) != hipSuccess)
            return bfail(b, LBM_E_NOMEM, "batch young: device allocation failed");
    }
    // counting parameters of every case with a contact line (the others are skipped)
    std::vector<YoungParams> yp((size_t)n);
    for (int c = 0; c < n; ++c)
        if (angles[c].status == LBM_OK)
            yp[c] = young_params(b->solids_h[c], angles[c], b->dim, b->pr.rho_g, b->pr.rho_l, lo, hi);
    BCHK(b, hipMemcpyAsync(b->yparams, yp.data(), yp.size() * sizeof(YoungParams), hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipMemsetAsync(b->ycounts, 0, cbytes, b->stream));
    bdispatch<BYoung>(b, grid_of(b));
    BCHK(b, hipGetLastError());
    std::vector<unsigned> h((size_t)n * 2 * LBM_MAX_SECTORS);
    BCHK(b, hipMemcpyAsync(h.data(), b->ycounts, cbytes, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    for (int c = 0; c < n; ++c) {
        young_clear(angles[c], (lbm_status)angles[c].status, &out[c]);
        if (angles[c].status == LBM_OK) young_from_counts(*yo, angles[c], &h[(size_t)c * 2 * LBM_MAX_SECTORS], &out[c]);
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_young(lbm_batch* b, const lbm_young_opts* yo) {
    if (!b) return LBM_E_ARG;
    if (yo && !young_opts_ok(*yo))
        return bfail(b, LBM_E_ARG, "batch set_young: gamma finite, roughness > 0, 0 < band_lo < band_hi < 1");
    BCHK(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    // off until every buffer below is allocated and initialised: the step
    // graphs launch the in-step kernels only when it is on
    b->young_on = false;
    if (!yo) return LBM_OK;
    b->yopts = *yo;
    const int n = b->ncases;
    const size_t cbytes = (size_t)n * 2 * LBM_MAX_SECTORS * sizeof(unsigned);
    auto get = [&](void** p, size_t bytes) {
        if (*p) return true;
        if (hipMalloc(p, bytes) == hipSuccess) return true;
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    };
    if (!get((void**)&b->ystep_params, (size_t)n * sizeof(YoungParams)) || !get((void**)&b->ystep_counts, cbytes) ||
        !get((void**)&b->ylast, (size_t)n * sizeof(YoungRec)))
        return bfail(b, LBM_E_NOMEM, "batch set_young: device allocation failed");
    // static counting parameters per case; the drop axis comes from each measurement
    double lo, hi;
    young_band(*yo, lo, hi);
    std::vector<YoungParams> yp((size_t)n);
    for (int c = 0; c < n; ++c) {
        lbm_angle a{};
        a.n_sectors = b->mp_h[c].n_sectors;
        yp[c] = young_params(b->solids_h[c], a, b->dim, b->pr.rho_g, b->pr.rho_l, lo, hi);
    }
    BCHK(b, hipMemcpy(b->ystep_params, yp.data(), yp.size() * sizeof(YoungParams), hipMemcpyHostToDevice));
    BCHK(b, hipMemset(b->ystep_counts, 0, cbytes));
    // records stay NaN until the first measurement
    std::vector<YoungRec> empty((size_t)n);
    for (auto& r : empty) {
        std::memset(&r, 0, sizeof r);
        r.status = LBM_E_NO_CONTACT_LINE;
        for (int k = 0; k < LBM_MAX_SECTORS; ++k) r.phi_d[k] = r.theta_eq_deg[k] = r.force[k] = NAN;
    }
    BCHK(b, hipMemcpy(b->ylast, empty.data(), empty.size() * sizeof(YoungRec), hipMemcpyHostToDevice));
    b->young_on = true;
    return LBM_OK;
}

lbm_status lbm_batch_young_last(lbm_batch* b, lbm_young* out, int n) {
    if (!b) return LBM_E_ARG;
    if (!out || n < 1 || n > b->ncases) return bfail(b, LBM_E_ARG, "batch young_last: bad count");
    if (!b->young_on) return bfail(b, LBM_E_STATE, "batch young_last: the in-step Young force is off");
    BCHK(b, hipStreamSynchronize(b->stream));
    BCHK(b, hipMemcpy(out, b->ylast, (size_t)n * sizeof(YoungRec), hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status lbm_batch_read(lbm_batch* b, int ci, int field, void* dst, size_t bytes, int dst_on_device) {
    if (!b || !dst) return b ? bfail(b, LBM_E_ARG, "batch read: null destination") : LBM_E_ARG;
    if (ci < 0 || ci >= b->ncases) return bfail(b, LBM_E_ARG, "batch read: case index out of range");
    const Dims& d = b->dims_h[ci];
    const size_t n = (size_t)d.nx * d.ny * d.nz, rows = (size_t)d.ny * d.nz;
    const size_t e = b->elem, w = (size_t)d.nx * e, sp = (size_t)d.px * e;  // row bytes, padded row bytes
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (field == LBM_FIELD_RHO || (field == LBM_FIELD_PHI && b->pf)) {
        if (bytes != n * e) return bfail(b, LBM_E_ARG, "batch read RHO/PHI: bytes must be n * elem");
        bdispatch<BDerive>(b, grid_of(b));
        const char* src = (const char*)(field == LBM_FIELD_RHO ? b->rho : b->phi);
        BCHK(b, hipMemcpy2DAsync(dst, w, src + (size_t)d.off * e, sp, w, rows, kind, b->stream));
    } else if (field == LBM_FIELD_F || (field == LBM_FIELD_G && b->pf)) {
        if (bytes != (size_t)b->Q * n * e) return bfail(b, LBM_E_ARG, "batch read F/G: bytes must be Q * n * elem");
        void* S = nullptr;
        bdispatch<BMaterialize>(b, grid_of(b), &S, field == LBM_FIELD_G);
        for (int i = 0; i < b->Q; ++i)
            BCHK(b, hipMemcpy2DAsync((char*)dst + (size_t)i * n * e, w,
                                     (char*)S + ((size_t)i * b->Ntot + (size_t)d.off) * e, sp, w, rows, kind,
                                     b->stream));
    } else if (field == LBM_FIELD_CLASS) {
        if (bytes != n) return bfail(b, LBM_E_ARG, "batch read CLASS: bytes must be n");
        std::vector<uint8_t> h(n);
        BCHK(b, hipStreamSynchronize(b->stream));
        BCHK(b, hipMemcpy2D(h.data(), d.nx, b->cls + d.off, d.px, d.nx, rows, hipMemcpyDeviceToHost));
        for (auto& v : h) v &= 3;
        if (dst_on_device) BCHK(b, hipMemcpyAsync(dst, h.data(), n, hipMemcpyHostToDevice, b->stream));
        else std::memcpy(dst, h.data(), n);
    } else {
        return bfail(b, LBM_E_ARG, "batch read: field must be RHO, F or CLASS (phase-field model: also PHI or G)");
    }
    BCHK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_write(lbm_batch* b, int ci, int field, const void* src, size_t bytes, int src_on_device) {
    if (!b || !src) return b ? bfail(b, LBM_E_ARG, "batch write: null source") : LBM_E_ARG;
    if (ci < 0 || ci >= b->ncases) return bfail(b, LBM_E_ARG, "batch write: case index out of range");
    const int want = b->pf ? LBM_FIELD_PHI : LBM_FIELD_RHO;
    if (field != want)
        return bfail(b, LBM_E_ARG, b->pf ? "batch write: field must be PHI (phase-field model)"
                                         : "batch write: field must be RHO");
    const Dims& d = b->dims_h[ci];
    const size_t n = (size_t)d.nx * d.ny * d.nz, rows = (size_t)d.ny * d.nz;
    if (bytes != n * b->elem) return bfail(b, LBM_E_ARG, "batch write RHO/PHI: bytes must be n * elem");
    // bring every case to form S (materialize; both population sets of the
    // phase-field model), then replace this case's populations
    if (b->fstar) {
        void* S = nullptr;
        bdispatch<BMaterialize>(b, grid_of(b), &S, false);
        if (b->pf) bdispatch<BMaterialize>(b, grid_of(b), &S, true);
        b->cur ^= 1;
        b->fstar = false;
        drop_graph(b);
    }
    BCHK(b, hipStreamSynchronize(b->stream));
    // stream-ordered: a device-to-device copy may otherwise still be in flight
    // when the state is formed (or when the caller reuses src).  The order
    // parameter is staged in the spare g buffer (free between steps) at the
    // case's offset; rho is the field itself.
    char* stage = (char*)(b->pf ? b->g[1 - b->cur] : b->rho);
    BCHK(b, hipMemcpy2DAsync(stage + (size_t)d.off * b->elem, (size_t)d.px * b->elem, src, (size_t)d.nx * b->elem,
                             (size_t)d.nx * b->elem, rows,
                             src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->stream));
    // the state at rest on this case's range of the packed arrays (pad nodes are solid: zero)
    const long long beg = d.off, end = d.off + (long long)d.px * d.ny * d.nz;
    bdispatch<BInit>(b, (const void*)stage, beg, end);
    if (b->pf) {
        const size_t fb = (size_t)b->Q * b->Ntot * b->elem;
        if (b->elem == 8) k_fill_value<double><<<2048, 256, 0, b->stream>>>((double*)stage, fb / 8, 0.0);
        else k_fill_value<float><<<2048, 256, 0, b->stream>>>((float*)stage, fb / 4, 0.0f);
    }
    BCHK(b, hipGetLastError());
    BCHK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_get_info(lbm_batch* b, lbm_batch_info* info) {
    if (!b || !info) return LBM_E_ARG;
    std::memset(info, 0, sizeof *info);
    info->total_nodes = b->n_nodes;
    info->fluid_nodes = b->n_fluid;
    info->ncases = b->ncases;
    info->tile_w = b->tile_w;
    info->blocks_per_cu = b->bpc;
    info->n_items = b->nitems;
    info->tune_ms_per_step = b->tune_ms;
    info->step = b->t;
    info->rho_g = b->pr.rho_g;
    info->rho_l = b->pr.rho_l;
    return LBM_OK;
}

lbm_status lbm_batch_tune(lbm_batch* b, const char* cache_path) {
    if (!b) return LBM_E_ARG;
    drop_graph(b);
    return autotune(b, cache_path);
}

}  // extern "C"
