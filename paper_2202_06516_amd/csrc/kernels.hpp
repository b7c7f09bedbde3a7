// kernels.hpp -- HIP kernels of one multiphase lattice Boltzmann step on gfx950.
//
// One step t -> t+1 (paper Sec. II and Sec. III A) on the split path, as
// separate launches (fused.hpp holds the one-pass step of D3Q19 lattices):
//   density     rho = sum_i S_i over fluid nodes; on measure steps also the
//               integer centroid sums of the liquid (rho >= rho_m)
//   fill        Eq. 14 over the compact list of first-layer solid nodes, then
//               (second launch) over the second layer
//   mu          mu = k^2 psi'(rho) - kappa lap4(rho) on fluid nodes (Eq. 11-12)
//   cross       on measure steps the isodensity crossings of Eq. 15 near the
//               substrate; per sector and band the crossing nearest 1 or 2 lu
//               from the wall (64-bit minimum of a packed key)
//   collide     F = -rho grad4(mu) + cs^2 grad4(rho) + rho g (Eq. 7), MRT or BGK
//               relaxation (Eq. 1-3) with exact-difference forcing (Eq. 13);
//               streaming (Eq. 4) is the gather at the start of the next step
//   finalize    one block per lattice: on measure steps turns the selected
//               crossings into contact angles (secant, contact point, tangent;
//               Fig. 1), then clears the reduction slots and advances t
// The wall chemical potential of the two solid layers is static and is written
// into mu once, when the solids are set.
//
// Every per-node computation is a device function ("body") shared by two kinds
// of launch: one lattice tiled by 256-thread workgroups (one 256-node row
// segment, or 128 x 2 / 64 x 4 nodes on narrower lattices), or many packed
// lattices walked by a persistent work list (the batched solver).  A lattice
// lives at offset off of the packed arrays; N is the population stride.
//
// Data layout in HBM: populations structure-of-arrays [Q][N], x fastest, two
// buffers; rho[N], mu[N] in the storage precision; cls[N] uint8 (bits 0-1
// class, bit 2 boundary fluid node); nbmask[N] uint32 (bit j: x+e_j solid) and
// bidx[N] (boundary-list index), read only for boundary nodes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

// bit 3: a boundary fluid node with a cut link of wall fraction other than 1/2
enum : uint8_t { CLS_FLUID = 0, CLS_L1 = 1, CLS_L2 = 2, CLS_DEEP = 3, CLS_MASK = 3, CLS_BOUNDARY = 4, CLS_CURVED = 8 };

struct Dims {
    int nx, ny, nz;
    int px;              // row pitch in nodes (>= nx): consecutive rows start px nodes apart
    long long N;         // population stride (all packed nodes)
    long long off;       // first node of this lattice in the packed arrays
    int tx, ty;          // tiles per row / per plane
    unsigned nblocks;    // tx * ty * nz workgroups
    int xcd_remap;       // 1: contiguous tile ranges per XCD
    int tws;             // log2 of the tile width: tiles of 2^tws x 256 / 2^tws nodes (one per 256-thread workgroup)
    int zc;              // planes per workgroup of the z-chunked chemical-potential kernel (<= 1: one plane)
    unsigned nblocks_zc; // tx * ty * ceil(nz / zc) workgroups of that kernel
};

__device__ __forceinline__ long long nid(const Dims& d, int x, int y, int z) {
    return d.off + ((long long)z * d.ny + y) * d.px + x;
}
// the same in 32 bits, for lattices of fewer than 2^32 packed nodes
__device__ __forceinline__ uint32_t nid32(const Dims& d, int x, int y, int z) {
    return (uint32_t)d.off + ((uint32_t)z * (uint32_t)d.ny + (uint32_t)y) * (uint32_t)d.px + (uint32_t)x;
}

// Node of this thread in tile t (x fastest, then y, then z).
__device__ __forceinline__ void tile_coords(const Dims& d, unsigned t, int& x, int& y, int& z) {
    const unsigned txi = t % (unsigned)d.tx, rest = t / (unsigned)d.tx;
    x = (int)(txi << d.tws) + (int)(threadIdx.x & ((1u << d.tws) - 1u));
    y = (int)(rest % (unsigned)d.ty) * (256 >> d.tws) + (int)(threadIdx.x >> d.tws);
    z = (int)(rest / (unsigned)d.ty);
}

// Node of this thread.  Workgroups are dispatched to the 8 XCDs round-robin
// by workgroup id; with xcd_remap each XCD receives one contiguous range of
// tiles (a slab of z planes), so the stencil neighbours of a tile sit in the
// same L2.  The map is a bijection of [0, nblocks).
__device__ __forceinline__ void tile_node(const Dims& d, int& x, int& y, int& z) {
    unsigned t = blockIdx.x;
    if (d.xcd_remap) {
        const unsigned q = d.nblocks >> 3, r = d.nblocks & 7u, xcd = t & 7u, loc = t >> 3;
        t = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + loc;
    }
    tile_coords(d, t, x, y, z);
}

// Tile and first plane of a z-chunked workgroup: the tile of blockIdx in the
// grid of nblocks_zc workgroups (XCD-contiguous as tile_node); the workgroup
// then walks zc consecutive planes, so the z-neighbour planes of its density
// stencil are the ones it read an iteration before.  (Chunking the collision
// the same way made it slower: 0.69-0.77 ms instead of 0.61 ms at 256^3.)
__device__ __forceinline__ void tile_node_zc(const Dims& d, int& x, int& y, int& z0) {
    unsigned t = blockIdx.x;
    if (d.xcd_remap) {
        const unsigned q = d.nblocks_zc >> 3, r = d.nblocks_zc & 7u, xcd = t & 7u, loc = t >> 3;
        t = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + loc;
    }
    int zi;
    tile_coords(d, t, x, y, zi);
    z0 = zi * d.zc;
}

// Peng-Robinson coefficients of psi'(rho) (Eq. 11, C = 0), pre-scaled by k^2.
// psi' is evaluated in double precision; the kernels store mu - mu_ref with
// mu_ref = k^2 mu_sat, which leaves every gradient unchanged and keeps FP32
// storage of mu accurate near coexistence.
struct Thermo {
    double k2RT;      // k^2 R T
    double k2A;       // k^2 a alpha / (2 sqrt2 b)
    double k2aal;     // k^2 a alpha
    double b;
    double s2m1, s2p1;  // sqrt2 - 1, sqrt2 + 1
    double mu_ref;
    double kappa;
};

template <typename R>
struct Collision {
    int bgk;
    R omega;         // 1/tau for the BGK path
    R rate[19];      // MRT: s_k / |row_k|^2 per moment
    double g[3];     // body acceleration (the force is formed in double)
    long long g_start;
    double sc_G;     // pseudopotential interaction strength
};

// Reduction slots of one lattice's in-step measurement.
struct MeasureSlots {
    unsigned long long cnt, sx, sy, sz;      // liquid centroid sums
    unsigned long long keys[64][2];          // per sector, per band (1 lu, 2 lu)
};

// Step counter, measurement cadence and status word (one per context).
struct DevCtl {
    long long t;                 // completed steps
    int every;                   // measurement cadence of the running step call
    int force_measure;           // 1: measure whatever t is (standalone measurement)
    int status;                  // bit 0: non-finite / non-physical density seen
    int series_count, series_cap;
    int pad_;
    MeasureSlots m;              // slots of a single-lattice context
};

struct MeasureParams {
    double c[3];     // substrate centre
    double R;        // substrate radius
    int concave;     // 0: convex ball, fluid outside; 1: cavity, fluid inside
    double rho_m;    // isodensity level
    double g[3];     // body acceleration (advancing side)
    int n_sectors;
    int dim;
};

// Result record; the layout is that of lbm_angle in lbm.h.
struct AngleRec {
    long long step;
    int status, n_sectors, n_valid, pad_;
    double mean_deg, adv_deg, rec_deg;
    double axis[3];
    double sector_deg[64];
    double contact[64][3];
};

__device__ __forceinline__ bool measuring(const DevCtl* ctl) {
    return ctl->force_measure || (ctl->every > 0 && (ctl->t % ctl->every) == 0);
}

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Element k of an array, addressed as its base plus a 32-bit byte offset:
// loads and stores then take the base from scalar registers and a single
// 32-bit vector offset, instead of a 64-bit address formed per access in
// vector registers.  Every array a kernel indexes this way is smaller than
// 4 GiB (lbm_create and lbm_batch_create keep N * Q below 2^32 nodes, and one
// population array holds N values).
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t k) {
    return *(T*)((char*)base + k * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& at(const T* base, uint32_t k) {
    return *(const T*)((const char*)base + k * (uint32_t)sizeof(T));
}

// Periodic neighbour offsets of coordinate v (0 <= v < n >= 2) along an axis
// of the given stride: index differences to v - 2, v - 1, v + 1, v + 2.
// Within one lattice they fit 32 bits; node indices stay 64-bit.
struct Nbr {
    int m2, m1, p1, p2;
};
__device__ __forceinline__ Nbr nbr_offsets(int v, int n, int stride) {
    Nbr o;
    o.m1 = (v >= 1 ? -1 : n - 1) * stride;
    o.m2 = (v >= 2 ? -2 : n - 2) * stride;
    o.p1 = (v + 1 < n ? 1 : 1 - n) * stride;
    o.p2 = (v + 2 < n ? 2 : 2 - n) * stride;
    return o;
}

template <typename T>
__device__ __forceinline__ T psi_prime(T rho, const Thermo& th) {
    const T br = (T)th.b * rho;
    const T om = T(1) - br;
    const T t1 = (T)th.k2RT * log(rho / om);
    const T t2 = (T)th.k2A * log(((T)th.s2m1 + br) / ((T)th.s2p1 - br));
    const T t3 = (T)th.k2RT / om;
    const T t4 = (T)th.k2aal * rho / (T(1) + T(2) * br - br * br);
    return t1 - t2 + t3 - t4;
}

// FP32 arithmetic: hardware reciprocal and logarithm (about one ulp each)
template <>
__device__ __forceinline__ float psi_prime<float>(float rho, const Thermo& th) {
    const float br = (float)th.b * rho;
    const float om = 1.f - br;
    const float iom = __fdividef(1.f, om);
    const float t1 = (float)th.k2RT * __logf(rho * iom);
    const float t2 = (float)th.k2A * __logf(__fdividef((float)th.s2m1 + br, (float)th.s2p1 - br));
    const float t3 = (float)th.k2RT * iom;
    const float t4 = __fdividef((float)th.k2aal * rho, 1.f + 2.f * br - br * br);
    return t1 - t2 + t3 - t4;
}

// fourth-order central differences (Sec. II B) written on differences of
// neighbouring values, which are exact in floating point where the field is smooth
template <typename R>
__device__ __forceinline__ R d1c(R m2, R m1, R p1, R p2) {
    return ((m2 - p2) + R(8) * (p1 - m1)) * R(1.0 / 12.0);
}
template <typename R>
__device__ __forceinline__ R d2c(R m2, R m1, R c, R p1, R p2) {
    return (R(16) * ((m1 - c) + (p1 - c)) - ((m2 - c) + (p2 - c))) * R(1.0 / 12.0);
}

// ---------------------------------------------------------------------------
// gather of the pre-collision populations S_t(x) of a fluid node
// ---------------------------------------------------------------------------
// The context keeps the populations in one of two forms.  Form S (after an
// initial condition or a checkpoint): buffer = S_t, read in place.  Form F*:
// buffer = post-collision populations of the previous step, and Eq. 4 is a
// pull, S_i(x) = f*_i(x - e_i).  A link whose source x - e_i is solid carries
// the missing population of the curved wall: halfway bounce-back
// S_i = f*_j(x) with j = opp(i), or the linear interpolation in the wall
// fraction q of the link from x along e_j, and the difference to f*_j(x) is
// added to S_0 so that the fluid mass is unchanged (Sec. III A).  For q < 1/2
// the interpolation partner is the node behind x; it is used only when its
// population lies within a factor of two of x's own (the same phase).
struct WallBC {
    const uint32_t* nbmask;  // bit j: x + e_j solid (boundary fluid nodes)
    const int* bidx;         // boundary-list index of a boundary fluid node
    const void* q;           // [n_boundary][Q] wall fractions (storage precision)
    int bouzidi;
};

template <class L, typename R, typename C, bool PULL>
__device__ __forceinline__ void gather(const R* __restrict__ f, const Dims& d, long long idx, int x, int y, int z,
                                       uint8_t c, const WallBC& bc, R S[L::Q]) {
    const uint32_t ix = (uint32_t)idx;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) S[i] = at(f + (size_t)i * d.N, ix);
        return;
    }
    // index offsets of x - 1, x, x + 1 along each axis (periodic wrap)
    const int ox[3] = {x >= 1 ? -1 : d.nx - 1, 0, x + 1 < d.nx ? 1 : 1 - d.nx};
    const int oy[3] = {(y >= 1 ? -1 : d.ny - 1) * d.px, 0, (y + 1 < d.ny ? 1 : 1 - d.ny) * d.px};
    const int sz = d.px * d.ny;
    const int oz[3] = {L::D == 3 ? (z >= 1 ? -1 : d.nz - 1) * sz : 0, 0, L::D == 3 ? (z + 1 < d.nz ? 1 : 1 - d.nz) * sz : 0};
    // source x - e_i
#define LBM_SRC(i) (ix + (uint32_t)(ox[1 - L::E[i][0]] + oy[1 - L::E[i][1]] + oz[1 - L::E[i][2]]))
    if (!(c & CLS_BOUNDARY)) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) S[i] = at(f + (size_t)i * d.N, i ? LBM_SRC(i) : ix);
        return;
    }
    const uint32_t bm = bc.nbmask[idx];
    const int k = bc.bouzidi ? bc.bidx[idx] : 0;
    C dm = C(0);
    S[0] = at(f, ix);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::OPP[i];
        if (!(bm & (1u << j))) {
            S[i] = at(f + (size_t)i * d.N, LBM_SRC(i));
            continue;
        }
        const R outj = at(f + (size_t)j * d.N, ix);  // what left x toward the wall
        if (!bc.bouzidi) {
            S[i] = outj;
            continue;
        }
        const C q = (C)((const R*)bc.q)[(size_t)k * L::Q + j];
        C v = (C)outj;
        if (q < C(0.5)) {
            if (!(bm & (1u << i))) {  // x + e_i is the fluid node behind x
                const uint32_t b = ix + (uint32_t)(ox[1 + L::E[i][0]] + oy[1 + L::E[i][1]] + oz[1 + L::E[i][2]]);
                // only a partner of the same phase: its population within a
                // factor of two of x's own (at a contact line the node behind
                // can be across the liquid-gas jump), else the halfway value
                const R fb = at(f + (size_t)j * d.N, b);
                if (fb <= R(2) * outj && outj <= R(2) * fb) v = C(2) * q * (C)outj + (C(1) - C(2) * q) * (C)fb;
            }
        } else {
            v = (C)outj / (C(2) * q) + (C(2) * q - C(1)) / (C(2) * q) * (C)at(f + (size_t)i * d.N, ix);
        }
        S[i] = (R)v;
        dm += (C)outj - v;
    }
#undef LBM_SRC
    if (bc.bouzidi) S[0] = (R)((C)S[0] + dm);
}

// ---------------------------------------------------------------------------
// density (+ liquid centroid on measure steps)
// ---------------------------------------------------------------------------
// rho of a fluid node from its gathered populations; true if liquid
template <class L, typename R, typename C, bool PULL>
__device__ __forceinline__ bool density_node(const R* __restrict__ f, R* __restrict__ rho,
                                             const uint8_t* __restrict__ cls, const Dims& d, const WallBC& bc, int x,
                                             int y, int z, bool in, double rho_m, R inv_b, int* status) {
    if (!in) return false;
    const long long idx = nid(d, x, y, z);
    const uint8_t c = at(cls, (uint32_t)idx);
    if ((c & CLS_MASK) != CLS_FLUID) return false;
    R S[L::Q];
    gather<L, R, C, PULL>(f, d, idx, x, y, z, c, bc, S);
    double s = 0.0;  // summed in double, as the collision's own moments are
#pragma unroll
    for (int i = 0; i < L::Q; ++i) s += (double)S[i];
    const R rs = (R)s;
    at(rho, (uint32_t)idx) = rs;
    if (!(s > 0.0 && s < (double)inv_b)) atomicOr(status, 1);  // also catches NaN
    return (double)rs >= rho_m;  // the stored value, as the crossing search sees it
}

// block reduction (256 threads, 4 waves) of the liquid centroid sums
__device__ __forceinline__ void centroid_reduce(bool liquid, int x, int y, int z, MeasureSlots* ms) {
    __shared__ unsigned long long red[4][4];
    unsigned long long v[4] = {liquid ? 1ull : 0ull, liquid ? (unsigned long long)x : 0ull,
                               liquid ? (unsigned long long)y : 0ull, liquid ? (unsigned long long)z : 0ull};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 4; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (wave == 0 && lane < 4) {
        const unsigned long long sum = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
        if (sum) atomicAdd((&ms->cnt) + lane, sum);
    }
    __syncthreads();
}

template <class L, typename R, typename C, bool PULL>
__global__ void __launch_bounds__(256) k_density(const R* __restrict__ f, R* __restrict__ rho,
                                                 const uint8_t* __restrict__ cls, Dims d, WallBC bc,
                                                 DevCtl* __restrict__ ctl, double rho_m, R inv_b) {
    int x, y, z;
    tile_node(d, x, y, z);
    const bool liquid = density_node<L, R, C, PULL>(f, rho, cls, d, bc, x, y, z, x < d.nx && y < d.ny, rho_m, inv_b,
                                                    &ctl->status);
    if (measuring(ctl)) centroid_reduce(liquid, x, y, z, &ctl->m);
}

// liquid centroid sums of a density field given as such (fluid nodes with
// rho >= rho_m), the sums k_density forms on measure steps: a grid-stride loop
// over the tiles, so that few workgroups add to the four sums (atomics on one
// address serialise)
template <class L, typename R>
__global__ void __launch_bounds__(256) k_centroid(const R* __restrict__ rho, const uint8_t* __restrict__ cls, Dims d,
                                                  double rho_m, MeasureSlots* __restrict__ ms) {
    unsigned long long cnt = 0, sx = 0, sy = 0, sz = 0;
    for (unsigned t = blockIdx.x; t < d.nblocks; t += gridDim.x) {
        int x, y, z;
        tile_coords(d, t, x, y, z);
        if (x < d.nx && y < d.ny) {
            const long long idx = nid(d, x, y, z);
            if ((cls[idx] & CLS_MASK) == CLS_FLUID && (double)rho[idx] >= rho_m) {
                cnt += 1;
                sx += (unsigned long long)x;
                sy += (unsigned long long)y;
                sz += (unsigned long long)z;
            }
        }
    }
    __shared__ unsigned long long red[4][4];
    unsigned long long v[4] = {cnt, sx, sy, sz};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 4; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (wave == 0 && lane < 4) {
        const unsigned long long sum = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
        if (sum) atomicAdd((&ms->cnt) + lane, sum);
    }
}

// state S_t of every node (zero on solid nodes) into out
template <class L, typename R, typename C, bool PULL>
__global__ void __launch_bounds__(256) k_materialize(const R* __restrict__ f, R* __restrict__ out,
                                                     const uint8_t* __restrict__ cls, Dims d, WallBC bc) {
    int x, y, z;
    tile_node(d, x, y, z);
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    const uint8_t c = cls[idx];
    R S[L::Q];
    if ((c & CLS_MASK) == CLS_FLUID) gather<L, R, C, PULL>(f, d, idx, x, y, z, c, bc, S);
    else
        for (int i = 0; i < L::Q; ++i) S[i] = R(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[(size_t)i * d.N + idx] = S[i];
}

// ---------------------------------------------------------------------------
// Eq. 14 over a compact list: rho(s) = sum_i w_i rho(s+e_i) s_w / sum_i w_i s_w
// ---------------------------------------------------------------------------
template <class L, typename R, typename C>
__device__ __forceinline__ void fill_entry(long long idx, uint32_t m, R inv_den, R* __restrict__ rho, const Dims& d) {
    // coordinates by 32-bit divisions (a lattice holds fewer than 2^32 nodes;
    // the 64-bit ones cost more than the rest of the entry)
    const uint32_t loc = (uint32_t)(idx - d.off), row = loc / (uint32_t)d.px;
    const int x = (int)(loc - row * (uint32_t)d.px), y = (int)(row % (uint32_t)d.ny), z = (int)(row / (uint32_t)d.ny);
    C num = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (m & (1u << i)) {
            const int X = wrapc(x + L::E[i][0], d.nx), Y = wrapc(y + L::E[i][1], d.ny);
            const int Z = L::D == 3 ? wrapc(z + L::E[i][2], d.nz) : 0;
            num += C(L::w(i)) * (C)rho[nid(d, X, Y, Z)];
        }
    }
    rho[idx] = (R)(num * (C)inv_den);
}

template <class L, typename R, typename C = R>
__global__ void __launch_bounds__(256) k_fill(const long long* __restrict__ node, const uint32_t* __restrict__ mask,
                                              const R* __restrict__ inv_den, int count, R* __restrict__ rho, Dims d) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    fill_entry<L, R, C>(node[k], mask[k], inv_den[k], rho, d);
}

// ---------------------------------------------------------------------------
// measurement helpers (double precision, shared by k_mu and k_finalize)
// ---------------------------------------------------------------------------
struct Frame {
    double a[3], b1[3], b2[3];
    bool ok;
};

// frame about the unit drop axis a: b1 = the lattice axis least aligned with
// a (compared on a 1/1024 grid), orthogonalised; b2 = a x b1
__device__ inline Frame frame_from_axis(const double a[3], int dim) {
    Frame F;
    F.ok = true;
    int kb = 0;
    long long best = 1ll << 40;
    for (int k = 0; k < dim; ++k) {
        long long qv = llround(fabs(a[k]) * 1024.0);
        if (qv < best) { best = qv; kb = k; }
    }
    double b[3] = {0, 0, 0};
    b[kb] = 1.0;
    const double ab = a[kb];
    for (int k = 0; k < 3; ++k) b[k] -= ab * a[k];
    const double bn = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    for (int k = 0; k < 3; ++k) { F.a[k] = a[k]; F.b1[k] = b[k] / bn; }
    F.b2[0] = a[1] * F.b1[2] - a[2] * F.b1[1];
    F.b2[1] = a[2] * F.b1[0] - a[0] * F.b1[2];
    F.b2[2] = a[0] * F.b1[1] - a[1] * F.b1[0];
    return F;
}

// frame of a measurement: the axis from the substrate centre to the liquid centroid
__device__ inline Frame make_frame(const MeasureSlots* ms, const MeasureParams& mp) {
    const unsigned long long n = ms->cnt;
    double G[3] = {0, 0, 0};
    if (n) {
        G[0] = (double)ms->sx / (double)n;
        G[1] = (double)ms->sy / (double)n;
        G[2] = mp.dim == 3 ? (double)ms->sz / (double)n : 0.0;
    }
    double a[3] = {G[0] - mp.c[0], G[1] - mp.c[1], mp.dim == 3 ? G[2] - mp.c[2] : 0.0};
    double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (an > 0) {
        a[0] /= an; a[1] /= an; a[2] /= an;
    } else {
        a[0] = 0; a[1] = mp.dim == 2 ? 1.0 : 0.0; a[2] = mp.dim == 2 ? 0.0 : 1.0;
    }
    Frame F = frame_from_axis(a, mp.dim);
    F.ok = n > 0;
    return F;
}

__device__ inline int sector_of(const double r[3], const Frame& F, int dim, int ns) {
    const double r1 = r[0] * F.b1[0] + r[1] * F.b1[1] + r[2] * F.b1[2];
    if (dim == 2) return r1 >= 0.0 ? 0 : 1;
    const double r2 = r[0] * F.b2[0] + r[1] * F.b2[1] + r[2] * F.b2[2];
    const double psi = atan2(r2, r1);
    int s = (int)floor((psi + M_PI) / (2.0 * M_PI) * ns);
    if (s >= ns) s -= ns;
    if (s < 0) s = 0;
    return s;
}

// crossing point of Eq. 15 on the link from gas node (x,y,z) along e
__device__ inline void crossing_point(double rho_g_node, double rho_l_node, double rho_m, int x, int y, int z,
                                      int ex, int ey, int ez, double p[3]) {
    const double t = (rho_m - rho_g_node) / (rho_l_node - rho_g_node);
    p[0] = x + t * ex;
    p[1] = y + t * ey;
    p[2] = z + t * ez;
}

// ---------------------------------------------------------------------------
// chemical potential (+ fused crossing search on measure steps)
// ---------------------------------------------------------------------------
template <class L, typename R, typename C, bool SC = false>
__device__ __forceinline__ bool mu_node(const R* __restrict__ rho, R* __restrict__ mu, const uint8_t* __restrict__ cls,
                                        const Dims& d, const Thermo& th, int x, int y, int z, bool in, R& r0) {
    r0 = R(0);
    if (!in) return false;
    if constexpr (SC) {
        // pseudopotential model: psi(rho) = 1 - exp(-rho) on fluid nodes
        const long long idx = nid(d, x, y, z);
        if ((cls[idx] & CLS_MASK) != CLS_FLUID) return false;
        r0 = rho[idx];
        mu[idx] = (R)(C(1) - exp(-(C)r0));
        return true;
    }
    // the class and the density stencil are loaded together (every offset is
    // in bounds: periodic images), and the class decides only the store
    const long long idx = nid(d, x, y, z);
    const uint32_t ix = (uint32_t)idx;
    const uint8_t c = at(cls, ix);
    const R rc = at(rho, ix);
    const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
    auto p = [&](int o) { return (C)at(rho, ix + (uint32_t)o); };
    const C c0 = (C)rc;
    C lap = d2c<C>(p(ox.m2), p(ox.m1), c0, p(ox.p1), p(ox.p2));
    lap += d2c<C>(p(oy.m2), p(oy.m1), c0, p(oy.p1), p(oy.p2));
    if (L::D == 3) {
        const Nbr oz = nbr_offsets(z, d.nz, d.px * d.ny);
        lap += d2c<C>(p(oz.m2), p(oz.m1), c0, p(oz.p1), p(oz.p2));
    }
    const C m = (psi_prime<C>(c0, th) - (C)th.mu_ref) - (C)th.kappa * lap;
    asm volatile("" : : "v"(m));  // keeps the loads above the class test
    if ((c & CLS_MASK) != CLS_FLUID) return false;
    r0 = rc;
    at(mu, ix) = (R)m;
    return true;
}

// gas-side fluid nodes near the substrate test their links for an isodensity
// crossing (Eq. 15) and offer it to the per-(sector, band) minimum.  Called by
// every lane of the wave (the ballot skips waves away from the contact region).
template <class L, typename R>
__device__ __forceinline__ void crossings_node(const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                               const Dims& d, int x, int y, int z, bool fluid, R r0,
                                               const MeasureParams& mp, MeasureSlots* ms,
                                               unsigned long long (*lkeys)[2] = nullptr) {
    bool cand = false;
    if (fluid && (double)r0 < mp.rho_m) {
        // crossings lie within sqrt(2) of the node and the bands end 2.5 from
        // the substrate, so only nodes within 4 of it can contribute; tested on
        // the squared distance in single precision, with half a node to spare
        const float rx = (float)(x - mp.c[0]), ry = (float)(y - mp.c[1]);
        const float rz = (L::D == 3) ? (float)(z - mp.c[2]) : 0.f;
        const float rr = rx * rx + ry * ry + rz * rz;
        const float hi = (float)mp.R + 4.5f, lo = fmaxf((float)mp.R - 4.5f, 0.f);
        cand = mp.concave ? rr > lo * lo : rr < hi * hi;
    }
    if (__ballot(cand) == 0) return;
    if (!cand) return;
    const Frame F = make_frame(ms, mp);
    if (!F.ok) return;
    const long long idx = nid(d, x, y, z), loc = idx - d.off;
    // the class and density of every lattice neighbour, loaded together (the
    // tests below would otherwise wait for them one link at a time)
    uint8_t cj[L::Q];
    R rj[L::Q];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int X = wrapc(x + L::E[i][0], d.nx), Y = wrapc(y + L::E[i][1], d.ny);
        const int Z = L::D == 3 ? wrapc(z + L::E[i][2], d.nz) : 0;
        const long long j = nid(d, X, Y, Z);
        cj[i] = cls[j];
        rj[i] = rho[j];
    }
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if ((cj[i] & CLS_MASK) != CLS_FLUID) continue;
        const double rl = (double)rj[i];
        if (!(rl >= mp.rho_m)) continue;
        double p[3];
        crossing_point((double)r0, rl, mp.rho_m, x, y, z, L::E[i][0], L::E[i][1], L::E[i][2], p);
        const double r[3] = {p[0] - mp.c[0], p[1] - mp.c[1], p[2] - mp.c[2]};
        const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const double dist = mp.concave ? mp.R - rn : rn - mp.R;  // distance from the substrate
        if (!(dist >= 0.5 && dist < 2.5)) continue;
        const int band = dist < 1.5 ? 1 : 2;
        const int s = sector_of(r, F, mp.dim, mp.n_sectors);
        const float kv = (float)fabs(dist - (double)band);
        // link id within the lattice: ties go to the lower node, then the lower direction
        const unsigned long long key =
            ((unsigned long long)__float_as_uint(kv) << 32) | (unsigned long long)(loc * L::Q + i);
        if (lkeys) atomicMin(&lkeys[s][band - 1], key);  // the workgroup's table in LDS
        else atomicMin(&ms->keys[s][band - 1], key);
    }
}

template <class L, typename R, typename C, bool SC = false, bool ZCH = false>
__global__ void __launch_bounds__(256) k_mu(const R* __restrict__ rho, R* __restrict__ mu,
                                            const uint8_t* __restrict__ cls, Dims d, Thermo th) {
    int x, y, z;
    R r0;
    if constexpr (ZCH) {
        tile_node_zc(d, x, y, z);
        const int z1 = z + d.zc < d.nz ? z + d.zc : d.nz;
        for (; z < z1; ++z) (void)mu_node<L, R, C, SC>(rho, mu, cls, d, th, x, y, z, x < d.nx && y < d.ny, r0);
    } else {
        tile_node(d, x, y, z);
        (void)mu_node<L, R, C, SC>(rho, mu, cls, d, th, x, y, z, x < d.nx && y < d.ny, r0);
    }
}

// Tiles that can hold a node within 4 of the substrate: the box |x - c| <
// R + 5 per axis (unwrapped coordinates, as the distance of Sec. III B),
// clamped to the lattice, in whole tiles.
struct TileBox {
    unsigned tx0, ty0, z0, ntx, nty, n;
};
__device__ __forceinline__ TileBox cand_box(const Dims& d, const MeasureParams& mp) {
    const double m = mp.R + 5.0;
    const int nn[3] = {d.nx, d.ny, d.nz};
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double l = floor(mp.c[a] - m), h = ceil(mp.c[a] + m);
        lo[a] = l < 0.0 ? 0 : (l > nn[a] - 1 ? nn[a] - 1 : (int)l);
        hi[a] = h > nn[a] - 1 ? nn[a] - 1 : (h < 0.0 ? 0 : (int)h);
    }
    const int th = 256 >> d.tws;
    TileBox b;
    b.tx0 = (unsigned)(lo[0] >> d.tws);
    b.ty0 = (unsigned)(lo[1] / th);
    b.z0 = (unsigned)lo[2];
    b.ntx = (unsigned)(hi[0] >> d.tws) - b.tx0 + 1u;
    b.nty = (unsigned)(hi[1] / th) - b.ty0 + 1u;
    b.n = b.ntx * b.nty * (unsigned)(hi[2] - lo[2] + 1);
    return b;
}

// The crossing search of a measure step (Sec. III B), its own launch so that
// the mu kernel carries none of its code: a grid-stride loop over the tiles
// of the box around the substrate that returns at once on steps that do not
// measure.  (The keys are minima, so the order of the scan does not matter.)
// The keys go to a table in LDS first and the workgroup's minima to the
// context's slots once at the end: many links of one contact line compete for
// the same few keys, and atomics on one address in device memory serialise.
template <class L, typename R>
__global__ void __launch_bounds__(256) k_cross(const R* __restrict__ rho, const uint8_t* __restrict__ cls, Dims d,
                                               DevCtl* __restrict__ ctl, MeasureParams mp) {
    if (!measuring(ctl)) return;
    __shared__ unsigned long long lkeys[64][2];
    if (threadIdx.x < 128) lkeys[threadIdx.x >> 1][threadIdx.x & 1] = ~0ull;
    __syncthreads();
    const TileBox b = cand_box(d, mp);
    for (unsigned t = blockIdx.x; t < b.n; t += gridDim.x) {
        const unsigned txi = b.tx0 + t % b.ntx, rest = t / b.ntx;
        const unsigned tyi = b.ty0 + rest % b.nty;
        const int x = (int)(txi << d.tws) + (int)(threadIdx.x & ((1u << d.tws) - 1u));
        const int y = (int)tyi * (256 >> d.tws) + (int)(threadIdx.x >> d.tws);
        const int z = (int)(b.z0 + rest / b.nty);
        bool fluid = false;
        R r0 = R(0);
        if (x < d.nx && y < d.ny) {
            const long long idx = nid(d, x, y, z);
            fluid = (cls[idx] & CLS_MASK) == CLS_FLUID;
            if (fluid) r0 = rho[idx];
        }
        crossings_node<L, R>(rho, cls, d, x, y, z, fluid, r0, mp, &ctl->m, lkeys);
    }
    __syncthreads();
    if (threadIdx.x < 128) {
        const unsigned long long k = lkeys[threadIdx.x >> 1][threadIdx.x & 1];
        if (k != ~0ull) atomicMin(&ctl->m.keys[threadIdx.x >> 1][threadIdx.x & 1], k);
    }
}

// ---------------------------------------------------------------------------
// collision (streaming is the pull at the start of the next step)
// ---------------------------------------------------------------------------
template <class L, typename R, typename C, bool MRT, bool NT>
__device__ __forceinline__ void collide_apply(const R S[L::Q], C Fx, C Fy, C Fz, const Collision<C>& cp,
                                              R* __restrict__ fout, long long idx, long long N);

// offset of the lattice neighbour x + e along one axis (e in {-1, 0, 1})
__device__ __forceinline__ long long step_off(int e, const Nbr& o) { return e < 0 ? o.m1 : (e > 0 ? o.p1 : 0); }

// Shan-Chen interaction of the pseudopotential model with the lattice
// weights, F = -G psi(x) sum_i w_i psi(x + e_i) e_i, in double precision;
// psi of fluid and solid-layer nodes is in the buffer passed as psi
template <class L, typename R>
__device__ __forceinline__ void sc_force(const R* __restrict__ psi, long long idx, const Nbr& ox, const Nbr& oy,
                                         const Nbr& oz, double G, double& Fx, double& Fy, double& Fz) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        long long o = step_off(L::E[i][0], ox) + step_off(L::E[i][1], oy);
        if (L::D == 3) o += step_off(L::E[i][2], oz);
        const double v = L::w(i) * (double)psi[idx + o];
        sx += v * L::E[i][0];
        sy += v * L::E[i][1];
        sz += v * L::E[i][2];
    }
    const double p0 = (double)psi[idx];
    Fx = -G * p0 * sx;
    Fy = -G * p0 * sy;
    Fz = -G * p0 * sz;
}

// Force at a node: Eq. 7 with fourth-order central differences (or the
// pseudopotential interaction), plus the body force from step g_start.  The
// stencil loads need no class: every offset is in bounds (periodic images).
// Formed in double whatever the storage and arithmetic types: the fourth-order
// differences of the density span the jump across an interface (a factor of
// up to 40 between neighbours), where single precision would leave an error of
// order 1e-7 in F that is the same step after step, so the interface would
// drift; and the two terms of Eq. 7 cancel almost exactly inside an interface
// at rest.  F is then rounded to the arithmetic type C.
template <class L, typename R, typename C, bool SC>
__device__ __forceinline__ void force_at(const R* __restrict__ rho, const R* __restrict__ mu, const Dims& d,
                                         long long idx, int x, int y, int z, const Collision<C>& cp, long long t,
                                         C& Fx, C& Fy, C& Fz) {
    const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
    if constexpr (SC) {
        const Nbr oz = L::D == 3 ? nbr_offsets(z, d.nz, d.px * d.ny) : Nbr{0, 0, 0, 0};
        double fx, fy, fz;
        sc_force<L, R>(mu, idx, ox, oy, oz, cp.sc_G, fx, fy, fz);
        if (t >= cp.g_start) {
            const double r0 = (double)rho[idx];
            fx += r0 * (double)cp.g[0];
            fy += r0 * (double)cp.g[1];
            fz += r0 * (double)cp.g[2];
        }
        Fx = (C)fx;
        Fy = (C)fy;
        Fz = (C)fz;
        return;
    }
    typedef double D;
    const uint32_t ix = (uint32_t)idx;
    auto pr = [&](int o) { return (D)at(rho, ix + (uint32_t)o); };
    auto pm = [&](int o) { return (D)at(mu, ix + (uint32_t)o); };
    const D r0 = pr(0);
    const D gmx = d1c<D>(pm(ox.m2), pm(ox.m1), pm(ox.p1), pm(ox.p2));
    const D grx = d1c<D>(pr(ox.m2), pr(ox.m1), pr(ox.p1), pr(ox.p2));
    const D gmy = d1c<D>(pm(oy.m2), pm(oy.m1), pm(oy.p1), pm(oy.p2));
    const D gry = d1c<D>(pr(oy.m2), pr(oy.m1), pr(oy.p1), pr(oy.p2));
    D gmz = D(0), grz = D(0);
    if (L::D == 3) {
        const Nbr oz = nbr_offsets(z, d.nz, d.px * d.ny);
        gmz = d1c<D>(pm(oz.m2), pm(oz.m1), pm(oz.p1), pm(oz.p2));
        grz = d1c<D>(pr(oz.m2), pr(oz.m1), pr(oz.p1), pr(oz.p2));
    }
    const D third = D(1.0 / 3.0);
    D fx = -r0 * gmx + grx * third;
    D fy = -r0 * gmy + gry * third;
    D fz = -r0 * gmz + grz * third;
    if (t >= cp.g_start) {
        fx += r0 * (D)cp.g[0];
        fy += r0 * (D)cp.g[1];
        fz += r0 * (D)cp.g[2];
    }
    Fx = (C)fx;
    Fy = (C)fy;
    Fz = (C)fz;
}

// The force of every node into F ([3][N], storage precision) for the one-pass
// step: Eq. 7 (or the pseudopotential interaction) plus the body force of
// step t; F of solid nodes is written but never read.  z-chunked as k_mu, so
// that a workgroup's stencil planes are the ones it read an iteration before,
// and software-pipelined: plane z+1's stencil is loaded before plane z's
// force is stored (a wave's loads and stores share one in-order counter, so
// loads issued after the stores would wait for them).
template <class L, typename R>
struct ForceStencil {
    static constexpr int K = 25;  // rho: centre and 12 axis neighbours; mu (or psi): 12 axis neighbours
    R v[K];
};

template <class L, typename R, bool SC>
__device__ __forceinline__ void force_stencil_load(const R* __restrict__ rho, const R* __restrict__ mu, const Dims& d,
                                                   int x, int y, int z, ForceStencil<L, R>& s) {
    const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
    const Nbr oz = L::D == 3 ? nbr_offsets(z, d.nz, d.px * d.ny) : Nbr{0, 0, 0, 0};
    if constexpr (SC) {
        const long long idx = nid(d, x, y, z);
        // psi at the lattice neighbours, rho at the node
        s.v[0] = rho[idx];
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            long long o = step_off(L::E[i][0], ox) + step_off(L::E[i][1], oy);
            if (L::D == 3) o += step_off(L::E[i][2], oz);
            s.v[i] = mu[idx + o];
        }
        s.v[L::Q] = mu[idx];
        return;
    }
    const Nbr ax[3] = {ox, oy, oz};
    const uint32_t ix = nid32(d, x, y, z);
    s.v[0] = at(rho, ix);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool on = a < L::D;
        const Nbr& o = ax[a];
        const uint32_t i2 = on ? ix + (uint32_t)o.m2 : ix, i1 = on ? ix + (uint32_t)o.m1 : ix;
        const uint32_t j1 = on ? ix + (uint32_t)o.p1 : ix, j2 = on ? ix + (uint32_t)o.p2 : ix;
        s.v[1 + 4 * a] = at(rho, i2);
        s.v[2 + 4 * a] = at(rho, i1);
        s.v[3 + 4 * a] = at(rho, j1);
        s.v[4 + 4 * a] = at(rho, j2);
        s.v[13 + 4 * a] = at(mu, i2);
        s.v[14 + 4 * a] = at(mu, i1);
        s.v[15 + 4 * a] = at(mu, j1);
        s.v[16 + 4 * a] = at(mu, j2);
    }
}

template <class L, typename R, typename C, bool SC>
__device__ __forceinline__ void force_from_stencil(const ForceStencil<L, R>& s, const Collision<C>& cp, long long t,
                                                   C& Fx, C& Fy, C& Fz) {
    // in double, as force_at
    typedef double D;
    const D r0 = (D)s.v[0];
    D fx, fy, fz;
    if constexpr (SC) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const double v = L::w(i) * (double)s.v[i];
            sx += v * L::E[i][0];
            sy += v * L::E[i][1];
            sz += v * L::E[i][2];
        }
        const double p0 = (double)s.v[L::Q];
        fx = -cp.sc_G * p0 * sx;
        fy = -cp.sc_G * p0 * sy;
        fz = -cp.sc_G * p0 * sz;
    } else {
        D gr[3], gm[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gr[a] = d1c<D>((D)s.v[1 + 4 * a], (D)s.v[2 + 4 * a], (D)s.v[3 + 4 * a], (D)s.v[4 + 4 * a]);
            gm[a] = d1c<D>((D)s.v[13 + 4 * a], (D)s.v[14 + 4 * a], (D)s.v[15 + 4 * a], (D)s.v[16 + 4 * a]);
        }
        const D third = D(1.0 / 3.0);
        fx = -r0 * gm[0] + gr[0] * third;
        fy = -r0 * gm[1] + gr[1] * third;
        fz = L::D == 3 ? -r0 * gm[2] + gr[2] * third : D(0);
    }
    if (t >= cp.g_start) {
        fx += r0 * (D)cp.g[0];
        fy += r0 * (D)cp.g[1];
        fz += r0 * (D)cp.g[2];
    }
    Fx = (C)fx;
    Fy = (C)fy;
    Fz = (C)fz;
}

template <class L, typename R, typename C, bool SC>
__global__ void __launch_bounds__(256) k_force(const R* __restrict__ rho, const R* __restrict__ mu,
                                               const uint8_t* __restrict__ cls, Dims d, Collision<C> cp,
                                               const DevCtl* __restrict__ ctl, R* __restrict__ F) {
    (void)cls;
    int x, y, z0;
    tile_node_zc(d, x, y, z0);
    if (x >= d.nx || y >= d.ny) return;
    const int z1 = z0 + d.zc < d.nz ? z0 + d.zc : d.nz;
    const long long t = ctl->t;
    ForceStencil<L, R> cur, nxt;
    force_stencil_load<L, R, SC>(rho, mu, d, x, y, z0, cur);
    for (int z = z0; z < z1; ++z) {
        force_stencil_load<L, R, SC>(rho, mu, d, x, y, z + 1 < z1 ? z + 1 : z, nxt);  // unconditional: counted
        C Fx, Fy, Fz;
        force_from_stencil<L, R, C, SC>(cur, cp, t, Fx, Fy, Fz);
        const uint32_t ix = (uint32_t)nid(d, x, y, z);
        at(F, ix) = (R)Fx;
        at(F + d.N, ix) = (R)Fy;
        at(F + 2 * d.N, ix) = (R)Fz;
#pragma unroll
        for (int k = 0; k < ForceStencil<L, R>::K; ++k) cur.v[k] = nxt.v[k];
    }
}

template <class L, typename R, typename C, bool PULL, bool MRT, bool NT = false, bool SC = false>
__device__ __forceinline__ void collide_node(const R* __restrict__ fin, R* __restrict__ fout,
                                             const R* __restrict__ rho, const R* __restrict__ mu,
                                             const uint8_t* __restrict__ cls, const Dims& d, const WallBC& bc,
                                             const Collision<C>& cp, long long t, int x, int y, int z) {
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    const uint8_t c = at(cls, (uint32_t)idx);
    // the force is formed before the class test so that its stencil loads go
    // out with the class load
    C Fx, Fy, Fz;
    force_at<L, R, C, SC>(rho, mu, d, idx, x, y, z, cp, t, Fx, Fy, Fz);
    asm volatile("" : : "v"(Fx), "v"(Fy), "v"(Fz));  // keeps the loads above the class test
    if ((c & CLS_MASK) != CLS_FLUID) return;
    R S[L::Q];
    gather<L, R, C, PULL>(fin, d, idx, x, y, z, c, bc, S);
    collide_apply<L, R, C, MRT, NT>(S, Fx, Fy, Fz, cp, fout, idx, d.N);
}

// Collision of one fluid node from its gathered populations S and the force
// F (Eq. 7, plus the body force): MRT or BGK relaxation with exact-difference
// forcing; post-collision populations stored at the node, o[i * N].
// A store of one post-collision population: non-temporal (NT) where the
// lattice is swept in whole aligned rows, so that the stream does not evict
// the density and chemical-potential planes the stencils re-read (the
// populations are next read one step later, after the whole lattice has
// passed through the caches).  The batched solver pads every row to 64 nodes
// for this: with ragged, unaligned rows NT stores turn into partial-line
// writes and cost more than they save.
template <bool NT, typename R>
__device__ __forceinline__ void put(R* p, R v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Second-order equilibrium (Eq. 2) of every direction for density rs and
// velocity a, formed per pair of opposite directions: w rs (1 + 4.5 (e.a)^2 -
// 1.5 a.a) plus and minus 3 w rs e.a.
template <class L, typename C>
__device__ __forceinline__ void feq_all(C rs, C ax, C ay, C az, C out[L::Q]) {
    const C aa = ax * ax + ay * ay + az * az;
    out[0] = rs * C(L::w(0)) * (C(1) - C(1.5) * aa);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::OPP[i] < i) continue;
        const C ea = C(L::E[i][0]) * ax + C(L::E[i][1]) * ay + C(L::E[i][2]) * az;
        const C wr = rs * C(L::w(i));
        const C sym = wr * (C(1) + C(4.5) * ea * ea - C(1.5) * aa);
        const C anti = wr * C(3) * ea;
        out[i] = sym + anti;
        out[L::OPP[i]] = sym - anti;
    }
}

// The post-collision populations of one node into fo (storage type).
template <class L, typename R, typename C, bool MRT>
__device__ __forceinline__ void collide_values(const R S[L::Q], C Fx, C Fy, C Fz, const Collision<C>& cp,
                                               R fo[L::Q]) {
    // the density moment of S (Eq. 2 argument) in double: the rest population
    // below takes the remainder of it
    double rd = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) rd += (double)S[i];
    C rs, ux, uy, uz, vx, vy, vz;
    if constexpr (sizeof(C) == 8) {
        typedef double D;
        D jx = D(0), jy = D(0), jz = D(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const D fi = (D)S[i];
            if (L::E[i][0]) jx += D(L::E[i][0]) * fi;
            if (L::E[i][1]) jy += D(L::E[i][1]) * fi;
            if (L::E[i][2]) jz += D(L::E[i][2]) * fi;
        }
        const D ird = D(1) / rd;
        rs = (C)rd;
        ux = (C)(jx * ird), uy = (C)(jy * ird), uz = (C)(jz * ird);
        vx = (C)((jx + Fx) * ird), vy = (C)((jy + Fy) * ird), vz = (C)((jz + Fz) * ird);  // u + F/rho (Eq. 13)
    } else {
        // FP32 arithmetic: the momentum from the differences of opposite
        // populations, which are exact where the two differ by less than a
        // factor of two (the populations near equilibrium), and 1 / rho from
        // the hardware reciprocal (1 ulp)
        C jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            if (L::OPP[i] < i) continue;
            const C df = (C)S[i] - (C)S[L::OPP[i]];
            if (L::E[i][0]) jx += C(L::E[i][0]) * df;
            if (L::E[i][1]) jy += C(L::E[i][1]) * df;
            if (L::E[i][2]) jz += C(L::E[i][2]) * df;
        }
        rs = (C)rd;
        const C ir = __builtin_amdgcn_rcpf(rs);
        ux = jx * ir, uy = jy * ir, uz = jz * ir;
        vx = (jx + Fx) * ir, vy = (jy + Fy) * ir, vz = (jz + Fz) * ir;  // u + F/rho (Eq. 13)
    }

    // With FP32 arithmetic the lattice weights are rounded (1/3, 1/18 and 1/36
    // in binary32 sum to 1 + 1.5e-8), so every collision would add that share
    // of the density to the node: a systematic drift of 1.5e-8 per step.  The
    // collision conserves mass exactly (Eq. 1: the density moment is not
    // relaxed and the forcing term has no mass), so the rest population takes
    // the remainder rho - sum_{i>0} f*_i of the stored values, in double.
    constexpr bool kRestRemainder = sizeof(C) == 4;
    double srest = 0.0;
    if (!MRT) {
        // BGK (Eq. 3) + exact-difference forcing (Eq. 13) with feq2 = f_eq(rho, u + F / rho):
        // f* = f - (f - feq) / tau + feq2 - feq = feq2 + (1 - 1/tau) (f - feq),
        // which for tau = 1 is feq2 alone (a uniform branch).  Per pair of
        // opposite directions, as feq_all forms them.
        const C om1 = C(1) - cp.omega;
        const bool relax = om1 != C(0);
        const C uu = ux * ux + uy * uy + uz * uz, vv = vx * vx + vy * vy + vz * vz;
        auto put2 = [&](int i, C v) {
            const R r = (R)v;
            if (kRestRemainder && i != 0) srest += (double)r;
            fo[i] = r;
        };
        {
            const C w0 = rs * C(L::w(0));
            C v0 = w0 * (C(1) - C(1.5) * vv);
            if (relax) v0 += om1 * ((C)S[0] - w0 * (C(1) - C(1.5) * uu));
            put2(0, v0);
        }
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            if (L::OPP[i] < i) continue;
            const int j = L::OPP[i];
            const C wr = rs * C(L::w(i));
            const C ev = C(L::E[i][0]) * vx + C(L::E[i][1]) * vy + C(L::E[i][2]) * vz;
            const C sym2 = wr * (C(1) + C(4.5) * ev * ev - C(1.5) * vv), anti2 = wr * C(3) * ev;
            C vi = sym2 + anti2, vj = sym2 - anti2;
            if (relax) {
                const C eu = C(L::E[i][0]) * ux + C(L::E[i][1]) * uy + C(L::E[i][2]) * uz;
                const C sym = wr * (C(1) + C(4.5) * eu * eu - C(1.5) * uu), anti = wr * C(3) * eu;
                vi += om1 * ((C)S[i] - (sym + anti));
                vj += om1 * ((C)S[j] - (sym - anti));
            }
            put2(i, vi);
            put2(j, vj);
        }
        if (kRestRemainder) fo[0] = (R)(rd - srest);
    } else {
        // MRT (Eq. 1): non-conserved moments of f - f_eq relaxed by s_k and
        // mapped back with M^T D^-1, plus the forcing term
        C dev[L::Q], out[L::Q], feq[L::Q], feq2[L::Q];
        feq_all<L, C>(rs, ux, uy, uz, feq);
        feq_all<L, C>(rs, vx, vy, vz, feq2);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            dev[i] = (C)S[i] - feq[i];
            out[i] = (C)S[i] + (feq2[i] - feq[i]);
        }
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            if (L::kind(k) == 0) continue;
            C mk = C(0);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const double mki = L::m(k, i);
                if (mki != 0.0) mk += C(mki) * dev[i];
            }
            const C ck = mk * cp.rate[k];
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const double mki = L::m(k, i);
                if (mki != 0.0) out[i] -= C(mki) * ck;
            }
        }
#pragma unroll
        for (int i = kRestRemainder ? 1 : 0; i < L::Q; ++i) {
            const R v = (R)out[i];
            if (kRestRemainder) srest += (double)v;
            fo[i] = v;
        }
        if (kRestRemainder) fo[0] = (R)(rd - srest);
    }
}

// Collision of one node with its post-collision populations stored at the
// node, o[i * N] (aligned stores; streaming is the next step's pull).
template <class L, typename R, typename C, bool MRT, bool NT>
__device__ __forceinline__ void collide_apply(const R S[L::Q], C Fx, C Fy, C Fz, const Collision<C>& cp,
                                              R* __restrict__ fout, long long idx, long long N) {
    R fo[L::Q];
    collide_values<L, R, C, MRT>(S, Fx, Fy, Fz, cp, fo);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) put<NT>(&at(fout + (size_t)i * N, (uint32_t)idx), fo[i]);
}

template <class L, typename R, typename C, bool PULL, bool MRT, bool SC = false>
__global__ void __launch_bounds__(256) k_collide(const R* __restrict__ fin, R* __restrict__ fout,
                                                 const R* __restrict__ rho, const R* __restrict__ mu,
                                                 const uint8_t* __restrict__ cls, Dims d, WallBC bc,
                                                 Collision<C> cp, const DevCtl* __restrict__ ctl) {
    int x, y, z;
    tile_node(d, x, y, z);
    collide_node<L, R, C, PULL, MRT, true, SC>(fin, fout, rho, mu, cls, d, bc, cp, ctl->t, x, y, z);
}

// ---------------------------------------------------------------------------
// finalize: contact angles from the selected crossings; clear; advance t
// ---------------------------------------------------------------------------
// One lattice's contact angles from its selected crossings (64 threads, one
// per sector).  Writes the record to *last (and *rec2 if not null) and clears
// the slots for the next measurement.
template <class L, typename R>
__device__ void finalize_slots(const R* __restrict__ rho, const Dims& d, const MeasureParams& mp,
                               MeasureSlots* __restrict__ ms, long long t, AngleRec* __restrict__ last,
                               AngleRec* __restrict__ rec2) {
    const int s = threadIdx.x;
    __shared__ double th[64];
    __shared__ double cpt[64][3];
    const Frame F = make_frame(ms, mp);
    double theta = NAN, cp3[3] = {NAN, NAN, NAN};
    if (F.ok && s < mp.n_sectors) {
        const unsigned long long k1 = ms->keys[s][0], k2 = ms->keys[s][1];
        if (k1 != ~0ull && k2 != ~0ull) {
            double P[2][3];
            const unsigned long long ks[2] = {k1, k2};
            for (int b = 0; b < 2; ++b) {
                const unsigned long long id = ks[b] & 0xffffffffull;
                const long long loc = (long long)(id / L::Q);
                const int i = (int)(id % L::Q);
                int ex = 0, ey = 0, ez = 0;
#pragma unroll
                for (int q = 0; q < L::Q; ++q)
                    if (q == i) { ex = L::E[q][0]; ey = L::E[q][1]; ez = L::E[q][2]; }
                const int x = (int)(loc % d.px), y = (int)((loc / d.px) % d.ny);
                const int z = (int)(loc / ((long long)d.px * d.ny));
                const int X = wrapc(x + ex, d.nx), Y = wrapc(y + ey, d.ny);
                const int Z = L::D == 3 ? wrapc(z + ez, d.nz) : 0;
                crossing_point((double)rho[d.off + loc], (double)rho[nid(d, X, Y, Z)], mp.rho_m, x, y, z, ex, ey, ez,
                               P[b]);
            }
            // meridional coordinates (w: distance from the drop axis, s: along it)
            double r1[3], r2[3];
            for (int k = 0; k < 3; ++k) { r1[k] = P[0][k] - mp.c[k]; r2[k] = P[1][k] - mp.c[k]; }
            const double s1 = r1[0] * F.a[0] + r1[1] * F.a[1] + r1[2] * F.a[2];
            const double s2 = r2[0] * F.a[0] + r2[1] * F.a[1] + r2[2] * F.a[2];
            double q1[3], q2[3];
            for (int k = 0; k < 3; ++k) { q1[k] = r1[k] - s1 * F.a[k]; q2[k] = r2[k] - s2 * F.a[k]; }
            const double w1 = sqrt(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2]);
            const double w2 = sqrt(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2]);
            const double dw = w2 - w1, ds = s2 - s1;
            const double A = dw * dw + ds * ds;
            if (A > 0.0) {
                // secant P1 + lam (P2 - P1) meets the substrate circle |.| = R
                const double B = w1 * dw + s1 * ds;
                const double C = w1 * w1 + s1 * s1 - mp.R * mp.R;
                const double disc = B * B - A * C;
                double lam;
                if (disc >= 0.0) {
                    const double sq = sqrt(disc);
                    const double lp = (-B + sq) / A, lm = (-B - sq) / A;
                    lam = lp <= 0.0 ? lp : lm;  // nearest hit behind P1, else the first one ahead
                } else {
                    lam = -B / A;  // no intersection: closest approach
                }
                const double w0 = w1 + lam * dw, s0 = s1 + lam * ds;
                const double r0 = sqrt(w0 * w0 + s0 * s0);
                const double ew = w0 / r0, es = s0 / r0;      // outward radial direction
                const double tw = -es, ts = ew;               // tangent toward the drop axis
                // substrate normal into the fluid
                const double nw = mp.concave ? -ew : ew, ns = mp.concave ? -es : es;
                const double vl = sqrt(A);
                const double vw = dw / vl, vs = ds / vl;
                const double ang = atan2(vw * nw + vs * ns, vw * tw + vs * ts) * (180.0 / M_PI);
                for (int k = 0; k < 3; ++k) cp3[k] = mp.c[k] + s0 * F.a[k] + (w1 > 0.0 ? w0 * q1[k] / w1 : 0.0);
                if (ang >= 0.0) theta = ang;
            }
        }
    }
    th[s] = theta;
    cpt[s][0] = cp3[0]; cpt[s][1] = cp3[1]; cpt[s][2] = cp3[2];
    __syncthreads();
    if (s == 0) {
        AngleRec* rec = last;
        rec->step = t;
        rec->n_sectors = mp.n_sectors;
        rec->pad_ = 0;
        double sum = 0.0;
        int nv = 0;
        for (int k = 0; k < 64; ++k) {
            const bool use = k < mp.n_sectors;
            rec->sector_deg[k] = use ? th[k] : NAN;
            rec->contact[k][0] = use ? cpt[k][0] : NAN;
            rec->contact[k][1] = use ? cpt[k][1] : NAN;
            rec->contact[k][2] = use ? cpt[k][2] : NAN;
            if (use && !isnan(th[k])) { sum += th[k]; ++nv; }
        }
        for (int k = 0; k < 3; ++k) rec->axis[k] = F.a[k];
        rec->n_valid = nv;
        rec->status = nv ? 0 : -6;
        rec->mean_deg = nv ? sum / nv : NAN;
        rec->adv_deg = rec->rec_deg = NAN;
        const double ga = mp.g[0] * F.a[0] + mp.g[1] * F.a[1] + mp.g[2] * F.a[2];
        const double gt[3] = {mp.g[0] - ga * F.a[0], mp.g[1] - ga * F.a[1], mp.g[2] - ga * F.a[2]};
        if (nv && gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2] > 0.0) {
            const int sa = sector_of(gt, F, mp.dim, mp.n_sectors);
            const int sr = mp.dim == 2 ? 1 - sa : (sa + mp.n_sectors / 2) % mp.n_sectors;
            rec->adv_deg = th[sa];
            rec->rec_deg = th[sr];
        }
        if (rec2) *rec2 = *rec;
    }
    __syncthreads();
    // clear the reduction slots for the next measurement
    ms->keys[s][0] = ~0ull;
    ms->keys[s][1] = ~0ull;
    if (s == 0) ms->cnt = ms->sx = ms->sy = ms->sz = 0ull;
}

// ---------------------------------------------------------------------------
// footprint of the contact lines for the unbalanced Young force (Sec. IV E)
// ---------------------------------------------------------------------------
// Fluid nodes with a lattice neighbour inside the substrate primitive whose
// density lies in [lo, hi] (the diffuse interface where its isodensity lines
// end on the substrate), counted per (sector of the measurement frame,
// surface kind): kind 0 on the primitive's mu_w surface (uniform, or an even
// latitude stripe), kind 1 on mu_w2.  counts[s * 2 + kind], zeroed by the caller.
struct YoungParams {
    double c[3], R;          // substrate centre and radius
    int concave;             // 1: cavity (solid outside the sphere)
    double pole[3], width;   // stripe pole (unit) and arc width
    int wet_mode;            // 0 uniform, 1 stripes
    int n_sectors, dim;
    double lo, hi;           // density band
    double axis[3];          // drop axis of the measurement
};

// One record of the unbalanced Young force; the layout of lbm_young.
struct YoungRec {
    long long step;
    int status, n_sectors;
    int count[64][2];
    double phi_d[64], theta_eq_deg[64], force[64];
};

// The Young force taken at every in-step measurement (on = 0: not taken).
struct YoungStep {
    int on;
    double gamma, c1, c2, roughness;   // gamma, cos theta_1, cos theta_2, r of Eq. 18
    unsigned* counts;                  // [64][2] footprint counts, zero between measurements
    YoungRec* last;                    // the latest record
};

// one node's contribution to the footprint counts: a fluid node in the
// density band with a lattice neighbour inside the substrate, counted in its
// sector and on the kind of surface at its own polar angle
template <class L, typename R>
__device__ __forceinline__ void young_node(const R* __restrict__ rho, const uint8_t* __restrict__ cls, const Dims& d,
                                           const YoungParams& yp, const Frame& F, int x, int y, int z,
                                           unsigned* __restrict__ counts) {
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    if ((cls[idx] & CLS_MASK) != CLS_FLUID) return;
    const double r0 = (double)rho[idx];
    if (!(r0 >= yp.lo && r0 <= yp.hi)) return;
    bool touches = false;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const double X = wrapc(x + L::E[i][0], d.nx) - yp.c[0], Y = wrapc(y + L::E[i][1], d.ny) - yp.c[1];
        const double Z = L::D == 3 ? wrapc(z + L::E[i][2], d.nz) - yp.c[2] : 0.0;
        const double d2 = X * X + Y * Y + Z * Z;
        touches = touches || (yp.concave ? d2 >= yp.R * yp.R : d2 <= yp.R * yp.R);
    }
    if (!touches) return;
    const double r[3] = {x - yp.c[0], y - yp.c[1], L::D == 3 ? z - yp.c[2] : 0.0};
    int kind = 0;
    if (yp.wet_mode) {
        const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double cp = rn > 0.0 ? (r[0] * yp.pole[0] + r[1] * yp.pole[1] + r[2] * yp.pole[2]) / rn : 1.0;
        cp = cp > 1.0 ? 1.0 : (cp < -1.0 ? -1.0 : cp);
        kind = (int)((long long)floor(yp.R * acos(cp) / yp.width) % 2);
    }
    atomicAdd(&counts[sector_of(r, F, yp.dim, yp.n_sectors) * 2 + kind], 1u);
}

// the footprint counts of an in-step measurement (returns at once on the
// other steps), in the frame the measurement's crossing search uses
template <class L, typename R>
__global__ void __launch_bounds__(256) k_young_step(const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                                    Dims d, YoungParams yp, MeasureParams mp,
                                                    const DevCtl* __restrict__ ctl, unsigned* __restrict__ counts) {
    if (!measuring(ctl)) return;
    const Frame F = make_frame(&ctl->m, mp);
    if (!F.ok) return;
    const unsigned ntiles = (unsigned)d.tx * (unsigned)d.ty * (unsigned)d.nz;
    for (unsigned t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int x, y, z;
        tile_coords(d, t, x, y, z);
        young_node<L, R>(rho, cls, d, yp, F, x, y, z, counts);
    }
}

// Eq. 18 and Eq. 17 for the record a measurement just wrote, one thread per
// sector (64 threads); clears the counts for the next measurement
__device__ inline void young_finish(const YoungStep& ys, const AngleRec* a, YoungRec* copy) {
    const int s = threadIdx.x;
    const bool ok = a->status == 0 && s < a->n_sectors;
    const unsigned h0 = ok ? ys.counts[2 * s] : 0u, h1 = ok ? ys.counts[2 * s + 1] : 0u;
    double phi = NAN, te = NAN, fo = NAN;
    if (ok && h0 + h1 > 0u) {
        phi = (double)h0 / (double)(h0 + h1);
        double ce = ys.roughness * phi * ys.c1 + (1.0 - phi) * ys.c2;
        ce = ce > 1.0 ? 1.0 : (ce < -1.0 ? -1.0 : ce);
        te = acos(ce) * (180.0 / M_PI);
        if (!isnan(a->sector_deg[s])) fo = ys.gamma * (cos(a->sector_deg[s] * (M_PI / 180.0)) - ce);
    }
    YoungRec* recs[2] = {ys.last, copy};
    for (int k = 0; k < 2; ++k) {
        YoungRec* r = recs[k];
        if (!r) continue;
        if (s == 0) {
            r->step = a->step;
            r->status = a->status;
            r->n_sectors = a->n_sectors;
        }
        r->count[s][0] = (int)h0;
        r->count[s][1] = (int)h1;
        r->phi_d[s] = phi;
        r->theta_eq_deg[s] = te;
        r->force[s] = fo;
    }
    ys.counts[2 * s] = 0u;
    ys.counts[2 * s + 1] = 0u;
}

template <class L, typename R>
__global__ void __launch_bounds__(256) k_young_count(const R* __restrict__ rho, const uint8_t* __restrict__ cls,
                                                     Dims d, YoungParams yp, unsigned* __restrict__ counts) {
    const Frame F = frame_from_axis(yp.axis, yp.dim);
    const unsigned ntiles = (unsigned)d.tx * (unsigned)d.ty * (unsigned)d.nz;
    for (unsigned t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int x, y, z;
        tile_coords(d, t, x, y, z);
        young_node<L, R>(rho, cls, d, yp, F, x, y, z, counts);
    }
}

template <class L, typename R>
__global__ void __launch_bounds__(64) k_finalize(const R* __restrict__ rho, DevCtl* __restrict__ ctl, Dims d,
                                                 MeasureParams mp, AngleRec* __restrict__ series,
                                                 AngleRec* __restrict__ last, int tick, YoungStep ys = YoungStep{},
                                                 YoungRec* __restrict__ yseries = nullptr) {
    if (measuring(ctl)) {
        const bool keep = series && ctl->series_count < ctl->series_cap;
        finalize_slots<L, R>(rho, d, mp, &ctl->m, ctl->t, last, keep ? series + ctl->series_count : nullptr);
        __syncthreads();
        if (ys.on) {
            young_finish(ys, last, keep && yseries ? yseries + ctl->series_count : nullptr);
            __syncthreads();
        }
        if (threadIdx.x == 0 && keep) ctl->series_count += 1;
    }
    if (threadIdx.x == 0 && tick) ctl->t += 1;
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_fill_value(R* __restrict__ p, size_t n, R v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

static __global__ void k_ctl_reset(DevCtl* ctl, int every, int force, int series_cap) {
    const int s = threadIdx.x;
    ctl->m.keys[s][0] = ~0ull;
    ctl->m.keys[s][1] = ~0ull;
    if (s == 0) {
        ctl->m.cnt = ctl->m.sx = ctl->m.sy = ctl->m.sz = 0ull;
        ctl->every = every;
        ctl->force_measure = force;
        ctl->series_count = 0;
        ctl->series_cap = series_cap;
    }
}

static __global__ void k_ctl_set(DevCtl* ctl, long long t, int every, int force, int series_cap, int clear_status) {
    if (threadIdx.x == 0) {
        ctl->t = t;
        ctl->every = every;
        ctl->force_measure = force;
        ctl->series_count = 0;
        ctl->series_cap = series_cap;
        if (clear_status) ctl->status = 0;
    }
}

// state = f_eq(rho, 0) on fluid nodes of [beg, end), zero on its other nodes
template <class L, typename R>
__global__ void k_init_feq(const R* __restrict__ rho, R* __restrict__ f, const uint8_t* __restrict__ cls, long long N,
                           long long beg, long long end) {
    for (long long n = beg + (long long)blockIdx.x * blockDim.x + threadIdx.x; n < end;
         n += (long long)gridDim.x * blockDim.x) {
        const bool fl = (cls[n] & CLS_MASK) == CLS_FLUID;
        const R r = fl ? rho[n] : R(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) f[(size_t)i * N + n] = r * R(L::w(i));
    }
}

// v = u + F / (2 rho) (Sec. II B), with F of Eq. 7 from the current rho and mu;
// fin holds S_t
template <class L, typename R, typename C = R, bool SC = false>
__global__ void __launch_bounds__(256) k_velocity(const R* __restrict__ fin, const R* __restrict__ rho,
                                                  const R* __restrict__ mu, const uint8_t* __restrict__ cls, Dims d,
                                                  Collision<C> cp, long long t, R* __restrict__ vel) {
    int x, y, z;
    tile_node(d, x, y, z);
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    if ((cls[idx] & CLS_MASK) != CLS_FLUID) {
        vel[idx] = vel[d.N + idx] = vel[2 * d.N + idx] = R(0);
        return;
    }
    typedef double D;
    const D r0 = (D)rho[idx];
    D Fa[3] = {D(0), D(0), D(0)};
    if constexpr (SC) {
        const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
        const Nbr oz = L::D == 3 ? nbr_offsets(z, d.nz, d.px * d.ny) : Nbr{0, 0, 0, 0};
        sc_force<L, R>(mu, idx, ox, oy, oz, cp.sc_G, Fa[0], Fa[1], Fa[2]);
        if (t >= cp.g_start)
            for (int a = 0; a < 3; ++a) Fa[a] += r0 * (D)cp.g[a];
    }
    for (int a = 0; a < L::D && !SC; ++a) {
        int o[3] = {0, 0, 0};
        long long id[5];
        for (int k = -2; k <= 2; ++k) {
            o[a] = k;
            const int X = wrapc(x + o[0], d.nx), Y = wrapc(y + o[1], d.ny), Z = L::D == 3 ? wrapc(z + o[2], d.nz) : 0;
            id[k + 2] = nid(d, X, Y, Z);
        }
        const D gm = d1c<D>(mu[id[0]], mu[id[1]], mu[id[3]], mu[id[4]]);
        const D gr = d1c<D>(rho[id[0]], rho[id[1]], rho[id[3]], rho[id[4]]);
        Fa[a] = -r0 * gm + gr * D(1.0 / 3.0);
        if (t >= cp.g_start) Fa[a] += r0 * (D)cp.g[a];
    }
    D rs = D(0), j[3] = {D(0), D(0), D(0)};
    for (int i = 0; i < L::Q; ++i) {
        const D fi = (D)fin[(size_t)i * d.N + idx];
        rs += fi;
        j[0] += D(L::E[i][0]) * fi;
        j[1] += D(L::E[i][1]) * fi;
        j[2] += D(L::E[i][2]) * fi;
    }
    for (int a = 0; a < 3; ++a) vel[(size_t)a * d.N + idx] = (R)(j[a] / rs + Fa[a] / (D(2) * rs));
}

// deterministic mass: per-block FP64 partial sums in a fixed order
template <class L, typename R>
__global__ void __launch_bounds__(256) k_mass_partial(const R* __restrict__ f, const uint8_t* __restrict__ cls,
                                                      long long N, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    const long long per = (N + gridDim.x - 1) / gridDim.x;
    const long long beg = (long long)blockIdx.x * per, end = beg + per < N ? beg + per : N;
    for (long long n = beg + threadIdx.x; n < end; n += 256) {
        if ((cls[n] & CLS_MASK) != CLS_FLUID) continue;
        for (int i = 0; i < L::Q; ++i) s += (double)f[(size_t)i * N + n];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

static __global__ void k_mass_final(const double* __restrict__ part, int n, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

}  // namespace lbm

namespace lbm {
template <typename R>
__global__ void k_add_value(R* __restrict__ p, size_t n, R v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] += v;
}
}  // namespace lbm
