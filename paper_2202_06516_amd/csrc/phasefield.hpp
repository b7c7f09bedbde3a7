// phasefield.hpp -- the phase-field model on the split step (a single lattice,
// and every case of the batched solver through the same per-node bodies).
//
// Sec. V names phase-field models among the multiphase models whose diffuse
// interface the measurement reads; the paper fixes none.  The model here is
// the free-energy one with an order parameter phi (liquid +1, gas -1):
//   free energy     A/4 (phi^2 - 1)^2 + kappa/2 |grad phi|^2
//   mu              A (phi^3 - phi) - kappa lap4(phi) on fluid nodes
//   force           F = mu grad4(phi) (+ rho g from step g_start)
//   fluid f         the collision of the other models (MRT or BGK with
//                   exact-difference forcing, halfway or interpolated walls)
//   order g         BGK with 1/tau_g toward
//                     g_i^eq = w_i (3 gamma mu + 3 phi e_i.v
//                                   + phi (4.5 (e_i.v)^2 - 1.5 v.v)),  i > 0
//                     g_0^eq = phi - sum_{i>0} g_i^eq
//                   with v = (sum_i f_i e_i + F / 2) / rho: the Cahn-Hilliard
//                   equation with mobility gamma (tau_g - 1/2); g streams with
//                   halfway bounce-back at every wall (no flux through a solid)
//   wetting         both solid layers hold the wall order parameter phi_w of
//                   their primitive, stripe, map entry or outer wall (written
//                   once, when the solids are set), which the Laplacian and the
//                   gradient reach
// The measurement reads phi at the isolevel 0, the mean of the two bulk values.
// A step: k_pf_density (phi of S_t, the liquid centroid sums of phi on measure
// steps; rho = sum f only where the fields are read, since the collision forms
// the density of its own gather), k_pf_mu, the crossing search on phi,
// k_pf_collide (f and g), the finalize.  mu and F are formed in double in
// every precision: mu is the difference of two terms that cancel inside an
// interface at rest.
#pragma once

#include "kernels.hpp"

namespace lbm {

struct PhaseField {
    double A, kappa;  // free-energy coefficients
    double gamma;     // mobility coefficient: M = gamma (tau_g - 1/2)
    double omega;     // 1 / tau_g
    double rho0;      // fluid density of the initial state (both phases)
};

// phi = sum g of the gathered populations of a fluid node, and with RHO also
// rho = sum f (the step itself needs no rho field); true if liquid.  Every
// per-node body below serves a single lattice tiled by workgroups and the
// packed lattices of the batched solver alike.
template <class L, typename R, typename C, bool PULL, bool RHO>
__device__ __forceinline__ bool pf_density_node(const R* __restrict__ f, const R* __restrict__ g,
                                                R* __restrict__ rho, R* __restrict__ phi,
                                                const uint8_t* __restrict__ cls, const Dims& d, const WallBC& bc,
                                                int* status, double phi_m, int x, int y, int z) {
    bool liquid = false;
    if (x < d.nx && y < d.ny) {
        const long long idx = nid(d, x, y, z);
        const uint32_t ix = (uint32_t)idx;
        const uint8_t c = at(cls, ix);
        if ((c & CLS_MASK) == CLS_FLUID) {
            R S[L::Q];
            if constexpr (RHO) {
                gather<L, R, C, PULL>(f, d, idx, x, y, z, c, bc, S);
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < L::Q; ++i) s += (double)S[i];
                at(rho, ix) = (R)s;
                if (!(s > 0.0 && s < 1e300)) atomicOr(status, 1);  // also catches NaN
            }
            WallBC hw = bc;
            hw.bouzidi = 0;
            gather<L, R, C, PULL>(g, d, idx, x, y, z, c, hw, S);
            double p = 0.0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) p += (double)S[i];
            const R ps = (R)p;
            at(phi, ix) = ps;
            if (!(fabs(p) < 1e300)) atomicOr(status, 1);
            liquid = (double)ps >= phi_m;
        }
    }
    return liquid;
}

template <class L, typename R, typename C, bool PULL, bool RHO>
__global__ void __launch_bounds__(256) k_pf_density(const R* __restrict__ f, const R* __restrict__ g,
                                                    R* __restrict__ rho, R* __restrict__ phi,
                                                    const uint8_t* __restrict__ cls, Dims d, WallBC bc,
                                                    DevCtl* __restrict__ ctl, double phi_m) {
    int x, y, z;
    tile_node(d, x, y, z);
    const bool liquid = pf_density_node<L, R, C, PULL, RHO>(f, g, rho, phi, cls, d, bc, &ctl->status, phi_m, x, y, z);
    if (measuring(ctl)) centroid_reduce(liquid, x, y, z, &ctl->m);
}

// mu = A (phi^3 - phi) - kappa lap4(phi) on fluid nodes, in double
template <class L, typename R>
__device__ __forceinline__ void pf_mu_node(const R* __restrict__ phi, R* __restrict__ mu,
                                           const uint8_t* __restrict__ cls, const Dims& d, const PhaseField& pf,
                                           int x, int y, int z) {
    const uint32_t ix = nid32(d, x, y, z);
    const uint8_t c = at(cls, ix);
    const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
    auto p = [&](int o) { return (double)at(phi, ix + (uint32_t)o); };
    const double c0 = p(0);
    double lap = d2c<double>(p(ox.m2), p(ox.m1), c0, p(ox.p1), p(ox.p2));
    lap += d2c<double>(p(oy.m2), p(oy.m1), c0, p(oy.p1), p(oy.p2));
    if (L::D == 3) {
        const Nbr oz = nbr_offsets(z, d.nz, d.px * d.ny);
        lap += d2c<double>(p(oz.m2), p(oz.m1), c0, p(oz.p1), p(oz.p2));
    }
    const double m = pf.A * (c0 * c0 * c0 - c0) - pf.kappa * lap;
    asm volatile("" : : "v"(m));  // keeps the stencil loads above the class test
    if ((c & CLS_MASK) != CLS_FLUID) return;
    at(mu, ix) = (R)m;
}

template <class L, typename R, bool ZCH>
__global__ void __launch_bounds__(256) k_pf_mu(const R* __restrict__ phi, R* __restrict__ mu,
                                               const uint8_t* __restrict__ cls, Dims d, PhaseField pf) {
    int x, y, z;
    if constexpr (ZCH) {
        tile_node_zc(d, x, y, z);
        if (x >= d.nx || y >= d.ny) return;
        const int z1 = z + d.zc < d.nz ? z + d.zc : d.nz;
        for (; z < z1; ++z) pf_mu_node<L, R>(phi, mu, cls, d, pf, x, y, z);
    } else {
        tile_node(d, x, y, z);
        if (x >= d.nx || y >= d.ny) return;
        pf_mu_node<L, R>(phi, mu, cls, d, pf, x, y, z);
    }
}

// F = mu grad4(phi), plus r0 g from step g_start (r0: the node's density), in double
template <class L, typename R, typename C>
__device__ __forceinline__ void pf_force(double r0, const R* __restrict__ phi, const R* __restrict__ mu,
                                         const Dims& d, uint32_t ix, int x, int y, int z, const Collision<C>& cp,
                                         long long t, double F[3]) {
    const Nbr ox = nbr_offsets(x, d.nx, 1), oy = nbr_offsets(y, d.ny, d.px);
    auto p = [&](int o) { return (double)at(phi, ix + (uint32_t)o); };
    const double m0 = (double)at(mu, ix);
    F[0] = m0 * d1c<double>(p(ox.m2), p(ox.m1), p(ox.p1), p(ox.p2));
    F[1] = m0 * d1c<double>(p(oy.m2), p(oy.m1), p(oy.p1), p(oy.p2));
    F[2] = 0.0;
    if (L::D == 3) {
        const Nbr oz = nbr_offsets(z, d.nz, d.px * d.ny);
        F[2] = m0 * d1c<double>(p(oz.m2), p(oz.m1), p(oz.p1), p(oz.p2));
    }
    if (t >= cp.g_start) {
#pragma unroll
        for (int a = 0; a < 3; ++a) F[a] += r0 * cp.g[a];
    }
}

// The fluid velocity v = (sum_i S_i e_i + F / 2) / rho of gathered populations
// S: in double with FP64 arithmetic; with FP32 arithmetic the momentum from
// the differences of opposite populations and 1 / rho from the hardware
// reciprocal, as the fluid collision forms them (the density sum in double).
template <class L, typename R, typename C>
__device__ __forceinline__ void pf_velocity(const R S[L::Q], const double F[3], C v[3]) {
    double rd = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) rd += (double)S[i];
    if constexpr (sizeof(C) == 8) {
        double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (L::E[i][a]) j[a] += (double)L::E[i][a] * (double)S[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = (j[a] + 0.5 * F[a]) / rd;
    } else {
        C j[3] = {C(0), C(0), C(0)};
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            if (L::OPP[i] < i) continue;
            const C df = (C)S[i] - (C)S[L::OPP[i]];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (L::E[i][a]) j[a] += C(L::E[i][a]) * df;
        }
        const C ir = __builtin_amdgcn_rcpf((C)rd);
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = (j[a] + C(0.5) * (C)F[a]) * ir;
    }
}

// BGK relaxation of the order-parameter populations G toward the equilibrium
// above.  With FP32 arithmetic the rest population takes the remainder
// phi - sum_{i>0} g*_i of the stored values, in double, so that the rounded
// lattice weights do not create or destroy order parameter (as the fluid
// collision does for the mass).
template <class L, typename R, typename C>
__device__ __forceinline__ void pf_collide_g(const R G[L::Q], const C v[3], C mu, const PhaseField& pf,
                                             R go[L::Q]) {
    double pd = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) pd += (double)G[i];
    const C ph = (C)pd, om = (C)pf.omega;
    const C vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const C gm3 = C(3) * (C)pf.gamma * mu;
    constexpr bool kRestRemainder = sizeof(C) == 4;
    C rest = ph;
    double srest = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::OPP[i] < i) continue;
        const int j = L::OPP[i];
        const C ev = C(L::E[i][0]) * v[0] + C(L::E[i][1]) * v[1] + C(L::E[i][2]) * v[2];
        const C wi = C(L::w(i));
        const C sym = wi * (gm3 + ph * (C(4.5) * ev * ev - C(1.5) * vv));
        const C anti = wi * C(3) * ph * ev;
        const C ei = sym + anti, ej = sym - anti;
        rest -= ei;
        rest -= ej;
        const R oi = (R)((C)G[i] - ((C)G[i] - ei) * om);
        const R oj = (R)((C)G[j] - ((C)G[j] - ej) * om);
        go[i] = oi;
        go[j] = oj;
        if (kRestRemainder) srest += (double)oi + (double)oj;
    }
    if (kRestRemainder) go[0] = (R)(pd - srest);
    else go[0] = (R)((C)G[0] - ((C)G[0] - rest) * om);
}

// Collision of both population sets of one fluid node; post-collision values
// stored at the node (streaming is the next step's pull).  The fluid density
// of the node is the sum of its gathered populations, checked here.
template <class L, typename R, typename C, bool PULL, bool MRT>
__device__ __forceinline__ void pf_collide_node(const R* __restrict__ fin, R* __restrict__ fout,
                                                const R* __restrict__ gin, R* __restrict__ gout,
                                                const R* __restrict__ phi, const R* __restrict__ mu,
                                                const uint8_t* __restrict__ cls, const Dims& d, const WallBC& bc,
                                                const Collision<C>& cp, const PhaseField& pf, int* status,
                                                long long t, int x, int y, int z) {
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    const uint32_t ix = (uint32_t)idx;
    const uint8_t c = at(cls, ix);
    if ((c & CLS_MASK) != CLS_FLUID) return;
    R S[L::Q];
    gather<L, R, C, PULL>(fin, d, idx, x, y, z, c, bc, S);
    double r0 = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) r0 += (double)S[i];
    if (!(r0 > 0.0 && r0 < 1e300)) atomicOr(status, 1);  // also catches NaN
    double F[3];
    pf_force<L, R, C>(r0, phi, mu, d, ix, x, y, z, cp, t, F);
    collide_apply<L, R, C, MRT, true>(S, (C)F[0], (C)F[1], (C)F[2], cp, fout, idx, d.N);
    C v[3];
    pf_velocity<L, R, C>(S, F, v);
    WallBC hw = bc;
    hw.bouzidi = 0;
    gather<L, R, C, PULL>(gin, d, idx, x, y, z, c, hw, S);
    R go[L::Q];
    pf_collide_g<L, R, C>(S, v, (C)at(mu, ix), pf, go);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) put<true>(&at(gout + (size_t)i * d.N, ix), go[i]);
}

template <class L, typename R, typename C, bool PULL, bool MRT>
__global__ void __launch_bounds__(256) k_pf_collide(const R* __restrict__ fin, R* __restrict__ fout,
                                                    const R* __restrict__ gin, R* __restrict__ gout,
                                                    const R* __restrict__ phi, const R* __restrict__ mu,
                                                    const uint8_t* __restrict__ cls, Dims d, WallBC bc,
                                                    Collision<C> cp, PhaseField pf, DevCtl* __restrict__ ctl) {
    int x, y, z;
    tile_node(d, x, y, z);
    pf_collide_node<L, R, C, PULL, MRT>(fin, fout, gin, gout, phi, mu, cls, d, bc, cp, pf, &ctl->status, ctl->t, x,
                                        y, z);
}

// The state of an order-parameter field src on nodes [beg, end) of arrays of
// stride N: on fluid nodes phi = src, rho = rho0, f = f^eq(rho0, 0), g at
// rest (g_0 = phi); populations zero elsewhere.  phi of the solid layers (the
// wall values) is left as it is.
template <class L, typename R>
__global__ void k_pf_init(const R* __restrict__ src, R* __restrict__ phi, R* __restrict__ rho, R* __restrict__ f,
                          R* __restrict__ g, const uint8_t* __restrict__ cls, long long N, double rho0, long long beg,
                          long long end) {
    for (long long n = beg + (long long)blockIdx.x * blockDim.x + threadIdx.x; n < end;
         n += (long long)gridDim.x * blockDim.x) {
        const bool fl = (cls[n] & CLS_MASK) == CLS_FLUID;
        const R p = fl ? src[n] : R(0);
        if (fl) phi[n] = p;
        rho[n] = fl ? (R)rho0 : R(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            f[(size_t)i * N + n] = fl ? (R)(L::w(i) * rho0) : R(0);
            g[(size_t)i * N + n] = (fl && i == 0) ? p : R(0);
        }
    }
}

// v = u + F / (2 rho) of S_t (fin) with the phase-field force
template <class L, typename R, typename C>
__global__ void __launch_bounds__(256) k_pf_velocity(const R* __restrict__ fin, const R* __restrict__ phi,
                                                     const R* __restrict__ mu,
                                                     const uint8_t* __restrict__ cls, Dims d, Collision<C> cp,
                                                     long long t, R* __restrict__ vel) {
    int x, y, z;
    tile_node(d, x, y, z);
    if (x >= d.nx || y >= d.ny) return;
    const long long idx = nid(d, x, y, z);
    if ((cls[idx] & CLS_MASK) != CLS_FLUID) {
        vel[idx] = vel[d.N + idx] = vel[2 * d.N + idx] = R(0);
        return;
    }
    double rs = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L::Q; ++i) {
        const double fi = (double)fin[(size_t)i * d.N + idx];
        rs += fi;
        j[0] += L::E[i][0] * fi;
        j[1] += L::E[i][1] * fi;
        j[2] += L::E[i][2] * fi;
    }
    double F[3];
    pf_force<L, R, C>(rs, phi, mu, d, (uint32_t)idx, x, y, z, cp, t, F);
    for (int a = 0; a < 3; ++a) vel[(size_t)a * d.N + idx] = (R)(j[a] / rs + F[a] / (2.0 * rs));
}

}  // namespace lbm
