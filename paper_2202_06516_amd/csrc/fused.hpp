// fused.hpp -- one time step of a D3Q19 lattice as a single pass over the
// populations.
//
// The split step reads every population twice: once to sum the density of
// S_t, once more to collide.  k_step reads them once.  For step t it does what
// k_collide does -- gathers S_t (pull streaming, Eq. 4, with the wall
// condition), takes the force of Eq. 7 from rho_t and mu_t, collides (Eq. 1-3,
// 13) and stores f*_t -- and in the same pass sums the density of step t+1
// (under the pseudopotential model the force comes from k_force, which formed
// it after the previous step):
//
//     rho_{t+1}(x) = sum over i of f*_i(x - e_i) where x - e_i is fluid,
//                  + f*_j(x) for every link j from x to a solid node,
//
// the second term being the populations the wall returns to x.  With the
// exact mass correction of the interpolated wall (Sec. III A) the density is
// the same as with halfway bounce-back, so the sum holds for both wall modes.
// Its summation order is not that of the split path's density pass, so the two
// paths agree to rounding, not bit for bit.
//
// Work decomposition.  A workgroup owns whole rows: thread = x (nx threads, nx
// a multiple of 64), TY consecutive rows in y, and it walks zc consecutive
// planes in z.  A node's moving populations go to the nine rows (y + e_y,
// z + e_z); within a row the x shift is a one-lane move across the wave (DPP),
// and between the waves of a row it goes through LDS once per plane.  Each
// thread keeps the partial densities of its column for the rows y0-1..y0+TY
// and the planes z-1, z, z+1 (in LDS); a target plane is complete, and
// stored, once the walk has passed the source plane above it.  Partial sums
// for rows and planes owned by other workgroups go to three ghost arrays, each
// entry with exactly one writer (the y neighbour, the z neighbour, the
// diagonal one; TY >= 2 and zc >= 2 guarantee it), and k_ghost adds them to
// the edge rows and planes after the launch.
#pragma once

#include "kernels.hpp"

namespace lbm {

// index of the D3Q19 direction (ex, ey, ez)
__host__ __device__ constexpr int d3q19_dir(int ex, int ey, int ez) {
    int k = -1;
    for (int i = 0; i < D3Q19::Q; ++i)
        if (D3Q19::E[i][0] == ex && D3Q19::E[i][1] == ey && D3Q19::E[i][2] == ez) k = i;
    return k;
}

// lane l receives the value of lane l - 1 of its wave (lane 0 receives 0)
template <typename T>
__device__ __forceinline__ T lane_from_below(T v) {
    return __builtin_amdgcn_update_dpp(T(0), v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
// lane l receives the value of lane l + 1 of its wave (lane 63 receives 0)
template <typename T>
__device__ __forceinline__ T lane_from_above(T v) {
    return __builtin_amdgcn_update_dpp(T(0), v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}

// workgroup id -> tile, with contiguous tile ranges per XCD (as tile_node)
__device__ __forceinline__ unsigned xcd_tile(unsigned t, unsigned n, int remap) {
    if (!remap) return t;
    const unsigned q = n >> 3, r = n & 7u, xcd = t & 7u, loc = t >> 3;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + loc;
}

// Directions by target row.  The rows (e_y, e_z) = (0,0), (+1,0), (-1,0),
// (0,+1), (0,-1) each receive three directions, with e_x = 0, +1, -1
// (GRP[g][0..2]); the four diagonal rows (+1,+1), (-1,-1), (+1,-1), (-1,+1)
// one each, with e_x = 0.
struct RowGroups {
    static constexpr int GRP[5][3] = {
        {d3q19_dir(0, 0, 0), d3q19_dir(1, 0, 0), d3q19_dir(-1, 0, 0)},
        {d3q19_dir(0, 1, 0), d3q19_dir(1, 1, 0), d3q19_dir(-1, 1, 0)},
        {d3q19_dir(0, -1, 0), d3q19_dir(1, -1, 0), d3q19_dir(-1, -1, 0)},
        {d3q19_dir(0, 0, 1), d3q19_dir(1, 0, 1), d3q19_dir(-1, 0, 1)},
        {d3q19_dir(0, 0, -1), d3q19_dir(1, 0, -1), d3q19_dir(-1, 0, -1)}};
    static constexpr int PP = d3q19_dir(0, 1, 1), MM = d3q19_dir(0, -1, -1);
    static constexpr int PM = d3q19_dir(0, 1, -1), MP = d3q19_dir(0, -1, 1);
};
static_assert(RowGroups::GRP[0][0] == 0 && RowGroups::PP > 0 && RowGroups::MM > 0 && RowGroups::PM > 0 &&
                  RowGroups::MP > 0, "D3Q19 direction table");

// Barrier for the LDS exchange between the waves of a workgroup: waits for
// this wave's LDS operations only.  (__syncthreads also waits for every
// outstanding global load and store, which would drain the walk's pipeline.)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// A streaming load: the populations are read once per step, and marked so
// that they leave the caches first, before the density and chemical-potential
// planes that the force stencils of the next nodes read again.
template <typename R>
__device__ __forceinline__ R ldnt(const R* p) { return __builtin_nontemporal_load(p); }

// Populations S_t of node idx for the walk's pipeline: every load is issued,
// unconditionally and without waiting for an earlier one.  A link whose
// source x - e_i is solid (bit opp(i) of the node's wall mask m) reads the
// population that left x toward the wall (halfway bounce-back).  Opposite
// directions are stored next to each other (i and opp(i) differ by one), so
// both candidates are addressed from the array of the lower of the two with
// one select of a 32-bit offset.  A lane on a solid node (mask 0) pulls from
// its periodic neighbours like a fluid one: every offset is in bounds and
// its values are never used.
template <class L, typename R, bool PULL>
__device__ __forceinline__ void gather_issue(const R* __restrict__ f, const Dims& d, uint32_t ix, int x, int y,
                                             int z, uint32_t m, R S[L::Q]) {
    const uint32_t N = (uint32_t)d.N;
    if (!PULL) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) S[i] = ldnt(&at(f + (size_t)i * d.N, ix));
        return;
    }
    const int ox[3] = {x >= 1 ? -1 : d.nx - 1, 0, x + 1 < d.nx ? 1 : 1 - d.nx};
    const int oy[3] = {(y >= 1 ? -1 : d.ny - 1) * d.px, 0, (y + 1 < d.ny ? 1 : 1 - d.ny) * d.px};
    const int sz = d.px * d.ny;
    const int oz[3] = {(z >= 1 ? -1 : d.nz - 1) * sz, 0, (z + 1 < d.nz ? 1 : 1 - d.nz) * sz};
    S[0] = ldnt(&at(f, ix));
    auto pull = [&](int i) {
        return ix + (uint32_t)(ox[1 - L::E[i][0]] + oy[1 - L::E[i][1]] + oz[1 - L::E[i][2]]);
    };
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::OPP[i], lo = i < j ? i : j;
        static_assert(L::OPP[1] == 2 && L::OPP[18] == 17, "opposite directions are adjacent");
        const bool back = (m >> j) & 1u;
        const uint32_t a = (i > lo ? N : 0u) + pull(i), b = (j > lo ? N : 0u) + ix;
        S[i] = ldnt(&at(f + (size_t)lo * d.N, back ? b : a));
    }
}

// The interpolated wall (Sec. III A) of one boundary fluid node from the
// halfway values: for every cut link (bit j of bm: x + e_j is solid) S_i,
// i = opp(j), holds f*_j(x); it becomes the linear interpolation in the link's
// wall fraction q -- with the node behind x when q < 1/2, only if that
// partner's population lies within a factor of two of x's own (the same
// phase), else from f*_i(x) -- and the difference goes to S_0, as the split
// path's gather forms them.  The mass correction leaves the node's density
// that of halfway bounce-back.
template <class L, typename R, typename C>
__device__ __forceinline__ void interp_wall(const R* __restrict__ f, const Dims& d, uint32_t ix, int x, int y, int z,
                                            uint32_t bm, const WallBC& bc, R S[L::Q]) {
    const int ox[3] = {x >= 1 ? -1 : d.nx - 1, 0, x + 1 < d.nx ? 1 : 1 - d.nx};
    const int oy[3] = {(y >= 1 ? -1 : d.ny - 1) * d.px, 0, (y + 1 < d.ny ? 1 : 1 - d.ny) * d.px};
    const int sz = d.px * d.ny;
    const int oz[3] = {(z >= 1 ? -1 : d.nz - 1) * sz, 0, (z + 1 < d.nz ? 1 : 1 - d.nz) * sz};
    const int k = bc.bidx[ix];
    const R* q_of = (const R*)bc.q + (size_t)k * L::Q;
    C dm = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::OPP[i];
        if (!(bm & (1u << j))) continue;
        const R outj = S[i];
        const C q = (C)q_of[j];
        C v = (C)outj;
        if (q < C(0.5)) {
            if (!(bm & (1u << i))) {  // x + e_i is the fluid node behind x
                const uint32_t b = ix + (uint32_t)(ox[1 + L::E[i][0]] + oy[1 + L::E[i][1]] + oz[1 + L::E[i][2]]);
                const R fb = at(f + (size_t)j * d.N, b);
                if (fb <= R(2) * outj && outj <= R(2) * fb) v = C(2) * q * (C)outj + (C(1) - C(2) * q) * (C)fb;
            }
        } else {
            v = (C)outj / (C(2) * q) + (C(2) * q - C(1)) / (C(2) * q) * (C)at(f + (size_t)i * d.N, ix);
        }
        S[i] = (R)v;
        dm += (C)outj - v;
    }
    S[0] = (R)((C)S[0] + dm);
}

// The one-pass step with the interpolated wall: after k_step has stored f*_t,
// each node whose cut links include one of wall fraction other than 1/2 (the
// box walls' links are halfway exactly) takes the values its next pull will
// read through those links from interp_wall, written into the slots that pull
// reads: f*_j(x) for a cut link j (which only x reads: x + e_j is solid) and
// f*_0(x).  Every value a node reads here is its own or that of the fluid node
// behind it along a cut link, whose slots in that direction are not cut links
// (its neighbour there is x), so no node reads a slot another one writes.
// The density of step t + 1 that k_step summed is unchanged by it (the mass
// correction).  Every later gather of this state takes halfway bounce-back.
template <class L, typename R, typename C>
__global__ void __launch_bounds__(256) k_interp_wall(const int* __restrict__ list, int n,
                                                     const long long* __restrict__ b_node,
                                                     const uint32_t* __restrict__ b_mask, R* __restrict__ f, Dims d,
                                                     WallBC bc) {
    const int t = (int)(blockIdx.x * 256 + threadIdx.x);
    if (t >= n) return;
    const int k = list[t];
    const long long node = b_node[k];
    const uint32_t ix = (uint32_t)node, bm = b_mask[k];
    const uint32_t row = ix / (uint32_t)d.px;
    const int x = (int)(ix - row * (uint32_t)d.px), y = (int)(row % (uint32_t)d.ny), z = (int)(row / (uint32_t)d.ny);
    R S[L::Q];
    S[0] = at(f, ix);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::OPP[i];
        S[i] = (bm & (1u << j)) ? at(f + (size_t)j * d.N, ix) : R(0);
    }
    interp_wall<L, R, C>(f, d, ix, x, y, z, bm, bc, S);
    at(f, ix) = S[0];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::OPP[i];
        if (bm & (1u << j)) at(f + (size_t)j * d.N, ix) = S[i];
    }
}

template <typename R, typename C, bool PULL, bool MRT, bool SC, int TY, int NX>
__global__ void __launch_bounds__(NX) k_step(const R* __restrict__ fin, R* __restrict__ fout,
                                             const R* __restrict__ rho, const R* __restrict__ mu,
                                             const R* __restrict__ force, R* __restrict__ rho_next,
                                             R* __restrict__ gy, R* __restrict__ gz, R* __restrict__ gyz,
                                             const uint8_t* __restrict__ cls, Dims d, WallBC bc, Collision<C> cp,
                                             const DevCtl* __restrict__ ctl, int zc, R* __restrict__ sink) {
    typedef D3Q19 L;
    static_assert(TY >= 2, "one writer per ghost entry needs two rows or more");
    const unsigned t = xcd_tile(blockIdx.x, gridDim.x, d.xcd_remap);
    const Dims d0 = d;
    const int x0 = threadIdx.x;
    const int nty = d.ny / TY;
    const int y0 = (int)(t % (unsigned)nty) * TY, z0 = (int)(t / (unsigned)nty) * zc;
    const int x = threadIdx.x, lane = x & 63, wave = x >> 6, nw = d.nx >> 6;
    const int ylo = y0 >= 1 ? y0 - 1 : d.ny - 1, yhi = y0 + TY < d.ny ? y0 + TY : 0;
    const int nn = TY * zc;  // nodes of this thread's column in the tile; node n is row n % TY of plane z0 + n / TY
    const long long tstep = ctl->t;

    // Partial densities of the tile's rows y0-1..y0+TY (index row - y0 + 1)
    // for three target planes, slot z mod 3; thread x owns column x, so its
    // additions need no synchronisation.  They live in LDS rather than in
    // registers, which keeps the walk at the register count of one node.
    __shared__ C acc[TY + 2][3][NX];
    // [plane parity][0: e_x = +1 values of lane 63, 1: e_x = -1 values of lane 0][wave][row][row group]
    __shared__ C edge[2][2][NX / 64][TY][5];
    // The rho and mu values of the planes z - 2 .. z + 1 of each column, one
    // slot per plane modulo 4 and per row of the tile: the force stencil
    // takes its centre and z neighbours from the thread's own column and its
    // x neighbours from the neighbouring columns' slots of plane z, and loads
    // only plane z + 2 and the y neighbours; the node then stores plane z + 2
    // into the slot of plane z - 2 (no longer needed by its row).  A slot is
    // written two planes before another thread reads it and overwritten two
    // planes after, with a barrier at the end of every plane in between.
    // FP32 storage and rows of up to 256 nodes (32 KB).  (Rows of 512 in a
    // 512-thread variant with the ring ran no faster at 512^3.)
    constexpr bool RING = !SC && sizeof(R) == 4 && NX <= 256;
    __shared__ R ring[RING ? 4 : 1][TY][2][RING ? NX : 1];
#pragma unroll
    for (int k = 0; k < TY + 2; ++k) acc[k][0][x] = acc[k][1][x] = acc[k][2][x] = C(0);

    // The walk is a software pipeline over the column's nodes: while node n is
    // collided, the populations and force of node n+1, the wall mask of node
    // n+2 and the class of node n+3 are in flight.  A wave's loads and stores
    // share one in-order counter, so loads issued after node n's stores would
    // also wait for them; issued before, they do not.  For the compiler to
    // count them, every load and store of the walk is unconditional: a lane
    // on a solid node reads and writes that node's own population slots,
    // which nothing else reads (the wall condition takes the populations of
    // the fluid node itself, and reads of the state give zero on solids), and
    // the walk's overrun past its last node reloads the last one.  (The
    // interpolated wall's loads depend on one another: k_interp_wall applies
    // it after the launch to the slots the next pull reads.)
    // The lattice sizes and the thread's x pass through an empty asm per
    // node, so that what is derived from them (population and stencil
    // offsets) is recomputed instead of held across the walk; held, it spilled
    // the scalar registers and doubled the vector ones.  (The pointers stay
    // untouched: through the asm they would lose their address space.)
    auto fresh = [&](Dims& dd, int& xx) {
        dd = d0;
        xx = x0;
        asm volatile("" : "+s"(dd.N), "+s"(dd.px), "+s"(dd.nx), "+s"(dd.ny), "+s"(dd.nz), "+s"(dd.off));
        asm volatile("" : "+v"(xx));
    };
    auto node_of = [&](int n, int& y, int& z) {
        z = z0 + n / TY;
        y = y0 + n % TY;
    };
    // the class of node n (past the last node: of the last one, unused)
    auto load_cls = [&](int n) -> uint8_t {
        Dims dd;
        int xx, y, z;
        fresh(dd, xx);
        node_of(n < nn ? n : nn - 1, y, z);
        return at(cls, nid32(dd, xx, y, z));
    };
    // the wall mask of a boundary fluid node, else a shared dummy read
    auto load_mask = [&](int n, uint8_t c) -> uint32_t {
        Dims dd;
        int xx, y, z;
        fresh(dd, xx);
        node_of(n < nn ? n : nn - 1, y, z);
        const bool b = n < nn && (c & CLS_BOUNDARY) && (c & CLS_MASK) == CLS_FLUID;
        const uint32_t m = at(bc.nbmask, b ? nid32(dd, xx, y, z) : 0u);
        return b ? m : 0u;
    };
    // the force: under the chemical-potential model from the rho and mu
    // stencils (Eq. 7), loaded with the populations; under the pseudopotential
    // model from the array k_force filled
    ForceStencil<L, R> Ga, Gb;
    auto issue = [&](int n, uint32_t m, R S[L::Q], R F[3], ForceStencil<L, R>& G) {
        Dims dd;
        int xx, y, z;
        fresh(dd, xx);
        node_of(n < nn ? n : nn - 1, y, z);
        const uint32_t ix = nid32(dd, xx, y, z);
        if constexpr (SC) {
            F[0] = at(force, ix);
            F[1] = at(force + dd.N, ix);
            F[2] = at(force + 2 * dd.N, ix);
        } else if constexpr (RING) {
            // y neighbours and plane z + 2 from memory, the rest from the ring:
            // the z neighbours from the thread's own slots, the x neighbours
            // from the slots of plane z of the neighbouring columns, written
            // two planes earlier with plane-end barriers in between
            const int nc = n < nn ? n : nn - 1, r = nc % TY, zz = nc / TY;
            const Nbr ox = nbr_offsets(xx, dd.nx, 1), oy = nbr_offsets(y, dd.ny, dd.px);
            const Nbr oz = nbr_offsets(z, dd.nz, dd.px * dd.ny);
            G.v[5] = at(rho, ix + (uint32_t)oy.m2);
            G.v[6] = at(rho, ix + (uint32_t)oy.m1);
            G.v[7] = at(rho, ix + (uint32_t)oy.p1);
            G.v[8] = at(rho, ix + (uint32_t)oy.p2);
            G.v[17] = at(mu, ix + (uint32_t)oy.m2);
            G.v[18] = at(mu, ix + (uint32_t)oy.m1);
            G.v[19] = at(mu, ix + (uint32_t)oy.p1);
            G.v[20] = at(mu, ix + (uint32_t)oy.p2);
            G.v[12] = at(rho, ix + (uint32_t)oz.p2);
            G.v[24] = at(mu, ix + (uint32_t)oz.p2);
            const int s0 = zz & 3, sm2 = (zz + 2) & 3, sm1 = (zz + 3) & 3, sp1 = (zz + 1) & 3;
            G.v[1] = ring[s0][r][0][xx + ox.m2];
            G.v[2] = ring[s0][r][0][xx + ox.m1];
            G.v[3] = ring[s0][r][0][xx + ox.p1];
            G.v[4] = ring[s0][r][0][xx + ox.p2];
            G.v[13] = ring[s0][r][1][xx + ox.m2];
            G.v[14] = ring[s0][r][1][xx + ox.m1];
            G.v[15] = ring[s0][r][1][xx + ox.p1];
            G.v[16] = ring[s0][r][1][xx + ox.p2];
            G.v[0] = ring[s0][r][0][xx];
            G.v[9] = ring[sm2][r][0][xx];
            G.v[10] = ring[sm1][r][0][xx];
            G.v[11] = ring[sp1][r][0][xx];
            G.v[21] = ring[sm2][r][1][xx];
            G.v[22] = ring[sm1][r][1][xx];
            G.v[23] = ring[sp1][r][1][xx];
        } else {
            force_stencil_load<L, R, false>(rho, mu, dd, xx, y, z, G);  // every offset in bounds: unconditional
        }
        gather_issue<L, R, PULL>(fin, dd, ix, xx, y, z, m, S);
    };
    if constexpr (RING) {
        // planes z0 - 2 .. z0 + 1 of every row of the tile
        const Nbr oz = nbr_offsets(z0, d.nz, d.px * d.ny);
        const int off[4] = {0, oz.p1, oz.m2, oz.m1};  // slots of planes z0, z0 + 1, z0 - 2, z0 - 1
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const uint32_t ix = nid32(d, x, y0 + r, z0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ring[k][r][0][x] = at(rho, ix + (uint32_t)off[k]);
                ring[k][r][1][x] = at(mu, ix + (uint32_t)off[k]);
            }
        }
        lds_barrier();  // the first plane's x neighbours are other threads' slots
    }

    uint8_t c0 = load_cls(0), c1 = load_cls(1), c2 = load_cls(2);
    uint32_t m0 = load_mask(0, c0), m1 = load_mask(1, c1);

    // One node of the walk: node n from the stage (Scur, Fcur, Gcur), while
    // node n + 1 is issued into (Snext, Fnext, Gnext).
    auto node = [&](int n, R(&Scur)[L::Q], R(&Fcur)[3], ForceStencil<L, R>& Gcur, R(&Snext)[L::Q],
                    R(&Fnext)[3], ForceStencil<L, R>& Gnext) {
        // stages ahead: class of n+3, wall mask of n+2, populations of n+1
        const uint8_t c3 = load_cls(n + 3);
        const uint32_t m2 = load_mask(n + 2, c2);
        issue(n + 1, m1, Snext, Fnext, Gnext);

        Dims dd;
        int xx, y, z;
        fresh(dd, xx);
        node_of(n, y, z);
        const int r = n % TY, zz = n / TY, par = zz & 1;
        const int sc = z % 3, sn = (z + 1) % 3, sp = (z + 2) % 3;  // slots of planes z, z + 1, z - 1
        if constexpr (RING) {
            // plane z + 2 of this row into the slot of plane z - 2
            ring[(zz + 2) & 3][r][0][xx] = Gcur.v[12];
            ring[(zz + 2) & 3][r][1][xx] = Gcur.v[24];
        }
        // What leaves x: f*_i, or nothing from a solid node.  A population that
        // leaves toward a wall is also added to the solid node it points to;
        // that node is on the first solid layer, whose density the fill of
        // Eq. 14 sets afterwards, so the addition is harmless and saves a select.
        C v[L::Q];
        C own = C(0);  // what the wall returns to x
        {
            const bool live = (c0 & CLS_MASK) == CLS_FLUID;
            const uint32_t idx = nid32(dd, xx, y, z);
            // a solid node's collision runs on values nothing uses; its results
            // go to its own slots and add nothing to the densities
            R fo[L::Q];
            C Fx, Fy, Fz;
            if constexpr (SC) {
                Fx = (C)Fcur[0];
                Fy = (C)Fcur[1];
                Fz = (C)Fcur[2];
            } else {
                force_from_stencil<L, R, C, false>(Gcur, cp, tstep, Fx, Fy, Fz);
            }
            collide_values<L, R, C, MRT>(Scur, Fx, Fy, Fz, cp, fo);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                // five arrays per base address, 32-bit offsets from it
                const int g = i / 5 * 5;
                put<true>(&at(fout + (size_t)g * dd.N, (uint32_t)(i - g) * (uint32_t)dd.N + idx), fo[i]);
            }
#pragma unroll
            for (int i = 0; i < L::Q; ++i) v[i] = live ? (C)fo[i] : C(0);
            if (__builtin_amdgcn_ballot_w64(m0 != 0u) != 0) {  // a wave with wall links (uniform branch)
#pragma unroll
                for (int i = 1; i < L::Q; ++i) own += ((m0 >> i) & 1u) ? v[i] : C(0);
            }
        }
        // row groups with their x shifts
        C grp[5];
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            const C vp = v[RowGroups::GRP[g][1]], vm = v[RowGroups::GRP[g][2]];
            grp[g] = v[RowGroups::GRP[g][0]] + lane_from_below(vp) + lane_from_above(vm);
            if (lane == 63) edge[par][0][wave][r][g] = vp;
            if (lane == 0) edge[par][1][wave][r][g] = vm;
        }
        acc[r + 1][sc][x0] += grp[0] + own;
        acc[r + 2][sc][x0] += grp[1];
        acc[r][sc][x0] += grp[2];
        acc[r + 1][sn][x0] += grp[3];
        acc[r + 1][sp][x0] += grp[4];
        acc[r + 2][sn][x0] += v[RowGroups::PP];
        acc[r][sp][x0] += v[RowGroups::MM];
        acc[r + 2][sp][x0] += v[RowGroups::PM];
        acc[r][sn][x0] += v[RowGroups::MP];

        if (r == TY - 1) {
            // the plane is done: x-moving populations across wave boundaries
            // (periodic in x), then target plane z - 1 is complete
            lds_barrier();
            if (lane == 0 || lane == 63) {
                const int side = lane == 0 ? 0 : 1;
                const int w = lane == 0 ? (wave == 0 ? nw - 1 : wave - 1) : (wave + 1 == nw ? 0 : wave + 1);
#pragma unroll
                for (int rr = 0; rr < TY; ++rr) {
                    const C* e = edge[par][side][w][rr];
                    acc[rr + 1][sc][x0] += e[0];
                    acc[rr + 2][sc][x0] += e[1];
                    acc[rr][sc][x0] += e[2];
                    acc[rr + 1][sn][x0] += e[3];
                    acc[rr + 1][sp][x0] += e[4];
                }
            }
            // inside the chunk plane z - 1 is stored; below the chunk (first
            // plane) it is the z neighbour's; its slot is cleared for plane z + 2
            C a[TY + 2];
#pragma unroll
            for (int k = 0; k < TY + 2; ++k) {
                a[k] = acc[k][sp][x0];
                acc[k][sp][x0] = C(0);
            }
            if (zz == 0) {
                const int zg = z0 >= 1 ? z0 - 1 : dd.nz - 1;
#pragma unroll
                for (int rr = 0; rr < TY; ++rr) at(gz, nid32(dd, xx, y0 + rr, zg)) = (R)a[rr + 1];
                at(gyz, nid32(dd, xx, ylo, zg)) = (R)a[0];
                at(gyz, nid32(dd, xx, yhi, zg)) = (R)a[TY + 1];
            } else {
#pragma unroll
                for (int rr = 0; rr < TY; ++rr) at(rho_next, nid32(dd, xx, y0 + rr, z - 1)) = (R)a[rr + 1];
                at(gy, nid32(dd, xx, ylo, z - 1)) = (R)a[0];
                at(gy, nid32(dd, xx, yhi, z - 1)) = (R)a[TY + 1];
            }
        }

        // advance the class and mask stages
        c0 = c1;
        c1 = c2;
        c2 = c3;
        m0 = m1;
        m1 = m2;
    };

    R Sa[L::Q], Fa[3], Sb[L::Q], Fb[3];
    issue(0, m0, Sa, Fa, Ga);
#pragma unroll 1
    for (int n = 0; n < nn; ++n) {
        node(n, Sa, Fa, Ga, Sb, Fb, Gb);
        // advance the population stage
#pragma unroll
        for (int i = 0; i < L::Q; ++i) Sa[i] = Sb[i];
        if constexpr (SC) {
            Fa[0] = Fb[0];
            Fa[1] = Fb[1];
            Fa[2] = Fb[2];
        } else {
#pragma unroll
            for (int k = 0; k < ForceStencil<L, R>::K; ++k) Ga.v[k] = Gb.v[k];
        }
    }
    // the chunk's last plane, and the plane above the chunk (the z neighbour's)
    const int zl = z0 + zc - 1, zg = z0 + zc < d.nz ? z0 + zc : 0;
    const int sl = zl % 3, sg = (zl + 1) % 3;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        at(rho_next, nid32(d, x, y0 + r, zl)) = (R)acc[r + 1][sl][x];
        at(gz, nid32(d, x, y0 + r, zg)) = (R)acc[r + 1][sg][x];
    }
    at(gy, nid32(d, x, ylo, zl)) = (R)acc[0][sl][x];
    at(gy, nid32(d, x, yhi, zl)) = (R)acc[TY + 1][sl][x];
    at(gyz, nid32(d, x, ylo, zg)) = (R)acc[0][sg][x];
    at(gyz, nid32(d, x, yhi, zg)) = (R)acc[TY + 1][sg][x];
}

// Adds the ghost sums to the edge rows (y % TY in {0, TY-1}) and edge planes
// (z % zc in {0, zc-1}) of k_step's tiles.  The edge rows are listed per chunk
// of zc planes: its two edge planes whole, then the 2 ny/TY edge rows of each
// plane between them.  A thread takes four consecutive nodes of a listed row
// (rows start on 64-node boundaries, so the four are one aligned vector);
// nrows rows in all.  With tick set, the launch also counts the step
// (ctl->t += 1), in place of k_finalize on steps that measure nothing.
template <typename R, int TY>
__global__ void __launch_bounds__(256) k_ghost(R* __restrict__ rho, const R* __restrict__ gy,
                                               const R* __restrict__ gz, const R* __restrict__ gyz, Dims d, int zc,
                                               long long nrows, DevCtl* __restrict__ tick) {
    typedef R V __attribute__((ext_vector_type(4)));
    const unsigned q = (unsigned)d.nx >> 2;
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    if (tick && g == 0) tick->t += 1;
    if (g >= nrows * (long long)q) return;
    const long long k = g / q;
    const int x = (int)(g - k * q) * 4;
    const int ein = 2 * (d.ny / TY);
    const long long per_chunk = 2LL * d.ny + (long long)(zc - 2) * ein;
    const int ch = (int)(k / per_chunk);
    long long rem = k - (long long)ch * per_chunk;
    int y, z;
    if (rem < d.ny) {
        z = ch * zc;
        y = (int)rem;
    } else if (rem < 2LL * d.ny) {
        z = ch * zc + zc - 1;
        y = (int)(rem - d.ny);
    } else {
        rem -= 2LL * d.ny;
        z = ch * zc + 1 + (int)(rem / ein);
        const int sr = (int)(rem % ein);
        y = (sr >> 1) * TY + ((sr & 1) ? TY - 1 : 0);
    }
    const int ry = y % TY, rz = z % zc;
    const bool ey = ry == 0 || ry == TY - 1, ez = rz == 0 || rz == zc - 1;
    const long long n = nid(d, x, y, z);
    const V r = *(const V*)(rho + n);
    const V a = ey ? *(const V*)(gy + n) : V(0);
    const V b = ez ? *(const V*)(gz + n) : V(0);
    const V c = (ey && ez) ? *(const V*)(gyz + n) : V(0);
    V out;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double v = (double)r[e];
        if (ey) v += (double)a[e];
        if (ez) v += (double)b[e];
        if (ey && ez) v += (double)c[e];
        out[e] = (R)v;
    }
    *(V*)(rho + n) = out;
}

// block reduction (256 threads) of per-thread liquid centroid sums
__device__ __forceinline__ void centroid_reduce_sums(unsigned long long cnt, unsigned long long sx,
                                                     unsigned long long sy, unsigned long long sz, MeasureSlots* ms) {
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

// Chemical potential (Eq. 11-12; psi of the pseudopotential model) of the
// density k_step and k_ghost completed, z-chunked as k_mu; besides, the check
// of the density that the split path's density pass makes, and on measure
// steps the liquid centroid sums of the measurement (Sec. III B).  The column
// values z-2 .. z+2 stay in registers as the walk moves up (one new load per
// plane), plane z+1's x and y neighbours are loaded before plane z's value is
// stored, and the store is unconditional (solid nodes write a sink slot: their
// mu is the wall value set with the solids), so that the loads do not wait for
// the stores.
template <class L, typename R, typename C, bool SC>
__global__ void __launch_bounds__(256) k_mu_step(const R* __restrict__ rho, R* __restrict__ mu,
                                                 const uint8_t* __restrict__ cls, Dims d, Thermo th,
                                                 DevCtl* __restrict__ ctl, double rho_m, R inv_b, R* __restrict__ sink) {
    int x, y, z0;
    tile_node_zc(d, x, y, z0);
    const bool in = x < d.nx && y < d.ny;
    const int xs = in ? x : 0, ys = in ? y : 0;
    const int z1 = z0 + d.zc < d.nz ? z0 + d.zc : d.nz;
    const Nbr ox = nbr_offsets(xs, d.nx, 1), oy = nbr_offsets(ys, d.ny, d.px);
    // the x and y neighbours of one plane (-2, -1, +1, +2 along x, then y) and the class
    auto load = [&](int z, R v[8], uint8_t& c) {
        const uint32_t ix = nid32(d, xs, ys, z);
        auto p = [&](int o) { return at(rho, ix + (uint32_t)o); };
        c = at(cls, ix);
        v[0] = p(ox.m2); v[1] = p(ox.m1); v[2] = p(ox.p1); v[3] = p(ox.p2);
        v[4] = p(oy.m2); v[5] = p(oy.m1); v[6] = p(oy.p1); v[7] = p(oy.p2);
    };
    // the column x, y: planes z - 2 .. z + 2 held in a sliding window, so that
    // each plane loads one new column value instead of five (periodic images)
    auto col = [&](int z) { return at(rho, nid32(d, xs, ys, wrapc(z, d.nz))); };
    unsigned long long cnt = 0, sx = 0, sy = 0, sz = 0;
    bool bad = false;
    R cur[8], nxt[8];
    R w0 = col(z0 - 2), w1 = col(z0 - 1), w2 = col(z0), w3 = col(z0 + 1), w4 = col(z0 + 2);
    uint8_t cc, cn;
    load(z0, cur, cc);
    for (int z = z0; z < z1; ++z) {
        load(z + 1 < z1 ? z + 1 : z, nxt, cn);
        const R w5 = col(z + 3);  // unconditional: counted, in bounds
        const bool fl = in && (cc & CLS_MASK) == CLS_FLUID;
        const C c0 = (C)w2;
        C m;
        if constexpr (SC) {
            m = C(1) - exp(-c0);  // pseudopotential model: psi(rho) = 1 - exp(-rho)
        } else {
            C lap = d2c<C>((C)cur[0], (C)cur[1], c0, (C)cur[2], (C)cur[3]);
            lap += d2c<C>((C)cur[4], (C)cur[5], c0, (C)cur[6], (C)cur[7]);
            lap += d2c<C>((C)w0, (C)w1, c0, (C)w3, (C)w4);
            m = (psi_prime<C>(c0, th) - (C)th.mu_ref) - (C)th.kappa * lap;
        }
        at(fl ? mu : sink, fl ? (uint32_t)nid(d, xs, ys, z) : (threadIdx.x & 1023u)) = (R)m;
        if (fl) {
            const R r0 = w2;
            bad = bad || !(r0 > R(0) && r0 < inv_b);  // also catches NaN
            if ((double)r0 >= rho_m) {
                cnt += 1;
                sx += (unsigned long long)x;
                sy += (unsigned long long)y;
                sz += (unsigned long long)z;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
        cc = cn;
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = w4;
        w4 = w5;
    }
    if (bad) atomicOr(&ctl->status, 1);
    if (measuring(ctl)) centroid_reduce_sums(cnt, sx, sy, sz, &ctl->m);
}

}  // namespace lbm
