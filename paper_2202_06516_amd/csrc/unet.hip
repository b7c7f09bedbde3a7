// unet.hip -- the learned warm start: a convolutional U-Net trained and run on
// gfx950 with hand-written BF16 MFMA kernels (FP32 accumulation), and the
// kernels that turn lattice fields into its inputs and targets and its output
// back into a mass-exact density field.
//
// The network maps (solid mask, wall chemical potential on the solid, drop
// volume plane) on a 2-D lattice to phi = (rho - rho_g) / (rho_l - rho_g) of
// the equilibrated drop.  Levels l = 0..L-1 carry C0 * 2^l channels: two 3x3
// same-padded convolutions with ReLU per level, 2x2 max pooling down, a 2x2
// stride-2 transposed convolution up, skip connections by channel
// concatenation (upsampled first, skip second), and a 1x1 head.  Activations
// and their gradients are NHWC BF16; master weights, gradients and the Adam
// moments are FP32, with BF16 copies for the products.
//
// Every product runs on MFMA 16x16x32 BF16 tiles with operands staged through
// LDS (four waves of 2 x 2 per group, the next stage's global loads in flight
// during the current stage's MFMAs), in three kernels:
//  - the 3x3 convolution and its data gradient (mirrored taps, transposed
//    weights, ReLU mask fused into the load) are tap-blocked: a stage holds
//    one input row of a pixel segment and the three taps of that row, and
//    feeds the three taps from LDS;
//  - the 3x3 weight gradient holds dY of a 32-pixel segment and the three
//    input rows around it, and accumulates all nine taps (split over pixel
//    chunks, partials summed in a fixed order: deterministic);
//  - the transposed convolution and its gradients use a generic implicit GEMM
//    whose loader functors gather 16-byte vectors along K or along M/N.
// Operands stored along M/N enter the MFMA through the transposing LDS read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"

namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef long long i64;

constexpr int BK = 32;    // K chunk per LDS stage (one MFMA 16x16x32 step)
constexpr int CPAD = 8;   // the network input is padded to 8 channels (one 16-byte vector)

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// MFMA operand of row r from an LDS stage stored k-major by row ([k][rows],
// row contiguous), with the transposing 64-bit LDS read.  Within each group of
// 16 lanes, lane t addresses 4 consecutive rows at one k, and lane i of the
// group receives, in slot j, element i % 4 of the vector that lane
// 4 j + i / 4 addressed.  Lane t = 4 j + q of group g therefore addresses
// rows 4 q .. 4 q + 3 at k = 8 g + j (and 8 g + 4 + j for the second read),
// which leaves lane i holding row i at k = 8 g .. 8 g + 7: the layout the
// MFMA takes.  p = &stage[0][row0]; stride = elements per k row.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
__device__ __forceinline__ bf16x8 ld_tr8(const bf16* p, int stride, int lane) {
    const int t = lane & 15, g = lane >> 4;
    const bf16* q = p + (8 * g + (t >> 2)) * stride + 4 * (t & 3);
    const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)q);
    const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(q + 4 * stride));
    bf16x8 r;
    __builtin_memcpy(&r, &lo, 8);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 8, &hi, 8);
    return r;
}
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (bf16)0.f;
    return v;
}
__device__ __forceinline__ bf16x8 masked8(bf16x8 v, bf16x8 m) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (!((float)m[j] > 0.f)) v[j] = (bf16)0.f;
    return v;
}

// ---------------------------------------------------------------------------
// Operand loaders.  elem(mn, k) is element (row mn, reduction index k) of A
// (mn = m) or of B (mn = n); vec(row(mn), mn, k) returns the 8 elements that
// follow along the loader's vector axis: k..k+7 when KMAJ, mn..mn+7
// otherwise.  A thread's mn is fixed for the whole K loop, so row(mn) holds
// what depends on it alone (pixel coordinates, tap and channel), computed once
// per tile.  The GEMM calls vec only for vectors wholly inside the matrix.
// ---------------------------------------------------------------------------

// Division by a kernel-invariant divisor d >= 1 of 0 <= n < 2^31: multiply by
// a precomputed 32-bit reciprocal and shift (the round-up method of Granlund
// and Montgomery); all GEMM indices stay below 2^31.
struct FastDiv {
    uint32_t d, m, s;
    __device__ __forceinline__ uint32_t div(uint32_t n) const { return (__umulhi(n, m) + n) >> s; }
};
inline FastDiv fastdiv(uint32_t d) {
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    return FastDiv{d, (uint32_t)((1ull << 32) * ((1ull << s) - d) / d + 1), s};
}

// pixel index m of a B x H x W grid -> (b, h, w)
struct Grid {
    int B, H, W;
    FastDiv fH, fW;
    __device__ __forceinline__ void split(uint32_t m, int& b, int& h, int& w) const {
        const uint32_t q = fW.div(m);
        w = (int)(m - q * (uint32_t)W);
        const uint32_t bb = fH.div(q);
        h = (int)(q - bb * (uint32_t)H);
        b = (int)bb;
    }
};
inline Grid make_grid(int B, int H, int W) { return Grid{B, H, W, fastdiv((uint32_t)H), fastdiv((uint32_t)W)}; }

// B of the transposed convolution: element (n = (2a + b) Co + co, k = ci) = Wb[n * K + k]
struct RowsK {
    static constexpr bool KMAJ = true;
    const bf16* P;
    i64 K;
    __device__ __forceinline__ bf16 elem(i64 n, i64 k) const { return P[n * K + k]; }
    struct Row {};
    __device__ __forceinline__ Row row(i64) const { return Row{}; }
    __device__ __forceinline__ bf16x8 vec(const Row&, i64 n, i64 k) const { return ld8(P + n * K + k); }
};

// A of the transposed convolution: element (m = pixel, k = ci) = X[pixel][ci]
struct RowsKA {
    static constexpr bool KMAJ = true;
    const bf16* X;
    int C;
    __device__ __forceinline__ bf16 elem(i64 m, i64 k) const { return X[m * C + k]; }
    struct Row {};
    __device__ __forceinline__ Row row(i64) const { return Row{}; }
    __device__ __forceinline__ bf16x8 vec(const Row&, i64 m, i64 k) const { return ld8(X + m * C + k); }
};

// output pixel of the transposed convolution for input pixel m and offset ab = 2a + b
struct UpMap {
    Grid g;  // the input grid; the output grid is B x 2H x 2W
    __device__ __forceinline__ i64 out(i64 m, int ab) const {
        int b, h, w;
        g.split((uint32_t)m, b, h, w);
        return ((i64)b * 2 * g.H + 2 * h + (ab >> 1)) * (2 * g.W) + 2 * w + (ab & 1);
    }
};

// A of the transposed convolution's data gradient: element (m = input pixel,
// k = ab * Co + co) = dY[out(m, ab)][co]
struct UpGatherK {
    static constexpr bool KMAJ = true;
    const bf16* dY;
    UpMap u;
    int Co;
    FastDiv fCo;
    __device__ __forceinline__ i64 at(i64 m, i64 k) const {
        const uint32_t kk = (uint32_t)k, ab = fCo.div(kk);
        return u.out(m, (int)ab) * Co + (kk - ab * (uint32_t)Co);
    }
    __device__ __forceinline__ bf16 elem(i64 m, i64 k) const { return dY[at(m, k)]; }
    struct Row {
        i64 base;  // output pixel (2h, 2w) of input pixel m
    };
    __device__ __forceinline__ Row row(i64 m) const { return Row{u.out(m, 0)}; }
    __device__ __forceinline__ bf16x8 vec(const Row& r, i64, i64 k) const {
        const uint32_t kk = (uint32_t)k, ab = fCo.div(kk);
        const i64 q = r.base + (i64)(ab >> 1) * (2 * u.g.W) + (ab & 1);
        return ld8(dY + q * Co + (kk - ab * (uint32_t)Co));
    }
};

// B of the transposed convolution's data gradient: element (n = ci, k = row) = Wt[row][ci]
struct RowsN {
    static constexpr bool KMAJ = false;
    const bf16* P;
    int C;
    __device__ __forceinline__ bf16 elem(i64 n, i64 k) const { return P[k * C + n]; }
    struct Row {};
    __device__ __forceinline__ Row row(i64) const { return Row{}; }
    __device__ __forceinline__ bf16x8 vec(const Row&, i64 n, i64 k) const { return ld8(P + k * C + n); }
};

// A of the transposed convolution's weight gradient: element (m = ab * Co + co,
// k = input pixel) = dY[out(k, ab)][co]
struct UpGatherM {
    static constexpr bool KMAJ = false;
    const bf16* dY;
    UpMap u;
    int Co;
    FastDiv fCo;
    __device__ __forceinline__ i64 at(i64 m, i64 k) const {
        const uint32_t mm = (uint32_t)m, ab = fCo.div(mm);
        return u.out(k, (int)ab) * Co + (mm - ab * (uint32_t)Co);
    }
    __device__ __forceinline__ bf16 elem(i64 m, i64 k) const { return dY[at(m, k)]; }
    struct Row {};
    __device__ __forceinline__ Row row(i64) const { return Row{}; }
    __device__ __forceinline__ bf16x8 vec(const Row&, i64 m, i64 k) const { return ld8(dY + at(m, k)); }
};

// B of the transposed convolution's weight gradient: element (n = ci, k = pixel)
// = X[pixel][ci] for n < C, 1 for n = C (the bias column)
struct ColsOnes {
    static constexpr bool KMAJ = false;
    const bf16* X;
    int C;
    __device__ __forceinline__ bf16 elem(i64 n, i64 k) const { return n == C ? (bf16)1.f : X[k * C + n]; }
    struct Row {};
    __device__ __forceinline__ Row row(i64) const { return Row{}; }
    __device__ __forceinline__ bf16x8 vec(const Row&, i64 n, i64 k) const { return ld8(X + k * C + n); }
};

// ---------------------------------------------------------------------------
// Epilogues (called once per output element, with bounds checks inside)
// ---------------------------------------------------------------------------
struct EpiBiasRelu {  // Y[m][n] = relu(acc + bias[n]) in BF16
    bf16* Y;
    const float* bias;
    i64 M;
    int N;
    __device__ __forceinline__ void operator()(i64 m, i64 n, float v) const {
        if (m >= M || n >= N) return;
        v += bias[n];
        Y[m * N + n] = (bf16)(v > 0.f ? v : 0.f);
    }
};

struct EpiSplit {  // columns [0, N1) -> Y1[m][n], [N1, N1 + N2) -> Y2[m][n - N1] (BF16)
    bf16* Y1;
    bf16* Y2;
    i64 M;
    int N1, N2;
    __device__ __forceinline__ void operator()(i64 m, i64 n, float v) const {
        if (m >= M || n >= N1 + N2) return;
        if (n < N1) Y1[m * N1 + n] = (bf16)v;
        else Y2[m * N2 + (n - N1)] = (bf16)v;
    }
};

struct EpiPartial {  // split-K partial sums, FP32 [z][M][N]
    float* P;
    i64 M, N;
    __device__ __forceinline__ void operator()(i64 m, i64 n, float v) const {
        if (m >= M || n >= N) return;
        P[(i64)blockIdx.z * M * N + m * N + n] = v;
    }
};

struct EpiUp {  // column n = ab * Co + co of input pixel m -> Y[out(m, ab)][co] = acc + bias[co]
    bf16* Y;
    const float* bias;
    UpMap u;
    i64 M;
    int Co;
    FastDiv fCo;
    __device__ __forceinline__ void operator()(i64 m, i64 n, float v) const {
        if (m >= M || n >= 4LL * Co) return;
        const uint32_t nn = (uint32_t)n, ab = fCo.div(nn), co = nn - ab * (uint32_t)Co;
        Y[u.out(m, (int)ab) * Co + co] = (bf16)(v + bias[co]);
    }
};

// ---------------------------------------------------------------------------
// The GEMM: C[M][N] = sum_k A(m, k) B(k, n) over k in [z kchunk, (z+1) kchunk)
// ---------------------------------------------------------------------------
template <class L>
__device__ __forceinline__ bf16x8 load_vec(const L& l, const typename L::Row& row, i64 mn, i64 k, i64 mnlim,
                                          i64 klim) {
    if constexpr (L::KMAJ) {
        if (mn < mnlim && k + 8 <= klim) return l.vec(row, mn, k);
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (mn < mnlim && k + j < klim) ? l.elem(mn, k + j) : (bf16)0.f;
        return v;
    } else {
        if (k < klim && mn + 8 <= mnlim) return l.vec(row, mn, k);
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (k < klim && mn + j < mnlim) ? l.elem(mn + j, k) : (bf16)0.f;
        return v;
    }
}

// tile coordinates of vector v of a BMN x BK stage
template <bool KMAJ, int BMN>
__device__ __forceinline__ void vec_coord(int v, int& mn, int& kk) {
    if (KMAJ) {
        mn = v / (BK / 8);
        kk = (v % (BK / 8)) * 8;
    } else {
        kk = v / (BMN / 8);
        mn = (v % (BMN / 8)) * 8;
    }
}

template <int BM, int BN, class LA, class LB, class EPI>
__global__ void __launch_bounds__(256) k_gemm(LA A, LB B, EPI epi, i64 M, i64 N, i64 K, i64 kchunk) {
    // LDS: K-major operands as [rows][BK + 8], M/N-major as [BK][rows + 8]
    constexpr int AC = (LA::KMAJ ? BK : BM) + 8, BC = (LB::KMAJ ? BK : BN) + 8;
    constexpr int AR = LA::KMAJ ? BM : BK, BR = LB::KMAJ ? BN : BK;
    __shared__ __attribute__((aligned(16))) bf16 As[2][AR * AC];  // two stages: one barrier per K chunk
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BR * BC];
    constexpr int NVA = BM * BK / 8, NVB = BN * BK / 8;
    constexpr int RA = (NVA + 255) / 256, RB = (NVB + 255) / 256;
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    static_assert(TM >= 1 && TN >= 1, "tile too small");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const i64 m0 = (i64)blockIdx.x * BM, n0 = (i64)blockIdx.y * BN;
    const i64 kb = (i64)blockIdx.z * kchunk;
    const i64 ke = kb + kchunk < K ? kb + kchunk : K;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    bf16x8 ra[RA], rb[RB];
    // per-slot row state, fixed for the whole K loop
    typename LA::Row rowa[RA];
    typename LB::Row rowb[RB];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
        int mn, kk;
        vec_coord<LA::KMAJ, BM>(tid + 256 * r, mn, kk);
        rowa[r] = A.row(m0 + mn);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        int mn, kk;
        vec_coord<LB::KMAJ, BN>(tid + 256 * r, mn, kk);
        rowb[r] = B.row(n0 + mn);
    }
    auto fetch = [&](i64 k0) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int v = tid + 256 * r;
            if (NVA % 256 == 0 || v < NVA) {
                int mn, kk;
                vec_coord<LA::KMAJ, BM>(v, mn, kk);
                ra[r] = load_vec(A, rowa[r], m0 + mn, k0 + kk, M, ke);
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int v = tid + 256 * r;
            if (NVB % 256 == 0 || v < NVB) {
                int mn, kk;
                vec_coord<LB::KMAJ, BN>(v, mn, kk);
                rb[r] = load_vec(B, rowb[r], n0 + mn, k0 + kk, N, ke);
            }
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int v = tid + 256 * r;
            if (NVA % 256 == 0 || v < NVA) {
                int mn, kk;
                vec_coord<LA::KMAJ, BM>(v, mn, kk);
                *reinterpret_cast<bf16x8*>(&As[st][LA::KMAJ ? mn * AC + kk : kk * AC + mn]) = ra[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int v = tid + 256 * r;
            if (NVB % 256 == 0 || v < NVB) {
                int mn, kk;
                vec_coord<LB::KMAJ, BN>(v, mn, kk);
                *reinterpret_cast<bf16x8*>(&Bs[st][LB::KMAJ ? mn * BC + kk : kk * BC + mn]) = rb[r];
            }
        }
    };

    // stage st is read by the MFMAs while the next chunk's global loads are in
    // flight and then land in stage st ^ 1; the barrier that ends a chunk
    // both publishes st ^ 1 and retires every read of st
    if (kb < ke) {
        fetch(kb);
        stash(0);
    }
    __syncthreads();
    int st = 0;
    for (i64 k0 = kb; k0 < ke; k0 += BK) {
        const bool more = k0 + BK < ke;
        if (more) fetch(k0 + BK);
        const bf16* As_ = As[st];
        const bf16* Bs_ = Bs[st];
        // MFMA 16x16x32 operands: lane holds row (lane % 16), k = 8 (lane / 16) .. + 7
        const int kg = (lane >> 4) * 8, rl = lane & 15;
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int row = wm + i * 16 + rl;
            if constexpr (LA::KMAJ) {
                a[i] = *reinterpret_cast<const bf16x8*>(&As_[row * AC + kg]);
            } else {
                a[i] = ld_tr8(&As_[wm + i * 16], AC, lane);
            }
        }
#pragma unroll
        for (int i = 0; i < TN; ++i) {
            const int row = wn + i * 16 + rl;
            if constexpr (LB::KMAJ) {
                b[i] = *reinterpret_cast<const bf16x8*>(&Bs_[row * BC + kg]);
            } else {
                b[i] = ld_tr8(&Bs_[wn + i * 16], BC, lane);
            }
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
    // D layout: lane holds column (lane % 16), rows 4 (lane / 16) .. + 3
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                epi(m0 + wm + i * 16 + (lane >> 4) * 4 + q, n0 + wn + j * 16 + (lane & 15), acc[i][j][q]);
}

// ---------------------------------------------------------------------------
// Weight gradient of a 3x3 convolution with all nine taps in one workgroup
// ---------------------------------------------------------------------------
// P[z][co][tap Cp + c] = sum over the pixels p of chunk z of dYm[p][co] X[p + s(tap)][c],
// P[z][co][9 Cp] = sum dYm[p][co] (the bias), dYm = dY where the ReLU output
// Y > 0, X = [X1 | X2] (C1 + C2 = Cp channels), s(tap) the tap's pixel shift
// (zero outside the image).  The reduction runs over segments of 32 pixels
// of one image row: a stage holds dYm of the segment ([32][BM] per pixel)
// and X of the three rows around it ([3][34][BN]), so each X element read
// from memory feeds the nine taps from LDS.  A workgroup is G groups of W
// waves; group q takes every G-th segment of the chunk with stages of its
// own, and the groups' sums are added in LDS in group order at the end
// (deterministic).  Within a group the W waves share the BM = 16 TM output
// channels and split the BN = 16 TN W input channels, each 16 TM x 16 TN of
// (co, c) for every tap; both operands enter the MFMA through the transposing
// LDS read.
constexpr int SEG = 32;  // pixels per segment = one MFMA K step

template <int TM, int TN, int W, int G>
__global__ void __launch_bounds__(64 * W * G) k_wgrad3x3(const bf16* __restrict__ dY, const bf16* __restrict__ Y,
                                                      const bf16* __restrict__ X1, const bf16* __restrict__ X2,
                                                      int C1, int C2, int Co, Grid g, int segs_row, int nsegs,
                                                      int spc, float* __restrict__ P) {
    constexpr int NT = 64 * W;  // threads per group
    constexpr int BM = 16 * TM, BN = 16 * TN * W, DC = BM + 8, XC = BN + 8, XW = SEG + 2;
    constexpr int NVD = SEG * BM / 8, NVX = 3 * XW * BN / 8;
    constexpr int RD = (NVD + NT - 1) / NT, RX = (NVX + NT - 1) / NT;
    constexpr int DS = SEG * DC, XS = 3 * XW * XC;  // elements per stage
    __shared__ __attribute__((aligned(16))) bf16 lds[G * 2 * (DS + XS)];
    static_assert(BM * BN * 4 <= G * 2 * (DS + XS) * 2, "reduction buffer");

    const int q = threadIdx.x / NT, tid = threadIdx.x % NT, lane = tid & 63, wave = tid >> 6;
    bf16* Ds = lds + q * 2 * (DS + XS);  // this group's two stages: Ds[st], then Xs[st]
    bf16* Xs = Ds + 2 * DS;
    const int co0 = blockIdx.x * BM, c0 = blockIdx.y * BN, Cp = C1 + C2;
    const int s0 = blockIdx.z * spc, s1 = min(nsegs, s0 + spc);
    const int iters = (s1 - s0 + G - 1) / G;  // the same for every group (barriers)
    const int wm = 0, wn = wave * 16 * TN;
    const bool bias = blockIdx.y == 0;

    floatx4 acc[9][TM][TN];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[t][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;

    bf16x8 rd[RD], rx[RX];
    auto fetch = [&](int s) {  // s < s1
        const int row = s / segs_row, w0 = (s - row * segs_row) * SEG;
        const int b = row / g.H, h = row - b * g.H;
#pragma unroll
        for (int r = 0; r < RD; ++r) {
            const int v = tid + NT * r;
            if (NVD % NT == 0 || v < NVD) {
                const int px = v / (BM / 8), cv = (v % (BM / 8)) * 8;
                const int w = w0 + px, co = co0 + cv;
                rd[r] = zero8();
                if (w < g.W && co < Co) {
                    const i64 i = (((i64)b * g.H + h) * g.W + w) * Co + co;
                    rd[r] = masked8(ld8(dY + i), ld8(Y + i));
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int v = tid + NT * r;
            if (NVX % NT == 0 || v < NVX) {
                const int dr = v / (XW * BN / 8), rem = v - dr * (XW * BN / 8);
                const int j = rem / (BN / 8), cv = (rem % (BN / 8)) * 8;
                const int hh = h + dr - 1, w = w0 + j - 1, c = c0 + cv;
                rx[r] = zero8();
                if (hh >= 0 && hh < g.H && w >= 0 && w < g.W && c < Cp) {
                    const i64 p = ((i64)b * g.H + hh) * g.W + w;
                    rx[r] = c < C1 ? ld8(X1 + p * C1 + c) : ld8(X2 + p * C2 + (c - C1));
                }
            }
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < RD; ++r) {
            const int v = tid + NT * r;
            if (NVD % NT == 0 || v < NVD) {
                const int px = v / (BM / 8), cv = (v % (BM / 8)) * 8;
                *reinterpret_cast<bf16x8*>(&Ds[st * DS + px * DC + cv]) = rd[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int v = tid + NT * r;
            if (NVX % NT == 0 || v < NVX) {
                const int dr = v / (XW * BN / 8), rem = v - dr * (XW * BN / 8);
                const int j = rem / (BN / 8), cv = (rem % (BN / 8)) * 8;
                *reinterpret_cast<bf16x8*>(&Xs[st * XS + (dr * XW + j) * XC + cv]) = rx[r];
            }
        }
    };

    // group q handles segments s0 + q + G it, it < iters, where they exist
    if (iters > 0 && s0 + q < s1) {
        fetch(s0 + q);
        stash(0);
    }
    __syncthreads();
    int st = 0;
    for (int it = 0; it < iters; ++it) {
        const int s = s0 + q + G * it;
        const bool have = s < s1, more = s + G < s1;
        if (more) fetch(s + G);
        if (have) {
            const bf16* D_ = Ds + st * DS;
            const bf16* X_ = Xs + st * XS;
            bf16x8 a[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = ld_tr8(D_ + wm + 16 * i, DC, lane);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, dx = t % 3;  // offsets into the stage's three rows and 34 columns
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const bf16x8 bv = ld_tr8(X_ + (dy * XW + dx) * XC + wn + 16 * j, XC, lane);
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[t][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv, acc[t][i][j], 0, 0, 0);
                }
            }
            if (bias && tid < BM) {
#pragma unroll 8
                for (int px = 0; px < SEG; ++px) bsum += (float)D_[px * DC + tid];
            }
        }
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }

    // sum the groups in LDS (group order), one tap at a time; group 0 writes
    const i64 N1 = 9LL * Cp + 1;
    float* Pz = P + (i64)blockIdx.z * Co * N1;
    float* red = reinterpret_cast<float*>(lds);  // [BM][BN]
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        for (int k = 1; k < G; ++k) {
            if (q == k) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            red[(wm + 16 * i + (lane >> 4) * 4 + e) * BN + wn + 16 * j + (lane & 15)] = acc[t][i][j][e];
            }
            __syncthreads();
            if (q == 0) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[t][i][j][e] += red[(wm + 16 * i + (lane >> 4) * 4 + e) * BN + wn + 16 * j + (lane & 15)];
            }
            __syncthreads();
        }
        if (q == 0) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int c = c0 + wn + 16 * j + (lane & 15);
                    if (c >= Cp) continue;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int co = co0 + wm + 16 * i + (lane >> 4) * 4 + e;
                        if (co < Co) Pz[(i64)co * N1 + (i64)t * Cp + c] = acc[t][i][j][e];
                    }
                }
        }
    }
    if (bias) {
        for (int k = 1; k < G; ++k) {
            if (q == k && tid < BM) red[tid] = bsum;
            __syncthreads();
            if (q == 0 && tid < BM) bsum += red[tid];
            __syncthreads();
        }
        if (q == 0 && tid < BM && co0 + tid < Co) Pz[(i64)(co0 + tid) * N1 + 9LL * Cp] = bsum;
    }
}

// ---------------------------------------------------------------------------
// 3x3 convolution and its data gradient, tap-blocked through LDS
// ---------------------------------------------------------------------------
// out[p][n] = epi(sum over taps u and input channels c of In[p + s(u)][c] B(n, u, c))
// with In = [X1 | X2] (C1 + C2 = Cin channels; zero outside the image and,
// when mask is set, where mask <= 0), s(u) = (u / 3 - 1, u % 3 - 1), and
//   forward (WT = false): B(n, u, c) = W[n][u][c]       (n = output channel)
//   data gradient (WT):   B(n, u, c) = W[c][8 - u][n]   (n = input channel of the forward)
// for BF16 weights W [Co][9][Cp].  The pixels are cut into segments of BM
// pixels of one image row; a workgroup owns BN channels and a strided set
// of segments, and runs through the stages of all of them in one pipeline
// (the next stage's loads in flight during the current stage's MFMAs, across
// segment boundaries too).  A stage is (32 input channels, one tap row dy)
// of a segment: the input row h + dy - 1 over BM + 2 pixels and the weights
// of the three taps of that row, so each staged input row feeds the three
// taps from LDS.  Workgroup ids are dealt to the 8 XCDs round-robin; the
// segment slots are permuted so that each XCD works on one contiguous band
// of segments (neighbouring rows share its L2).
__device__ __forceinline__ int xcd_slot(unsigned b, unsigned G) {
    const unsigned q = G >> 3, r = G & 7u, xcd = b & 7u, loc = b >> 3;
    return (int)((xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + loc);
}

template <int TM, int TN, bool WT, class EPI>
__global__ void __launch_bounds__(256) k_conv3x3(const bf16* __restrict__ X1, const bf16* __restrict__ X2,
                                                 const bf16* __restrict__ mask, int C1, int C2,
                                                 const bf16* __restrict__ Wb, int Cp, int Nout, Grid g, int segs_row,
                                                 int nsegs, EPI epi) {
    constexpr int BM = 32 * TM, BN = 32 * TN, XW = BM + 2, XC = BK + 8;
    constexpr int WC = WT ? BN + 8 : BK + 8, WR = WT ? BK : BN;  // per tap: [WR][WC]
    constexpr int XS = XW * XC, WS = 3 * WR * WC;
    constexpr int NVX = XW * BK / 8, NVW = 3 * BN * BK / 8;
    constexpr int RX = (NVX + 255) / 256, RW = (NVW + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 Xs[2][XS];
    __shared__ __attribute__((aligned(16))) bf16 Ws[2][WS];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = xcd_slot(blockIdx.x, gridDim.x), stride = (int)gridDim.x;
    const int n0 = blockIdx.y * BN, Cin = C1 + C2;
    const int wm = (wave >> 1) * 16 * TM, wn = (wave & 1) * 16 * TN;
    const int nst = 3 * ((Cin + BK - 1) / BK);  // stages per segment: (channel chunk, dy)
    const int total = slot < nsegs ? ((nsegs - 1 - slot) / stride + 1) * nst : 0;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // stage k of this workgroup: segment slot + (k / nst) stride, (chunk, dy) from k % nst
    auto locate = [&](int k, int& b, int& h, int& w0, int& cc, int& dy) {
        const int ks = k / nst, kk = k - ks * nst;
        const int seg = slot + ks * stride, row = seg / segs_row;
        w0 = (seg - row * segs_row) * BM;
        b = row / g.H;
        h = row - b * g.H;
        cc = (kk / 3) * BK;
        dy = kk - (kk / 3) * 3;
    };
    bf16x8 rx[RX], rw[RW];
    auto fetch = [&](int k) {
        int b, h, w0, cc, dy;
        locate(k, b, h, w0, cc, dy);
        const int hh = h + dy - 1;
        const bool hin = hh >= 0 && hh < g.H;
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int v = tid + 256 * r;
            if (NVX % 256 == 0 || v < NVX) {
                const int j = v / (BK / 8), cv = (v % (BK / 8)) * 8;
                const int w = w0 + j - 1, c = cc + cv;
                rx[r] = zero8();
                if (hin && w >= 0 && w < g.W && c < Cin) {
                    const i64 p = ((i64)b * g.H + hh) * g.W + w;
                    if (c < C1) {
                        const bf16x8 x = ld8(X1 + p * C1 + c);
                        rx[r] = mask ? masked8(x, ld8(mask + p * C1 + c)) : x;
                    } else {
                        rx[r] = ld8(X2 + p * C2 + (c - C1));
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int v = tid + 256 * r;
            if (NVW % 256 == 0 || v < NVW) {
                rw[r] = zero8();
                if constexpr (!WT) {  // [dx][n][c]: 8 consecutive c of output channel n
                    const int dx = v / (BN * BK / 8), rem = v - dx * (BN * BK / 8);
                    const int n = rem / (BK / 8), cv = (rem % (BK / 8)) * 8;
                    const int co = n0 + n, c = cc + cv;
                    if (co < Nout && c < Cin) rw[r] = ld8(Wb + ((i64)co * 9 + 3 * dy + dx) * Cp + c);
                } else {  // [dx][c][n]: 8 consecutive n (forward input channels) of channel c
                    const int dx = v / (BN * BK / 8), rem = v - dx * (BN * BK / 8);
                    const int c = rem / (BN / 8), nv = (rem % (BN / 8)) * 8;
                    const int co = cc + c, ci = n0 + nv;
                    if (co < Cin && ci < Nout) rw[r] = ld8(Wb + ((i64)co * 9 + 8 - (3 * dy + dx)) * Cp + ci);
                }
            }
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int v = tid + 256 * r;
            if (NVX % 256 == 0 || v < NVX) {
                const int j = v / (BK / 8), cv = (v % (BK / 8)) * 8;
                *reinterpret_cast<bf16x8*>(&Xs[st][j * XC + cv]) = rx[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int v = tid + 256 * r;
            if (NVW % 256 == 0 || v < NVW) {
                const int dx = v / (BN * BK / 8), rem = v - dx * (BN * BK / 8);
                int a, e;
                if constexpr (!WT) {
                    a = rem / (BK / 8);
                    e = (rem % (BK / 8)) * 8;
                } else {
                    a = rem / (BN / 8);
                    e = (rem % (BN / 8)) * 8;
                }
                *reinterpret_cast<bf16x8*>(&Ws[st][(dx * WR + a) * WC + e]) = rw[r];
            }
        }
    };

    if (total > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    int st = 0;
    const int kg = (lane >> 4) * 8, rl = lane & 15;
    for (int k = 0; k < total; ++k) {
        const bool more = k + 1 < total;
        if (more) fetch(k + 1);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            bf16x8 a[TM], bv[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&Xs[st][(wm + 16 * i + rl + dx) * XC + kg]);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (!WT) bv[j] = *reinterpret_cast<const bf16x8*>(&Ws[st][(dx * WR + wn + 16 * j + rl) * WC + kg]);
                else bv[j] = ld_tr8(&Ws[st][dx * WR * WC + wn + 16 * j], WC, lane);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (k % nst == nst - 1) {  // the segment is complete: write it, start the next from zero
            int b, h, w0, cc, dy;
            locate(k, b, h, w0, cc, dy);
            const i64 prow = ((i64)b * g.H + h) * g.W;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int w = w0 + wm + 16 * i + (lane >> 4) * 4 + q;
                    if (w < g.W) {
#pragma unroll
                        for (int j = 0; j < TN; ++j) epi(prow + w, n0 + wn + 16 * j + (lane & 15), acc[i][j][q]);
                    }
                }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
}

// One tap-blocked convolution pass: segments of 128 pixels (64 on rows of
// 64, 32 on rows of at most 32), 64 channels per workgroup (32 when there are
// at most 32), one segment per workgroup
template <bool WT, class EPI>
void conv3x3(hipStream_t s, const bf16* X1, const bf16* X2, const bf16* mask, int C1, int C2, const bf16* Wb, int Cp,
             int Nout, const Grid& g, const EPI& e) {
    const int bm = g.W > 64 ? 128 : g.W > 32 ? 64 : 32;
    const int segs_row = (g.W + bm - 1) / bm, nsegs = g.B * g.H * segs_row;
    const bool narrow = Nout <= 32;
    const dim3 grid((unsigned)nsegs, narrow ? 1u : (unsigned)((Nout + 63) / 64));
#define LBM_CONV(tm, tn) \
    k_conv3x3<tm, tn, WT, EPI><<<grid, 256, 0, s>>>(X1, X2, mask, C1, C2, Wb, Cp, Nout, g, segs_row, nsegs, e)
    if (bm == 128) {
        if (narrow) LBM_CONV(4, 1);
        else LBM_CONV(4, 2);
    } else if (bm == 64) {
        if (narrow) LBM_CONV(2, 1);
        else LBM_CONV(2, 2);
    } else {
        if (narrow) LBM_CONV(1, 1);
        else LBM_CONV(1, 2);
    }
#undef LBM_CONV
}

// K split into z chunks (multiples of BK); returns the number of chunks launched
inline i64 kchunk_of(i64 K, int z) {
    const i64 c = ((K + z - 1) / z + BK - 1) / BK * BK;
    return c < BK ? BK : c;
}
inline int nchunks(i64 K, int z) {
    const i64 c = kchunk_of(K, z);
    const i64 n = (K + c - 1) / c;
    return (int)(n < 1 ? 1 : n);
}

template <int BM, int BN, class LA, class LB, class EPI>
void launch_gemm(hipStream_t s, const LA& A, const LB& B, const EPI& e, i64 M, i64 N, i64 K, int z) {
    dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)nchunks(K, z));
    k_gemm<BM, BN, LA, LB, EPI><<<grid, 256, 0, s>>>(A, B, e, M, N, K, kchunk_of(K, z));
}

// A GEMM without split-K: 128-row tiles when they give at least 1024
// workgroups, 64-row tiles otherwise; 32 columns when N <= 32, else 64
template <class LA, class LB, class EPI>
void gemm(hipStream_t s, const LA& A, const LB& B, const EPI& e, i64 M, i64 N, i64 K) {
    const bool narrow = N <= 32;
    const i64 big = ((M + 127) / 128) * ((N + (narrow ? 31 : 63)) / (narrow ? 32 : 64));
    if (narrow) {
        if (big >= 1024) launch_gemm<128, 32>(s, A, B, e, M, N, K, 1);
        else launch_gemm<64, 32>(s, A, B, e, M, N, K, 1);
    } else {
        if (big >= 1024) launch_gemm<128, 64>(s, A, B, e, M, N, K, 1);
        else launch_gemm<64, 64>(s, A, B, e, M, N, K, 1);
    }
}

// K splits for a weight gradient: about 1024 workgroups, at least 2048 pixels
// per chunk, and no more partials than the buffer holds
int splits_for(i64 M, i64 N, i64 K, i64 cap_elems) {
    const i64 tiles = ((M + 63) / 64) * ((N + 63) / 64);
    i64 z = (1024 + tiles - 1) / tiles;
    z = std::min<i64>(z, std::max<i64>(1, K / 2048));
    while (z > 1 && (i64)nchunks(K, (int)z) * M * N > cap_elems) --z;
    return (int)std::max<i64>(1, z);
}

// ---------------------------------------------------------------------------
// Reductions, elementwise layers, loss and optimiser
// ---------------------------------------------------------------------------
inline int blocks_for(i64 n) {
    const i64 b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}


#define GRID_STRIDE(i, n) \
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (i64)gridDim.x * blockDim.x)

// Sum over k of P[k][i] for the OUT outputs i = base + (thread % OUT) of a
// workgroup: its 256 / OUT slices of threads add interleaved parts of k,
// combined in slice order (deterministic); valid in the first OUT threads.
// OUT = 16 when there are many partials (more workgroups, more loads in
// flight), 64 otherwise.
template <int OUT>
__device__ __forceinline__ float zsum(const float* __restrict__ P, int z, i64 MN, i64 idx, float* red) {
    constexpr int NS = 256 / OUT;
    const int o = threadIdx.x % OUT, sl = threadIdx.x / OUT;
    float s = 0.f;
    if (idx < MN) {
#pragma unroll 4
        for (int k = sl; k < z; k += NS) s += P[(i64)k * MN + idx];
    }
    red[sl * OUT + o] = s;
    __syncthreads();
    float t = 0.f;
    if (sl == 0)
        for (int k = 0; k < NS; ++k) t += red[k * OUT + o];
    __syncthreads();
    return t;
}

// split-K partials of a convolution's weight gradient, [z][Co][9 Cp + 1], summed
// into gw [Co][9][Ci] (channels >= Ci are padding) and gb [Co]
template <int OUT>
__global__ void __launch_bounds__(256) k_reduce_conv(const float* __restrict__ P, int z, int Co, int Cp, int Ci,
                                                     float* __restrict__ gw, float* __restrict__ gb) {
    __shared__ float red[256];
    const i64 N1 = 9LL * Cp + 1, MN = (i64)Co * N1;
    for (i64 base = (i64)blockIdx.x * OUT; base < MN; base += (i64)gridDim.x * OUT) {
        const i64 idx = base + (threadIdx.x % OUT);
        const float s = zsum<OUT>(P, z, MN, idx, red);
        if (threadIdx.x < OUT && idx < MN) {
            const i64 co = idx / N1, n = idx - co * N1;
            if (n == 9LL * Cp) {
                gb[co] = s;
            } else {
                const i64 t = n / Cp, c = n - t * Cp;
                if (c < Ci) gw[(co * 9 + t) * Ci + c] = s;
            }
        }
    }
}

// partials of a transposed convolution's weight gradient, [z][4 Co][Ci + 1]:
// the weight columns into gw [4 Co][Ci]; the ones column into T [4 Co]
template <int OUT>
__global__ void __launch_bounds__(256) k_reduce_up(const float* __restrict__ P, int z, int Co, int Ci,
                                                   float* __restrict__ gw, float* __restrict__ T) {
    __shared__ float red[256];
    const i64 N1 = Ci + 1, MN = 4LL * Co * N1;
    for (i64 base = (i64)blockIdx.x * OUT; base < MN; base += (i64)gridDim.x * OUT) {
        const i64 idx = base + (threadIdx.x % OUT);
        const float s = zsum<OUT>(P, z, MN, idx, red);
        if (threadIdx.x < OUT && idx < MN) {
            const i64 r = idx / N1, c = idx - r * N1;
            if (c < Ci) gw[r * Ci + c] = s;
            else T[r] = s;
        }
    }
}

inline int reduce_blocks(i64 outputs, int per) {  // per outputs per workgroup
    const i64 b = (outputs + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// transposed-convolution bias gradient: the four offsets of each channel, in order
__global__ void k_up_bias(const float* __restrict__ T, int Co, float* __restrict__ gb) {
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co < Co) gb[co] = ((T[co] + T[Co + co]) + T[2 * Co + co]) + T[3 * Co + co];
}

// 2x2 max pooling (NHWC), with the position (0..3) of the first maximum kept
__global__ void k_pool_fwd(const bf16* __restrict__ X, bf16* __restrict__ Y, uint8_t* __restrict__ arg, Grid g, int C) {
    const uint32_t Ho = g.H / 2, Wo = g.W / 2, uC = C;
    const i64 n = (i64)g.B * Ho * Wo * C;
    GRID_STRIDE(i, n) {
        const uint32_t ii = (uint32_t)i, q = ii / uC, c = ii - q * uC, q2 = q / Wo;
        const int w = (int)(q - q2 * Wo), h = (int)(q2 % Ho), b = (int)(q2 / Ho);
        float best = -INFINITY;
        int bi = 0;
        for (int a = 0; a < 4; ++a) {
            const i64 p = ((i64)b * g.H + 2 * h + (a >> 1)) * g.W + 2 * w + (a & 1);
            const float v = (float)X[p * C + c];
            if (v > best) {
                best = v;
                bi = a;
            }
        }
        Y[i] = (bf16)best;
        arg[i] = (uint8_t)bi;
    }
}

// dX += dY at the position of each window's maximum (dX already holds the
// gradient that reaches the pooled tensor's input through the skip connection)
__global__ void k_pool_bwd(const bf16* __restrict__ dY, const uint8_t* __restrict__ arg, bf16* __restrict__ dX, Grid g,
                           int C) {
    const uint32_t Ho = g.H / 2, Wo = g.W / 2, uC = C;
    const i64 n = (i64)g.B * Ho * Wo * C;
    GRID_STRIDE(i, n) {
        const uint32_t ii = (uint32_t)i, q = ii / uC, c = ii - q * uC, q2 = q / Wo;
        const int w = (int)(q - q2 * Wo), h = (int)(q2 % Ho), b = (int)(q2 / Ho);
        const int a = arg[i];
        const i64 p = ((i64)b * g.H + 2 * h + (a >> 1)) * g.W + 2 * w + (a & 1);
        dX[p * C + c] = (bf16)((float)dX[p * C + c] + (float)dY[i]);
    }
}

// 1x1 head to one FP32 channel (C a multiple of 8)
__global__ void k_head_fwd(const bf16* __restrict__ X, const float* __restrict__ w, const float* __restrict__ b,
                           float* __restrict__ y, i64 P, int C) {
    GRID_STRIDE(p, P) {
        float s = b[0];
        for (int c = 0; c < C; c += 8) {
            const bf16x8 v = ld8(X + p * C + c);
#pragma unroll
            for (int j = 0; j < 8; ++j) s += (float)v[j] * w[c + j];
        }
        y[p] = s;
    }
}

__global__ void k_head_bwd_x(const float* __restrict__ dy, const float* __restrict__ w, bf16* __restrict__ dX, i64 P,
                             int C) {
    GRID_STRIDE(i, P * C) {
        const uint32_t ii = (uint32_t)i, p = ii / (uint32_t)C;
        dX[i] = (bf16)(dy[p] * w[ii - p * (uint32_t)C]);
    }
}

// head weight and bias gradients: per-block partials [blk][C + 1] (C a multiple
// of 8 dividing 256).  A thread takes 8 channels (one 16-byte vector) of
// every (256 / (C / 8))-th pixel of the block's range; the pixel lanes are
// summed in LDS in lane order (deterministic).
__global__ void __launch_bounds__(256) k_head_bwd_w(const float* __restrict__ dy, const bf16* __restrict__ X, i64 P,
                                                    int C, float* __restrict__ part) {
    __shared__ float red[256 * 8];
    __shared__ float redb[256];
    const int nv = C / 8, cv = (int)threadIdx.x % nv, lane = (int)threadIdx.x / nv, nl = 256 / nv;
    const i64 per = (P + gridDim.x - 1) / gridDim.x;
    const i64 beg = (i64)blockIdx.x * per, end = std::min<i64>(P, beg + per);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, sb = 0.f;
#pragma unroll 4
    for (i64 p = beg + lane; p < end; p += nl) {
        const float d = dy[p];
        const bf16x8 x = ld8(X + p * C + 8 * cv);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += d * (float)x[j];
        sb += d;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) red[lane * C + 8 * cv + j] = s[j];
    redb[threadIdx.x] = sb;
    __syncthreads();
    if ((int)threadIdx.x < C) {
        float t = 0.f;
        for (int k = 0; k < nl; ++k) t += red[k * C + threadIdx.x];
        part[(i64)blockIdx.x * (C + 1) + threadIdx.x] = t;
    }
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < nl; ++k) t += redb[k * nv];   // the cv = 0 thread of each lane
        part[(i64)blockIdx.x * (C + 1) + C] = t;
    }
}

// sums of the head partials: one workgroup per channel (and one for the bias), fixed-order tree
__global__ void __launch_bounds__(256) k_head_reduce(const float* __restrict__ part, int nblk, int C,
                                                     float* __restrict__ gw, float* __restrict__ gb) {
    __shared__ float red[256];
    const int c = blockIdx.x;  // 0..C
    float s = 0.f;
    for (int k = threadIdx.x; k < nblk; k += 256) s += part[(i64)k * (C + 1) + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < C) gw[c] = red[0];
        else gb[0] = red[0];
    }
}

// mean squared error: dL/dy and per-block FP64 partial sums
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t, i64 n,
                                             float* __restrict__ dy, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    GRID_STRIDE(i, n) {
        const float e = y[i] - t[i];
        s += (double)e * e;
        dy[i] = 2.f * e / (float)n;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_parts(const double* __restrict__ part, int n, double scale,
                                                   double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam with bias correction (c1 = 1 - beta1^t, c2 = 1 - beta2^t)
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       i64 n, float lr, float b1, float b2, float eps, float c1, float c2) {
    GRID_STRIDE(i, n) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// FP32 [rows][Ci] -> BF16 [rows][Cp], zero in the padding channels
__global__ void k_cast_pad(const float* __restrict__ x, bf16* __restrict__ y, i64 rows, int Ci, int Cp) {
    GRID_STRIDE(i, rows * Cp) {
        const i64 r = i / Cp;
        const int c = (int)(i - r * Cp);
        y[i] = (bf16)(c < Ci ? x[r * Ci + c] : 0.f);
    }
}

// one FP32 -> BF16 weight copy of the batched cast below: rows x Ci into rows x Cp,
// elements [start, start + rows Cp) of the concatenated index space
struct CastJob {
    const float* x;
    bf16* y;
    i64 rows, start;
    int Ci, Cp;
};

// every BF16 weight copy in one launch (after each Adam step): element i of the
// concatenated index space belongs to the last job that starts at or before it
__global__ void k_cast_pad_all(const CastJob* __restrict__ jobs, int njobs, i64 total) {
    GRID_STRIDE(i, total) {
        int j = 0;
        while (j + 1 < njobs && jobs[j + 1].start <= i) ++j;
        const CastJob J = jobs[j];
        const i64 k = i - J.start, r = k / J.Cp;
        const int c = (int)(k - r * J.Cp);
        J.y[k] = (bf16)(c < J.Ci ? J.x[r * J.Ci + c] : 0.f);
    }
}

__global__ void k_fill_f32(float* __restrict__ p, i64 n, float v) {
    GRID_STRIDE(i, n) { p[i] = v; }
}

// ---------------------------------------------------------------------------
// Lattice <-> network fields
// ---------------------------------------------------------------------------
constexpr uint8_t SOLID_BITS = 3;  // low two class bits: 0 fluid, 1..3 solid layers

// x[i] = {solid, solid ? solid_value : 0, plane[, phi0[i]]} (3 or 4 channels)
__global__ void k_encode(const uint8_t* __restrict__ cls, const float* __restrict__ phi0, i64 n, float solid_value,
                         float plane, float* __restrict__ x) {
    const int C = phi0 ? 4 : 3;
    GRID_STRIDE(i, n) {
        const bool s = (cls[i] & SOLID_BITS) != 0;
        x[C * i + 0] = s ? 1.f : 0.f;
        x[C * i + 1] = s ? solid_value : 0.f;
        x[C * i + 2] = plane;
        if (phi0) x[C * i + 3] = phi0[i];
    }
}

template <typename R>
__global__ void k_target(const R* __restrict__ rho, const uint8_t* __restrict__ cls, i64 n, double rho_g, double rho_l,
                         float* __restrict__ phi) {
    GRID_STRIDE(i, n) {
        phi[i] = (cls[i] & SOLID_BITS) ? 0.f : (float)(((double)rho[i] - rho_g) / (rho_l - rho_g));
    }
}

// Mean of phi over the fluid nodes of the (2 r + 1)^2 window around each fluid
// node (periodic images; solid nodes neither contribute nor receive: 0), in
// a fixed order.  Removes the sub-interface-width artefacts a prediction can
// carry, whose one-node jumps the fourth-order force would turn into a blow-up.
__global__ void k_smooth_fluid(const float* __restrict__ phi, const uint8_t* __restrict__ cls, int nx, int ny, int r,
                               float* __restrict__ out) {
    GRID_STRIDE(i, (i64)nx * ny) {
        if (cls[i] & SOLID_BITS) {
            out[i] = 0.f;
            continue;
        }
        const int x = (int)(i % nx), y = (int)(i / nx);
        float num = 0.f, den = 0.f;
        for (int dy = -r; dy <= r; ++dy) {
            int yy = (y + dy) % ny;
            if (yy < 0) yy += ny;
            for (int dx = -r; dx <= r; ++dx) {
                int xx = (x + dx) % nx;
                if (xx < 0) xx += nx;
                const i64 j = (i64)yy * nx + xx;
                if (!(cls[j] & SOLID_BITS)) {
                    num += phi[j];
                    den += 1.f;
                }
            }
        }
        out[i] = num / den;
    }
}

// One workgroup: the mass-exact density from a predicted phi.  Fluid nodes get
// rho = rho_g + (rho_l - rho_g) s clamp((phi + delta - cut) / (1 - 2 cut), 0, 1)
// with delta found by bisection so that the fluid mass equals that of
// rho_ref, and s (close to 1) removing what the bisection leaves; solid nodes
// get 0.  out = {mass of rho_ref, mass written, delta, s, fluid nodes}.
template <typename R>
__global__ void __launch_bounds__(1024) k_warm_rho(const float* __restrict__ phi, const R* __restrict__ rho_ref,
                                                   const uint8_t* __restrict__ cls, i64 n, double rho_g, double rho_l,
                                                   double cut, R* __restrict__ rho, double* __restrict__ out) {
    __shared__ double red[1024];
    const int t = threadIdx.x;
    auto block_sum = [&](double v) {
        red[t] = v;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        const double s = red[0];
        __syncthreads();
        return s;
    };
    const double span = 1.0 - 2.0 * cut;
    auto clamped = [&](i64 i, double d) { return fmin(1.0, fmax(0.0, ((double)phi[i] + d - cut) / span)); };
    double m = 0.0, nf = 0.0;
    for (i64 i = t; i < n; i += 1024)
        if (!(cls[i] & SOLID_BITS)) {
            m += (double)rho_ref[i];
            nf += 1.0;
        }
    const double mass = block_sum(m), nfl = block_sum(nf);
    const double target = (mass - nfl * rho_g) / (rho_l - rho_g);  // wanted sum of clamp(phi + delta, 0, 1)
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        double s = 0.0;
        for (i64 i = t; i < n; i += 1024)
            if (!(cls[i] & SOLID_BITS)) s += clamped(i, mid);
        if (block_sum(s) < target) lo = mid;
        else hi = mid;
    }
    const double delta = 0.5 * (lo + hi);
    double s = 0.0;
    for (i64 i = t; i < n; i += 1024)
        if (!(cls[i] & SOLID_BITS)) s += clamped(i, delta);
    const double got = block_sum(s);
    const double scale = got > 0.0 ? target / got : 1.0;
    double mw = 0.0;
    for (i64 i = t; i < n; i += 1024) {
        R r = R(0);
        if (!(cls[i] & SOLID_BITS)) {
            r = (R)(rho_g + (rho_l - rho_g) * scale * clamped(i, delta));
            mw += (double)r;
        }
        rho[i] = r;
    }
    const double written = block_sum(mw);
    if (t == 0) {
        out[0] = mass;
        out[1] = written;
        out[2] = delta;
        out[3] = scale;
        out[4] = nfl;
    }
}

// ---------------------------------------------------------------------------
// Network state
// ---------------------------------------------------------------------------
struct Param {
    i64 n = 0, off = 0;
};

struct Conv {  // 3x3 conv + ReLU over [Ci1 | Ci2] input channels
    int Ci1, Ci2, Co;
    int Cp;  // input channels of the BF16 weight copy (Ci1 + Ci2, or the padded network input)
    Param w, b;
    bf16* wb = nullptr;  // BF16 [Co][9][Cp]
};

struct Up {  // 2x2 stride-2 transposed convolution, weights [4 Co][Ci]
    int Ci, Co;
    Param w, b;
    bf16* wb = nullptr;
};

struct Act {  // an activation and its gradient, BF16 NHWC
    bf16* x = nullptr;
    bf16* d = nullptr;
};

}  // namespace

struct lbm_unet {
    lbm_unet_config cfg{};
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int H = 0, W = 0, B = 0, L = 0, C0 = 0, Cin = 0, Cinp = 0;
    int nb = 0;  // samples in the current call
    std::vector<Conv> enc, dec;
    std::vector<Up> up;
    Param hw, hb;
    i64 nparam = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    std::vector<Act> c1, c2, pool, upo, d1, d2;
    std::vector<uint8_t*> arg;
    bf16* x0 = nullptr;  // BF16 input, channels padded
    float *y = nullptr, *dy = nullptr;
    float* part = nullptr;
    i64 part_n = 0;
    float* hpart = nullptr;
    float* upb = nullptr;   // transposed-convolution bias partials [4 Co]
    float* sphi = nullptr;  // smoothed phi of lbm_unet_warm_rho [H W]
    double *lpart = nullptr, *loss = nullptr, *winfo = nullptr;
    CastJob* casts = nullptr;  // the BF16 weight copies, one launch (built on first use)
    int ncasts = 0;
    i64 cast_total = 0;
    i64 step = 0;
    // lbm_unet_train_step's forward and backward passes, captured as two
    // graphs for graph_nb samples (the input cast, the loss and the Adam step,
    // which read the caller's pointers or the step count, stay eager);
    // LBM_UNET_GRAPHS=0 keeps every launch eager
    bool use_graphs = true;
    int graph_nb = 0;
    hipGraphExec_t gfwd = nullptr, gbwd = nullptr;
};

namespace {

constexpr int HEAD_BLOCKS = 2048;
constexpr int MSE_BLOCKS = 1024;

lbm_status ufail(lbm_unet* u, lbm_status s, const std::string& msg) {
    if (u) u->err = msg;
    return s;
}

#define UCHK(u, call)                                                                                           \
    do {                                                                                                        \
        hipError_t e_ = (call);                                                                                 \
        if (e_ != hipSuccess) return ufail(u, LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Grid grid_of(const lbm_unet* u, int l) { return make_grid(u->nb, u->H >> l, u->W >> l); }
i64 pixels(const lbm_unet* u, int l) { return (i64)u->nb * (u->H >> l) * (u->W >> l); }

void refresh_bf16(lbm_unet* u) {
    if (!u->casts) {
        std::vector<CastJob> jobs;
        i64 start = 0;
        auto add = [&](const float* x, bf16* y, i64 rows, int Ci, int Cp) {
            jobs.push_back(CastJob{x, y, rows, start, Ci, Cp});
            start += rows * Cp;
        };
        for (auto* layers : {&u->enc, &u->dec})
            for (auto& c : *layers) add(u->w + c.w.off, c.wb, (i64)c.Co * 9, c.Ci1 + c.Ci2, c.Cp);
        for (auto& p : u->up) add(u->w + p.w.off, p.wb, 4LL * p.Co, p.Ci, p.Ci);
        if (hipMalloc((void**)&u->casts, jobs.size() * sizeof(CastJob)) == hipSuccess &&
            hipMemcpy(u->casts, jobs.data(), jobs.size() * sizeof(CastJob), hipMemcpyHostToDevice) == hipSuccess) {
            u->ncasts = (int)jobs.size();
            u->cast_total = start;
        } else {
            if (u->casts) (void)hipFree(u->casts);
            u->casts = nullptr;
            (void)hipGetLastError();
        }
    }
    if (u->casts) {
        k_cast_pad_all<<<blocks_for(u->cast_total), 256, 0, u->stream>>>(u->casts, u->ncasts, u->cast_total);
        return;
    }
    // one launch per layer if the job table could not be allocated
    for (auto* layers : {&u->enc, &u->dec})
        for (auto& c : *layers) {
            const i64 rows = (i64)c.Co * 9;
            k_cast_pad<<<blocks_for(rows * c.Cp), 256, 0, u->stream>>>(u->w + c.w.off, c.wb, rows, c.Ci1 + c.Ci2, c.Cp);
        }
    for (auto& p : u->up)
        k_cast_pad<<<blocks_for(4LL * p.Co * p.Ci), 256, 0, u->stream>>>(u->w + p.w.off, p.wb, 4LL * p.Co, p.Ci, p.Ci);
}

// y = relu(conv3x3([x1 | x2]) + b); x1 holds C1 channels (Cp - Ci2 of them)
void conv_fwd(lbm_unet* u, const Conv& c, const bf16* x1, const bf16* x2, bf16* y, int l) {
    const i64 P = pixels(u, l);
    EpiBiasRelu e{y, u->w + c.b.off, P, c.Co};
    conv3x3<false>(u->stream, x1, x2, nullptr, c.Cp - c.Ci2, c.Ci2, c.wb, c.Cp, c.Co, grid_of(u, l), e);
}

// split-K partials of a convolution's weight and bias gradients into u->part
// ([z][Co][9 Cp + 1]); returns z.  Tiles of 32 output by 64 input channels
// (four waves per group, three groups) or, for at most 32 input channels, 32
// by 32 (two waves per group, six groups): 12 waves per workgroup; about 256
// workgroups (one per compute unit) and at least two segments per group, so
// that the partials stay small.
int wgrad3x3(lbm_unet* u, const Conv& c, const bf16* x1, const bf16* x2, const bf16* y, const bf16* dy, const Grid& g) {
    const bool wide = c.Cp > 32;
    const int BN = wide ? 64 : 32, G = wide ? 3 : 6;
    const int segs_row = (g.W + SEG - 1) / SEG, nsegs = g.B * g.H * segs_row;
    const int tiles = ((c.Co + 31) / 32) * ((c.Cp + BN - 1) / BN);
    const i64 N1 = 9LL * c.Cp + 1;
    int z = std::max(1, std::min((256 + tiles - 1) / tiles, nsegs / (2 * G)));
    z = (int)std::min<i64>(z, std::max<i64>(1, u->part_n / ((i64)c.Co * N1)));
    const int spc = (nsegs + z - 1) / z;
    z = (nsegs + spc - 1) / spc;  // every chunk holds at least one segment
    const dim3 grid((unsigned)((c.Co + 31) / 32), (unsigned)((c.Cp + BN - 1) / BN), (unsigned)z);
    if (wide)
        k_wgrad3x3<2, 1, 4, 3><<<grid, 768, 0, u->stream>>>(dy, y, x1, x2, c.Cp - c.Ci2, c.Ci2, c.Co, g, segs_row,
                                                            nsegs, spc, u->part);
    else
        k_wgrad3x3<2, 1, 2, 6><<<grid, 768, 0, u->stream>>>(dy, y, x1, x2, c.Cp - c.Ci2, c.Ci2, c.Co, g, segs_row,
                                                            nsegs, spc, u->part);
    return z;
}

// backward of y = relu(conv3x3([x1 | x2]) + b): weight and bias gradients into
// g; data gradients written to dx1 / dx2 when dx1 is set
void conv_bwd(lbm_unet* u, const Conv& c, const bf16* x1, const bf16* x2, const bf16* y, const bf16* dy, bf16* dx1,
              bf16* dx2, int l) {
    const i64 P = pixels(u, l);
    const Grid g = grid_of(u, l);
    if (dx1) {
        EpiSplit e{dx1, dx2, P, c.Ci1, c.Ci2};
        conv3x3<true>(u->stream, dy, nullptr, y, c.Co, 0, c.wb, c.Cp, c.Ci1 + c.Ci2, g, e);
    }
    const i64 N1 = 9LL * c.Cp + 1;
    const int nz = wgrad3x3(u, c, x1, x2, y, dy, g);
    if (nz >= 32)
        k_reduce_conv<16><<<reduce_blocks((i64)c.Co * N1, 16), 256, 0, u->stream>>>(u->part, nz, c.Co, c.Cp,
                                                                                     c.Ci1 + c.Ci2, u->g + c.w.off,
                                                                                     u->g + c.b.off);
    else
        k_reduce_conv<64><<<reduce_blocks((i64)c.Co * N1, 64), 256, 0, u->stream>>>(u->part, nz, c.Co, c.Cp,
                                                                                     c.Ci1 + c.Ci2, u->g + c.w.off,
                                                                                     u->g + c.b.off);
}

void up_fwd(lbm_unet* u, const Up& p, const bf16* x, bf16* y, int lin) {
    const i64 P = pixels(u, lin);
    RowsKA A{x, p.Ci};
    RowsK B{p.wb, p.Ci};
    EpiUp e{y, u->w + p.b.off, UpMap{grid_of(u, lin)}, P, p.Co, fastdiv((uint32_t)p.Co)};
    gemm(u->stream, A, B, e, P, 4LL * p.Co, p.Ci);
}

void up_bwd(lbm_unet* u, const Up& p, const bf16* x, const bf16* dy, bf16* dx, int lin) {
    const i64 P = pixels(u, lin);
    const UpMap um{grid_of(u, lin)};
    UpGatherK A{dy, um, p.Co, fastdiv((uint32_t)p.Co)};
    RowsN B{p.wb, p.Ci};
    EpiSplit e{dx, nullptr, P, p.Ci, 0};
    gemm(u->stream, A, B, e, P, p.Ci, 4LL * p.Co);
    const i64 N1 = p.Ci + 1;
    UpGatherM A2{dy, um, p.Co, fastdiv((uint32_t)p.Co)};
    ColsOnes B2{x, p.Ci};
    const int z = splits_for(4LL * p.Co, N1, P, u->part_n);
    EpiPartial e2{u->part, 4LL * p.Co, N1};
    launch_gemm<64, 64>(u->stream, A2, B2, e2, 4LL * p.Co, N1, P, z);
    const int nz = nchunks(P, z);
    if (nz >= 32)
        k_reduce_up<16><<<reduce_blocks(4LL * p.Co * N1, 16), 256, 0, u->stream>>>(u->part, nz, p.Co, p.Ci,
                                                                                   u->g + p.w.off, u->upb);
    else
        k_reduce_up<64><<<reduce_blocks(4LL * p.Co * N1, 64), 256, 0, u->stream>>>(u->part, nz, p.Co, p.Ci,
                                                                                   u->g + p.w.off, u->upb);
    k_up_bias<<<(p.Co + 255) / 256, 256, 0, u->stream>>>(u->upb, p.Co, u->g + p.b.off);
}

void forward(lbm_unet* u) {
    const int L = u->L;
    const bf16* in = u->x0;
    for (int l = 0; l < L; ++l) {
        conv_fwd(u, u->enc[2 * l], in, nullptr, u->c1[l].x, l);
        conv_fwd(u, u->enc[2 * l + 1], u->c1[l].x, nullptr, u->c2[l].x, l);
        if (l < L - 1) {
            const int C = u->enc[2 * l].Co;
            const i64 n = pixels(u, l + 1) * C;
            k_pool_fwd<<<blocks_for(n), 256, 0, u->stream>>>(u->c2[l].x, u->pool[l].x, u->arg[l], grid_of(u, l), C);
            in = u->pool[l].x;
        }
    }
    const bf16* x = u->c2[L - 1].x;
    for (int j = 0; j < L - 1; ++j) {
        const int l = L - 2 - j;  // output level
        up_fwd(u, u->up[j], x, u->upo[j].x, l + 1);
        conv_fwd(u, u->dec[2 * j], u->upo[j].x, u->c2[l].x, u->d1[j].x, l);
        conv_fwd(u, u->dec[2 * j + 1], u->d1[j].x, nullptr, u->d2[j].x, l);
        x = u->d2[j].x;
    }
    const i64 P0 = pixels(u, 0);
    k_head_fwd<<<blocks_for(P0), 256, 0, u->stream>>>(x, u->w + u->hw.off, u->w + u->hb.off, u->y, P0, u->C0);
}

void backward(lbm_unet* u) {
    const int L = u->L;
    const i64 P0 = pixels(u, 0);
    const Act& last = L > 1 ? u->d2[L - 2] : u->c2[0];
    k_head_bwd_x<<<blocks_for(P0 * u->C0), 256, 0, u->stream>>>(u->dy, u->w + u->hw.off, last.d, P0, u->C0);
    k_head_bwd_w<<<HEAD_BLOCKS, 256, 0, u->stream>>>(u->dy, last.x, P0, u->C0, u->hpart);
    k_head_reduce<<<u->C0 + 1, 256, 0, u->stream>>>(u->hpart, HEAD_BLOCKS, u->C0, u->g + u->hw.off, u->g + u->hb.off);
    for (int j = L - 2; j >= 0; --j) {
        const int l = L - 2 - j;
        const Conv& a = u->dec[2 * j];
        const Conv& b = u->dec[2 * j + 1];
        conv_bwd(u, b, u->d1[j].x, nullptr, u->d2[j].x, u->d2[j].d, u->d1[j].d, nullptr, l);
        // the first decoder convolution reads [up | skip]: its data gradient
        // splits into d(up) and the skip part of d(c2) (written here, added to below)
        conv_bwd(u, a, u->upo[j].x, u->c2[l].x, u->d1[j].x, u->d1[j].d, u->upo[j].d, u->c2[l].d, l);
        const Act& xin = j == 0 ? u->c2[L - 1] : u->d2[j - 1];
        up_bwd(u, u->up[j], xin.x, u->upo[j].d, xin.d, l + 1);
    }
    for (int l = L - 1; l >= 0; --l) {
        const Conv& a = u->enc[2 * l];
        const Conv& b = u->enc[2 * l + 1];
        if (l < L - 1) {
            const i64 n = pixels(u, l + 1) * a.Co;
            k_pool_bwd<<<blocks_for(n), 256, 0, u->stream>>>(u->pool[l].d, u->arg[l], u->c2[l].d, grid_of(u, l), a.Co);
        }
        conv_bwd(u, b, u->c1[l].x, nullptr, u->c2[l].x, u->c2[l].d, u->c1[l].d, nullptr, l);
        const bf16* xin = l == 0 ? u->x0 : u->pool[l - 1].x;
        conv_bwd(u, a, xin, nullptr, u->c1[l].x, u->c1[l].d, l == 0 ? nullptr : u->pool[l - 1].d, nullptr, l);
    }
}

lbm_status load_input(lbm_unet* u, const float* x, int n) {
    if (n < 1 || n > u->B) return ufail(u, LBM_E_ARG, "sample count must be in 1..batch");
    u->nb = n;
    const i64 P = pixels(u, 0);
    k_cast_pad<<<blocks_for(P * u->Cinp), 256, 0, u->stream>>>(x, u->x0, P, u->Cin, u->Cinp);
    return LBM_OK;
}

void drop_graphs(lbm_unet* u) {
    for (hipGraphExec_t* g : {&u->gfwd, &u->gbwd})
        if (*g) {
            (void)hipGraphExecDestroy(*g);
            *g = nullptr;
        }
    u->graph_nb = 0;
}

// the launches of fn(u) on u's stream as an executable graph
lbm_status capture(lbm_unet* u, void (*fn)(lbm_unet*), hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    UCHK(u, hipStreamBeginCapture(u->stream, hipStreamCaptureModeThreadLocal));
    fn(u);
    const hipError_t e = hipStreamEndCapture(u->stream, &g);
    if (e != hipSuccess) return ufail(u, LBM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        *out = nullptr;
        return ufail(u, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    return LBM_OK;
}

lbm_status fwd_bwd(lbm_unet* u, const float* x, const float* t, int n, double* loss) {
    lbm_status s = load_input(u, x, n);
    if (s) return s;
    forward(u);
    const i64 np = pixels(u, 0);
    k_mse<<<MSE_BLOCKS, 256, 0, u->stream>>>(u->y, t, np, u->dy, u->lpart);
    k_sum_parts<<<1, 256, 0, u->stream>>>(u->lpart, MSE_BLOCKS, 1.0 / (double)np, u->loss);
    backward(u);
    UCHK(u, hipGetLastError());
    if (loss) UCHK(u, hipMemcpyAsync(loss, u->loss, 8, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_unet_last_error(const lbm_unet* u) { return u ? u->err.c_str() : "null network"; }

void lbm_unet_config_default(lbm_unet_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->H = 256;
    c->W = 256;
    c->batch = 8;
    c->in_channels = 3;
    c->base_channels = 32;
    c->levels = 4;
    c->lr = 1e-3;
    c->beta1 = 0.9;
    c->beta2 = 0.999;
    c->eps = 1e-8;
    c->stream = nullptr;
}

lbm_status lbm_unet_destroy(lbm_unet* u) {
    if (!u) return LBM_OK;
    if (u->stream) (void)hipStreamSynchronize(u->stream);
    drop_graphs(u);
    auto fr = [](void* p) {
        if (p) (void)hipFree(p);
    };
    for (auto* layers : {&u->enc, &u->dec})
        for (auto& c : *layers) fr(c.wb);
    for (auto& p : u->up) fr(p.wb);
    for (auto* acts : {&u->c1, &u->c2, &u->pool, &u->upo, &u->d1, &u->d2})
        for (auto& a : *acts) {
            fr(a.x);
            fr(a.d);
        }
    for (auto p : u->arg) fr(p);
    for (void* p : {(void*)u->w, (void*)u->g, (void*)u->m, (void*)u->v, (void*)u->x0, (void*)u->y, (void*)u->dy,
                    (void*)u->part, (void*)u->hpart, (void*)u->upb, (void*)u->lpart, (void*)u->loss, (void*)u->winfo, (void*)u->sphi,
                    (void*)u->casts})
        fr(p);
    if (u->own_stream && u->stream) (void)hipStreamDestroy(u->stream);
    delete u;
    return LBM_OK;
}

lbm_status lbm_unet_create(const lbm_unet_config* cfg, lbm_unet** out) {
    if (!out || !cfg) return LBM_E_ARG;
    *out = nullptr;
    const int L = cfg->levels, C0 = cfg->base_channels;
    if (L < 1 || L > 6 || C0 < 8 || C0 > 128 || C0 % 8 || 256 % C0 || cfg->batch < 1 || cfg->in_channels < 1 ||
        cfg->in_channels > CPAD || cfg->H < 1 || cfg->W < 1 || cfg->H % (1 << (L - 1)) || cfg->W % (1 << (L - 1)) ||
        !(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) ||
        !(cfg->eps > 0))
        return LBM_E_ARG;
    // GEMM row indices (pixels) and element offsets within one activation stay below 2^31
    if ((i64)cfg->batch * cfg->H * cfg->W * (C0 << 1) >= (1LL << 31)) return LBM_E_ARG;
    lbm_unet* u = new (std::nothrow) lbm_unet();
    if (!u) return LBM_E_NOMEM;
    u->cfg = *cfg;
    {
        const char* e = std::getenv("LBM_UNET_GRAPHS");
        u->use_graphs = !(e && std::atoi(e) == 0);
    }
    u->H = cfg->H;
    u->W = cfg->W;
    u->B = cfg->batch;
    u->L = L;
    u->C0 = C0;
    u->Cin = cfg->in_channels;
    u->Cinp = CPAD;
    if (cfg->stream) {
        u->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&u->stream, hipStreamNonBlocking) != hipSuccess) {
            delete u;
            return LBM_E_DEVICE;
        }
        u->own_stream = true;
    }
    // parameters in the order lbm.h documents for lbm_unet_get_params
    i64 off = 0;
    auto param = [&](i64 n) {
        Param p;
        p.n = n;
        p.off = off;
        off += n;
        return p;
    };
    int ci = u->Cin, cip = u->Cinp;
    for (int l = 0; l < L; ++l) {
        const int co = C0 << l;
        for (int k = 0; k < 2; ++k) {
            Conv c;
            c.Ci1 = k == 0 ? ci : co;
            c.Ci2 = 0;
            c.Co = co;
            c.Cp = k == 0 ? cip : co;
            c.w = param((i64)co * 9 * c.Ci1);
            c.b = param(co);
            u->enc.push_back(c);
        }
        ci = cip = co;
    }
    for (int l = L - 2; l >= 0; --l) {
        const int co = C0 << l;
        Up p;
        p.Ci = 2 * co;
        p.Co = co;
        p.w = param(4LL * co * p.Ci);
        p.b = param(co);
        u->up.push_back(p);
        for (int k = 0; k < 2; ++k) {
            Conv c;
            c.Ci1 = co;
            c.Ci2 = k == 0 ? co : 0;
            c.Co = co;
            c.Cp = c.Ci1 + c.Ci2;
            c.w = param((i64)co * 9 * c.Cp);
            c.b = param(co);
            u->dec.push_back(c);
        }
    }
    u->hw = param(C0);
    u->hb = param(1);
    u->nparam = off;

    bool ok = true;
    auto dalloc = [&](void** p, i64 bytes) {
        ok = ok && hipMalloc(p, (size_t)std::max<i64>(bytes, 16)) == hipSuccess;
    };
    const i64 P0 = (i64)u->B * u->H * u->W;
    dalloc((void**)&u->w, off * 4);
    dalloc((void**)&u->g, off * 4);
    dalloc((void**)&u->m, off * 4);
    dalloc((void**)&u->v, off * 4);
    dalloc((void**)&u->x0, P0 * u->Cinp * 2);
    dalloc((void**)&u->y, P0 * 4);
    dalloc((void**)&u->dy, P0 * 4);
    dalloc((void**)&u->hpart, (i64)HEAD_BLOCKS * (C0 + 1) * 4);
    dalloc((void**)&u->upb, 4LL * (C0 << (L - 1)) * 4);
    dalloc((void**)&u->lpart, MSE_BLOCKS * 8);
    dalloc((void**)&u->loss, 8);
    dalloc((void**)&u->winfo, 8 * 8);
    dalloc((void**)&u->sphi, (i64)u->H * u->W * 4);
    for (auto* layers : {&u->enc, &u->dec})
        for (auto& c : *layers) dalloc((void**)&c.wb, (i64)c.Co * 9 * c.Cp * 2);
    for (auto& p : u->up) dalloc((void**)&p.wb, 4LL * p.Co * p.Ci * 2);
    auto act = [&](i64 n) {
        Act a;
        dalloc((void**)&a.x, n * 2);
        dalloc((void**)&a.d, n * 2);
        return a;
    };
    for (int l = 0; l < L; ++l) {
        const i64 P = (i64)u->B * (u->H >> l) * (u->W >> l);
        const int co = C0 << l;
        u->c1.push_back(act(P * co));
        u->c2.push_back(act(P * co));
        if (l < L - 1) {
            const i64 Pn = (i64)u->B * (u->H >> (l + 1)) * (u->W >> (l + 1));
            u->pool.push_back(act(Pn * co));
            uint8_t* a = nullptr;
            dalloc((void**)&a, Pn * co);
            u->arg.push_back(a);
        }
    }
    for (int l = L - 2; l >= 0; --l) {
        const i64 P = (i64)u->B * (u->H >> l) * (u->W >> l);
        const int co = C0 << l;
        u->upo.push_back(act(P * co));
        u->d1.push_back(act(P * co));
        u->d2.push_back(act(P * co));
    }
    i64 maxw = 0;
    for (auto* layers : {&u->enc, &u->dec})
        for (auto& c : *layers) maxw = std::max<i64>(maxw, (i64)c.Co * (9LL * c.Cp + 1));
    for (auto& p : u->up) maxw = std::max<i64>(maxw, 4LL * p.Co * (p.Ci + 1));
    u->part_n = std::max<i64>(maxw * 8, (i64)16 << 20);
    dalloc((void**)&u->part, u->part_n * 4);
    if (!ok) {
        (void)hipGetLastError();
        lbm_unet_destroy(u);
        return LBM_E_NOMEM;
    }
    for (float* p : {u->w, u->g, u->m, u->v}) k_fill_f32<<<blocks_for(off), 256, 0, u->stream>>>(p, off, 0.f);
    refresh_bf16(u);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(u->stream) != hipSuccess) {
        lbm_unet_destroy(u);
        return LBM_E_DEVICE;
    }
    *out = u;
    return LBM_OK;
}

int64_t lbm_unet_param_count(const lbm_unet* u) { return u ? u->nparam : 0; }

lbm_status lbm_unet_set_params(lbm_unet* u, const float* p, int64_t n, int on_device) {
    if (!u || !p) return u ? ufail(u, LBM_E_ARG, "set_params: null pointer") : LBM_E_ARG;
    if (n != u->nparam) return ufail(u, LBM_E_ARG, "set_params: count differs from lbm_unet_param_count");
    UCHK(u, hipMemcpyAsync(u->w, p, (size_t)n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           u->stream));
    k_fill_f32<<<blocks_for(n), 256, 0, u->stream>>>(u->m, n, 0.f);
    k_fill_f32<<<blocks_for(n), 256, 0, u->stream>>>(u->v, n, 0.f);
    u->step = 0;
    refresh_bf16(u);
    UCHK(u, hipGetLastError());
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

lbm_status lbm_unet_get_params(lbm_unet* u, float* p, int64_t n, int which, int on_device) {
    if (!u || !p) return u ? ufail(u, LBM_E_ARG, "get_params: null pointer") : LBM_E_ARG;
    if (n != u->nparam) return ufail(u, LBM_E_ARG, "get_params: count differs from lbm_unet_param_count");
    const float* src = which == LBM_UNET_WEIGHTS ? u->w : which == LBM_UNET_GRADS ? u->g : nullptr;
    if (!src) return ufail(u, LBM_E_ARG, "get_params: which must be LBM_UNET_WEIGHTS or LBM_UNET_GRADS");
    UCHK(u, hipMemcpyAsync(p, src, (size_t)n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

lbm_status lbm_unet_forward(lbm_unet* u, const float* x, float* y, int n) {
    if (!u || !x || !y) return u ? ufail(u, LBM_E_ARG, "forward: null pointer") : LBM_E_ARG;
    lbm_status s = load_input(u, x, n);
    if (s) return s;
    forward(u);
    UCHK(u, hipGetLastError());
    UCHK(u, hipMemcpyAsync(y, u->y, (size_t)pixels(u, 0) * 4, hipMemcpyDeviceToDevice, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

lbm_status lbm_unet_loss(lbm_unet* u, const float* x, const float* target, int n, double* loss) {
    if (!u || !x || !target || !loss) return u ? ufail(u, LBM_E_ARG, "loss: null pointer") : LBM_E_ARG;
    lbm_status s = load_input(u, x, n);
    if (s) return s;
    forward(u);
    const i64 np = pixels(u, 0);
    k_mse<<<MSE_BLOCKS, 256, 0, u->stream>>>(u->y, target, np, u->dy, u->lpart);
    k_sum_parts<<<1, 256, 0, u->stream>>>(u->lpart, MSE_BLOCKS, 1.0 / (double)np, u->loss);
    UCHK(u, hipGetLastError());
    UCHK(u, hipMemcpyAsync(loss, u->loss, 8, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

lbm_status lbm_unet_backward(lbm_unet* u, const float* x, const float* target, int n, double* loss) {
    if (!u || !x || !target) return u ? ufail(u, LBM_E_ARG, "backward: null pointer") : LBM_E_ARG;
    return fwd_bwd(u, x, target, n, loss);
}

lbm_status lbm_unet_train_step(lbm_unet* u, const float* x, const float* target, int n, double* loss) {
    if (!u || !x || !target) return u ? ufail(u, LBM_E_ARG, "train_step: null pointer") : LBM_E_ARG;
    lbm_status s;
    if (!u->use_graphs) {
        if ((s = fwd_bwd(u, x, target, n, loss))) return s;
    } else {
        if ((s = load_input(u, x, n))) return s;
        if (u->graph_nb != n) {
            drop_graphs(u);
            if ((s = capture(u, forward, &u->gfwd)) || (s = capture(u, backward, &u->gbwd))) {
                drop_graphs(u);
                return s;
            }
            u->graph_nb = n;
        }
        const i64 np = pixels(u, 0);
        UCHK(u, hipGraphLaunch(u->gfwd, u->stream));
        k_mse<<<MSE_BLOCKS, 256, 0, u->stream>>>(u->y, target, np, u->dy, u->lpart);
        k_sum_parts<<<1, 256, 0, u->stream>>>(u->lpart, MSE_BLOCKS, 1.0 / (double)np, u->loss);
        UCHK(u, hipGraphLaunch(u->gbwd, u->stream));
        UCHK(u, hipGetLastError());
        if (loss) UCHK(u, hipMemcpyAsync(loss, u->loss, 8, hipMemcpyDeviceToHost, u->stream));
    }
    u->step += 1;
    const double b1 = u->cfg.beta1, b2 = u->cfg.beta2;
    const float c1 = (float)(1.0 - std::pow(b1, (double)u->step));
    const float c2 = (float)(1.0 - std::pow(b2, (double)u->step));
    k_adam<<<blocks_for(u->nparam), 256, 0, u->stream>>>(u->w, u->g, u->m, u->v, u->nparam, (float)u->cfg.lr,
                                                         (float)b1, (float)b2, (float)u->cfg.eps, c1, c2);
    refresh_bf16(u);
    UCHK(u, hipGetLastError());
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

// checkpoint file: "LBMUNET1", int32 {in_channels, base_channels, levels, 0},
// int64 {parameter count, Adam step}, then FP32 weights, first and second
// Adam moments (little-endian, as the host writes them)
static const char kUnetMagic[8] = {'L', 'B', 'M', 'U', 'N', 'E', 'T', '1'};

lbm_status lbm_unet_save(lbm_unet* u, const char* path) {
    if (!u || !path) return u ? ufail(u, LBM_E_ARG, "save: null path") : LBM_E_ARG;
    std::vector<float> buf((size_t)u->nparam * 3);
    UCHK(u, hipMemcpyAsync(buf.data(), u->w, (size_t)u->nparam * 4, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipMemcpyAsync(buf.data() + u->nparam, u->m, (size_t)u->nparam * 4, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipMemcpyAsync(buf.data() + 2 * u->nparam, u->v, (size_t)u->nparam * 4, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    FILE* f = std::fopen(path, "wb");
    if (!f) return ufail(u, LBM_E_ARG, std::string("save: cannot open ") + path);
    const int32_t hdr[4] = {u->Cin, u->C0, u->L, 0};
    const int64_t cnt[2] = {u->nparam, u->step};
    bool ok = std::fwrite(kUnetMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 && std::fwrite(cnt, 8, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? LBM_OK : ufail(u, LBM_E_ARG, std::string("save: write failed: ") + path);
}

lbm_status lbm_unet_load(lbm_unet* u, const char* path) {
    if (!u || !path) return u ? ufail(u, LBM_E_ARG, "load: null path") : LBM_E_ARG;
    FILE* f = std::fopen(path, "rb");
    if (!f) return ufail(u, LBM_E_ARG, std::string("load: cannot open ") + path);
    char magic[8];
    int32_t hdr[4];
    int64_t cnt[2];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kUnetMagic, 8) == 0 && std::fread(hdr, 4, 4, f) == 4 &&
              std::fread(cnt, 8, 2, f) == 2;
    if (!ok || hdr[0] != u->Cin || hdr[1] != u->C0 || hdr[2] != u->L || cnt[0] != u->nparam || cnt[1] < 0) {
        std::fclose(f);
        return ufail(u, LBM_E_ARG, std::string("load: not a checkpoint of this architecture: ") + path);
    }
    std::vector<float> buf((size_t)u->nparam * 3);
    ok = std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return ufail(u, LBM_E_ARG, std::string("load: truncated file: ") + path);
    UCHK(u, hipMemcpyAsync(u->w, buf.data(), (size_t)u->nparam * 4, hipMemcpyHostToDevice, u->stream));
    UCHK(u, hipMemcpyAsync(u->m, buf.data() + u->nparam, (size_t)u->nparam * 4, hipMemcpyHostToDevice, u->stream));
    UCHK(u, hipMemcpyAsync(u->v, buf.data() + 2 * u->nparam, (size_t)u->nparam * 4, hipMemcpyHostToDevice, u->stream));
    u->step = cnt[1];
    refresh_bf16(u);
    UCHK(u, hipGetLastError());
    UCHK(u, hipStreamSynchronize(u->stream));
    return LBM_OK;
}

lbm_status lbm_unet_set_lr(lbm_unet* u, double lr) {
    if (!u) return LBM_E_ARG;
    if (!(lr > 0)) return ufail(u, LBM_E_ARG, "set_lr: the rate must be positive");
    u->cfg.lr = lr;
    return LBM_OK;
}

lbm_status lbm_unet_encode(const uint8_t* cls, const float* phi0, int64_t n, double solid_value, double plane,
                           float* x, void* stream) {
    if (!cls || !x || n < 1) return LBM_E_ARG;
    k_encode<<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(cls, phi0, n, (float)solid_value, (float)plane, x);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

lbm_status lbm_unet_target(const void* rho, int precision, const uint8_t* cls, int64_t n, double rho_g, double rho_l,
                           float* phi, void* stream) {
    if (!rho || !cls || !phi || n < 1 || !(rho_l > rho_g)) return LBM_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (precision == LBM_F64)
        k_target<double><<<blocks_for(n), 256, 0, s>>>((const double*)rho, cls, n, rho_g, rho_l, phi);
    else if (precision == LBM_F32 || precision == LBM_F32_MIXED)
        k_target<float><<<blocks_for(n), 256, 0, s>>>((const float*)rho, cls, n, rho_g, rho_l, phi);
    else
        return LBM_E_ARG;
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

lbm_status lbm_unet_warm_rho(lbm_unet* u, const float* phi, const void* rho_ref, const uint8_t* cls, int nx, int ny,
                             int precision, double rho_g, double rho_l, double cut, int smooth, void* rho_out,
                             double* info) {
    if (!u) return LBM_E_ARG;
    const i64 n = (i64)nx * ny;
    if (!phi || !rho_ref || !cls || !rho_out || nx < 1 || ny < 1 || !(rho_l > rho_g))
        return ufail(u, LBM_E_ARG, "warm_rho: null pointer, empty field or rho_l <= rho_g");
    if (!(cut >= 0.0 && cut < 0.25)) return ufail(u, LBM_E_ARG, "warm_rho: cut must be in [0, 0.25)");
    if (smooth < 0 || smooth > 8) return ufail(u, LBM_E_ARG, "warm_rho: smooth must be in 0..8");
    if (smooth > 0) {
        if (n > (i64)u->H * u->W) return ufail(u, LBM_E_ARG, "warm_rho: smoothing needs nx * ny <= H * W");
        k_smooth_fluid<<<blocks_for(n), 256, 0, u->stream>>>(phi, cls, nx, ny, smooth, u->sphi);
        phi = u->sphi;
    }
    if (precision == LBM_F64)
        k_warm_rho<double><<<1, 1024, 0, u->stream>>>(phi, (const double*)rho_ref, cls, n, rho_g, rho_l, cut,
                                                      (double*)rho_out, u->winfo);
    else if (precision == LBM_F32 || precision == LBM_F32_MIXED)
        k_warm_rho<float><<<1, 1024, 0, u->stream>>>(phi, (const float*)rho_ref, cls, n, rho_g, rho_l, cut,
                                                     (float*)rho_out, u->winfo);
    else
        return ufail(u, LBM_E_ARG, "warm_rho: unknown precision");
    double h[5];
    UCHK(u, hipGetLastError());
    UCHK(u, hipMemcpyAsync(h, u->winfo, sizeof h, hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    if (info) std::memcpy(info, h, sizeof h);
    const double target = (h[0] - h[4] * rho_g) / (rho_l - rho_g);
    if (!(target > 0.0 && target < h[4]))
        return ufail(u, LBM_E_ARG, "warm_rho: the reference mass is outside (n_fluid rho_g, n_fluid rho_l)");
    return LBM_OK;
}

}  // extern "C"
