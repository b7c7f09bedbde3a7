// lattice.hpp -- compile-time lattice descriptors for the GPU path.
//
// D2Q9 (the paper's lattice, Sec. II A) and D3Q19 (the three-dimensional
// extension).  Velocities, weights, opposite directions and the orthogonal
// MRT moment basis are constexpr so that fully unrolled device loops fold
// every table entry into an immediate.
//
// The MRT basis rows are polynomials of the lattice velocity: D2Q9 in the
// Lallemand-Luo order (rho, e, eps, jx, qx, jy, qy, pxx, pxy) that the
// relaxation matrix S of Sec. II A is written in; D3Q19 in the d'Humieres et
// al. 19-moment order.  The rows are mutually orthogonal, so the inverse
// transform is M^T D^-1 with D = diag(M M^T); the kernels use that form.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int E[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // moment polynomial k at velocity i
    __host__ __device__ static constexpr double m(int k, int i) {
        double x = E[i][0], y = E[i][1];
        double c2 = x * x + y * y;
        switch (k) {
            case 0: return 1.0;
            case 1: return 3.0 * c2 - 4.0;
            case 2: return 4.5 * c2 * c2 - 10.5 * c2 + 4.0;
            case 3: return x;
            case 4: return (3.0 * c2 - 5.0) * x;
            case 5: return y;
            case 6: return (3.0 * c2 - 5.0) * y;
            case 7: return x * x - y * y;
            default: return x * y;
        }
    }
    // moment classes: 0 conserved, 1 e, 2 eps, 3 q, 4 stress (s_v), 5 pi, 6 m
    __host__ __device__ static constexpr int kind(int k) {
        return (k == 0 || k == 3 || k == 5) ? 0 : (k == 1 ? 1 : (k == 2 ? 2 : ((k == 4 || k == 6) ? 3 : 4)));
    }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int E[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                     {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                     {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                     {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr double m(int k, int i) {
        double x = E[i][0], y = E[i][1], z = E[i][2];
        double c2 = x * x + y * y + z * z;
        switch (k) {
            case 0: return 1.0;
            case 1: return 19.0 * c2 - 30.0;
            case 2: return 0.5 * (21.0 * c2 * c2 - 53.0 * c2 + 24.0);
            case 3: return x;
            case 4: return (5.0 * c2 - 9.0) * x;
            case 5: return y;
            case 6: return (5.0 * c2 - 9.0) * y;
            case 7: return z;
            case 8: return (5.0 * c2 - 9.0) * z;
            case 9: return 3.0 * x * x - c2;
            case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
            case 11: return y * y - z * z;
            case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
            case 13: return x * y;
            case 14: return y * z;
            case 15: return x * z;
            case 16: return (y * y - z * z) * x;
            case 17: return (z * z - x * x) * y;
            default: return (x * x - y * y) * z;
        }
    }
    __host__ __device__ static constexpr int kind(int k) {
        return (k == 0 || k == 3 || k == 5 || k == 7) ? 0
             : k == 1 ? 1
             : k == 2 ? 2
             : (k == 4 || k == 6 || k == 8) ? 3
             : (k == 9 || k == 11 || k == 13 || k == 14 || k == 15) ? 4
             : (k == 10 || k == 12) ? 5
             : 6;
    }
};

// squared norm of moment row k (diagonal of M M^T)
template <class L>
__host__ __device__ constexpr double row_norm2(int k) {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += L::m(k, i) * L::m(k, i);
    return s;
}

}  // namespace lbm
