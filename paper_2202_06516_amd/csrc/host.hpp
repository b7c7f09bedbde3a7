// host.hpp -- host-side thermodynamics and geometry of the GPU library.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace lbm {

// node class codes (low two bits), the boundary-fluid flag, and the flag of a
// boundary fluid node with a cut link whose wall fraction is not 1/2 (where
// the interpolated wall differs from halfway bounce-back)
constexpr uint8_t CLS_FLUID_ = 0, CLS_BOUNDARY_ = 4, CLS_CURVED_ = 8;

// Peng-Robinson fluid (Eq. 10-11) at a reduced temperature.
struct PRState {
    double a, b, R, omega, Tr;
    double Tc, rhoc, T, alpha;
    double rho_g, rho_l, p_sat, mu_sat;
};

double pr_alpha(double Tr, double omega);
double pr_pressure(double rho, double T, double a, double b, double R, double alpha);
double pr_chem(double rho, double T, double a, double b, double R, double alpha);  // psi'(rho), C = 0
// critical point and Maxwell coexistence; returns false if no two-phase region
bool pr_solve(PRState& s, std::string& err);

struct Solid {
    double c[3], r;
    bool concave;  // false: solid ball |x - c| <= r; true: solid outside, |x - c| >= r
    int wet_mode;  // 0 uniform, 1 stripes
    double mu1, mu2, width, pole[3];
};

// Node classes, neighbour masks and compact boundary lists.
struct Geometry {
    int dim = 2, Q = 9, nx = 0, ny = 0, nz = 1;
    long long N = 0;
    std::vector<uint8_t> cls;          // class | boundary flag
    std::vector<uint32_t> nbmask;      // solid-neighbour bits (boundary fluid nodes)
    std::vector<long long> l1_node, l2_node;
    std::vector<uint32_t> l1_mask, l2_mask;
    std::vector<double> l1_inv, l2_inv;
    std::vector<double> l1_mu, l2_mu;  // wall chemical potential of the layer nodes
    std::vector<long long> b_node;     // boundary fluid nodes
    std::vector<uint32_t> b_mask;
    std::vector<double> b_q;           // [nb][Q] wall fraction of each cut link
    long long n_fluid = 0;
};

// Build the geometry of a lattice with the given solids.  wall[d]: two solid
// layers at both ends of axis d.  mu_map (N doubles) overrides wettability.
bool build_geometry(Geometry& g, int dim, const int n[3], const int wall[3], const std::vector<Solid>& solids,
                    const double* mu_map, double wall_mu, std::string& err);

}  // namespace lbm
