// Reference tetrahedron data for the P_N AFE basis and the Gauss-Legendre
// time basis (host side, computed once per degree).
#pragma once
#include <array>
#include <vector>

namespace afe {

constexpr int kMaxN = 4;
constexpr int kMaxNp = 35;  // (N+1)(N+2)(N+3)/6 at N = 4
constexpr int kMaxNf = 15;  // (N+1)(N+2)/2 at N = 4
constexpr int kMaxNt = 5;   // N + 1 time nodes

struct RefData {
    int N = 0, np = 0, nf = 0, nt = 0;
    // node lattice: integer barycentric weights N*(lambda1..lambda4) per node,
    // lambda1 = 1 - r - s - t, lambda2 = r, lambda3 = s, lambda4 = t
    std::vector<std::array<int, 4>> bary;
    std::vector<std::array<double, 3>> xi;  // reference coordinates (r, s, t)
    std::vector<int> face_nodes;            // nodes with t = 0, in node order
    std::vector<double> M;                  // [np][np]   int phi_m phi_l
    std::vector<double> K;                  // [3][np][np] int phi_m d_d phi_l
    std::vector<double> D;                  // [3][np][np] d_d phi_l (x_m)
    std::vector<double> Z;                  // [nf][nf]  face mass, reference triangle
    // time basis on [0, 1]
    std::vector<double> tau, w;             // Gauss-Legendre nodes and weights
    std::vector<double> Ktau, Ktau_inv;     // [nt][nt]
    // volume quadrature for error norms: conical product of (N + 3)-point
    // Gauss-Legendre rules, xi = (a (1-b)(1-c), b (1-c), c), weight
    // w_a w_b w_c (1-b)(1-c)^2; exact for polynomials of degree 2N + 3
    int nq = 0;
    std::vector<double> qxi;                // [nq][3]
    std::vector<double> qw;                 // [nq], sum 1/6
    std::vector<double> qphi;               // [nq][np] phi_m(xi_q)
};

constexpr int kMaxNq = (kMaxN + 3) * (kMaxN + 3) * (kMaxN + 3);

// Builds the exact reference data for 1 <= N <= 4 (cached).
const RefData &ref_data(int N);

}  // namespace afe
