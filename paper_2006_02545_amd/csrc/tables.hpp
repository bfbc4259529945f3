// tables.hpp -- host-side reference data per degree (Section 2 of the paper)
// and the Gauss rules used by the quadratures.
#pragma once

#include <string>
#include <vector>

namespace nfq {

struct RefData {
    int d = 0, nd = 0;
    std::vector<double> uv;   // [nd][2] interpolation nodes on T0
    std::vector<double> V;    // [nd][nd], V[a * nd + l]: values -> Koornwinder coefficients
    std::vector<double> w;    // [nd] quadrature weights at the nodes
    std::vector<double> D;    // [2][nd][nd]: D[0][a][m] = int_T0 dK_a/du K_m, D[1]: d/dv
                              // (K orthonormal on T0, so dK_a/du = sum_m D[0][a][m] K_m)
    double normV = 0.0;       // ||V||_2
    double cond = 0.0;        // ||U||_2 ||V||_2
};

// Build U_(nm),j = K_nm(u_j, v_j), V = U^{-1} (LU with partial pivoting in
// long double), ||V||_2 (power iteration on V^T V), and the interpolatory
// weights w_l = int_T0 L_l = V_(00),l / sqrt(2) when w_in is null.
// Returns an empty string on success, else the reason.
std::string build_reference(int d, const double *uv, const double *w_in, RefData &out);

// Gauss rule with n points on [0,1] for the weight (1-y)^a y^b (a, b >= 0
// integers), by Golub-Welsch: eigen-decomposition of the Jacobi matrix of
// the monic recurrence (implicit QL on the symmetric tridiagonal matrix).
void gauss_rule(int n, int a, int b, std::vector<double> &y, std::vector<double> &w);

// Conical-product rule on T0 with ng*ng points: v = y (Gauss-Jacobi, weight
// 1 - y), u = x (1 - y) (Gauss-Legendre); exact for total degree 2 ng - 1.
// Output [q][3] = (u, v, w), weights sum to 1/2.
void conical_rule(int ng, std::vector<double> &uvw);

}  // namespace nfq
