// Host-side numerics of the setup phase: Gauss rules, B-spline evaluation,
// small dense linear algebra, the 1D factors of the subspace corrected mass
// smoother and the 1D embedding between dyadic spline spaces.
#pragma once
#include <vector>

#include "internal.h"

namespace igamg {

// q-point Gauss-Legendre rule on [0,1] (Newton iteration on P_q).
GaussRule gauss_rule(int q);

// Open uniform knot vector with n_el elements, degree p on [0,1].
std::vector<double> open_knots(int n_el, int p);

// Derivatives 0..nd of the p+1 B-splines that are non-zero on knot span
// [t_m, t_{m+1}) at x: out[k][a] = d^k/dx^k N_{m-p+a}(x).
void bspline_span_ders(const std::vector<double> &t, int p, int m, double x, int nd,
                       double out[][MAXP + 1]);

// Tables of values and parameter derivatives at the q Gauss points of every
// element: B[(e*q + g)*(p+1) + a] = N_{e+a}(x_{e,g}), D likewise.
void element_tables(int n_el, int p, const GaussRule &gr, std::vector<double> &B,
                    std::vector<double> &D);

// Dense row-major helpers (n x n unless stated).
bool cholesky(std::vector<double> &A, int n);  // in place, lower factor; false if not SPD
void chol_solve(const std::vector<double> &L, int n, double *b);  // b <- A^-1 b
std::vector<double> spd_inverse(const std::vector<double> &A, int n);
// Symmetric eigen-decomposition by cyclic Jacobi: A = V diag(w) V^T.
void jacobi_eigen(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V);
// Orthonormal basis (n x (n-m)) of the null space of the m x n matrix C (Householder QR of C^T).
std::vector<double> null_space(const std::vector<double> &C, int m, int n);

// 1D factors of the subspace corrected mass smoother (Section 5) on the
// interior B-splines N_1..N_{n-2} of S_{p,1/n_el}: Q (n' x n', row-major,
// Q^T M Q = I) and lam (n'), lam = 0 on the subspace of splines whose even
// derivatives 2l (1 <= l, 2l < p) vanish at both ends, generalized
// eigenvalues of the stiffness matrix on its mass-orthogonal complement.
void scms_factors_1d(int n_el, int p, std::vector<double> &Q, std::vector<double> &lam);

// Canonical embedding S_{p,1/n_c} -> S_{p,1/(2 n_c)} as a dense (n_f x n_c)
// row-major matrix, computed as the L2 projection M_ff^-1 M_fc (exact).
std::vector<double> embedding_1d(int n_c, int p);

}  // namespace igamg
