// Geometry and quadrature helpers shared by host setup and device kernels.
//
// Patch maps are multilinear interpolations of the 2^d corners (corner b has
// parameter coordinates bit_delta(b)).  The stiffness integrand of Section 2,
// eq. model, on the parameter domain is grad_hat(u)^T G grad_hat(v) with the
// metric G = |det J| J^-1 J^-T.
#pragma once
#include "internal.h"

namespace igamg {

template <int D>
__host__ __device__ inline void multilinear_jac(const double (*c)[3], const double *xh,
                                                double J[D][D]) {
  for (int a = 0; a < D; ++a)
    for (int g = 0; g < D; ++g) J[a][g] = 0.0;
  for (int b = 0; b < (1 << D); ++b) {
    double f[D];
    for (int d = 0; d < D; ++d) f[d] = ((b >> d) & 1) ? xh[d] : 1.0 - xh[d];
    for (int g = 0; g < D; ++g) {
      double dw = ((b >> g) & 1) ? 1.0 : -1.0;
      for (int d = 0; d < D; ++d)
        if (d != g) dw *= f[d];
      for (int a = 0; a < D; ++a) J[a][g] += dw * c[b][a];
    }
  }
}

template <int D>
__host__ __device__ inline void multilinear_map(const double (*c)[3], const double *xh, double *X) {
  for (int a = 0; a < D; ++a) X[a] = 0.0;
  for (int b = 0; b < (1 << D); ++b) {
    double w = 1.0;
    for (int d = 0; d < D; ++d) w *= ((b >> d) & 1) ? xh[d] : 1.0 - xh[d];
    for (int a = 0; a < D; ++a) X[a] += w * c[b][a];
  }
}

// Inverse and determinant of a D x D matrix.
template <int D>
__host__ __device__ inline double inverse(const double J[D][D], double Ji[D][D]) {
  if (D == 2) {
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
    return det;
  } else {
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    Ji[0][0] = c00 / det;
    Ji[1][0] = c01 / det;
    Ji[2][0] = c02 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    return det;
  }
}

// w |det J| J^-1 J^-T at parameter point xh; returns det J.
template <int D>
__host__ __device__ inline double metric(const double (*c)[3], const double *xh, double w,
                                         double G[D][D]) {
  double J[D][D], Ji[D][D];
  multilinear_jac<D>(c, xh, J);
  double det = inverse<D>(J, Ji);
  double s = w * (det < 0 ? -det : det);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double v = 0.0;
      for (int g = 0; g < D; ++g) v += Ji[a][g] * Ji[b][g];
      G[a][b] = s * v;
    }
  return det;
}

// Volume stiffness entry a(phi_j, phi_i) = sum over common elements and Gauss
// points of grad_hat(phi_i)^T G grad_hat(phi_j) for the tensor B-splines with
// multi-indices i and j of one patch (q = p+1 points per direction).
template <int D>
__host__ __device__ inline double vol_entry(const PatchDev &pt, const double *tabB,
                                            const double *tabD, const GaussRule &gr, int p,
                                            const int *i, const int *j) {
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    int a = i[d] > j[d] ? i[d] : j[d];
    int b = i[d] < j[d] ? i[d] : j[d];
    lo[d] = a - p < 0 ? 0 : a - p;
    hi[d] = b > pt.nel[d] - 1 ? pt.nel[d] - 1 : b;
    if (lo[d] > hi[d]) return 0.0;
  }
  const int q = gr.q, P1 = p + 1;
  double sum = 0.0;
  int e[3] = {lo[0], lo[1], lo[2]};
  for (;;) {
    int g[3] = {0, 0, 0};
    for (;;) {
      double xh[D], w = 1.0;
      double bi[D], di[D], bj[D], dj[D];
      for (int d = 0; d < D; ++d) {
        xh[d] = ((double)e[d] + gr.x[g[d]]) / (double)pt.nel[d];
        w *= gr.w[g[d]] / (double)pt.nel[d];
        size_t row = (size_t)pt.tab[d] + ((size_t)e[d] * q + g[d]) * P1;
        bi[d] = tabB[row + (i[d] - e[d])];
        di[d] = tabD[row + (i[d] - e[d])];
        bj[d] = tabB[row + (j[d] - e[d])];
        dj[d] = tabD[row + (j[d] - e[d])];
      }
      double G[D][D];
      metric<D>(pt.corners, xh, w, G);
      double gi[D], gj[D];
      for (int a = 0; a < D; ++a) {
        gi[a] = di[a];
        gj[a] = dj[a];
        for (int d = 0; d < D; ++d)
          if (d != a) {
            gi[a] *= bi[d];
            gj[a] *= bj[d];
          }
      }
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) sum += gi[a] * G[a][b] * gj[b];
      int d = 0;
      while (d < D && ++g[d] == q) g[d++] = 0;
      if (d == D) break;
    }
    int d = 0;
    while (d < D && ++e[d] > hi[d]) {
      e[d] = lo[d];
      ++d;
    }
    if (d == D) break;
  }
  return sum;
}

}  // namespace igamg
