// Internal data structures of the igamg library (host setup, kernels, cycle).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/igamg.h"

namespace igamg {

constexpr int MAXP = 8;   // largest spline degree
constexpr int MAXQ = 12;  // largest Gauss rule

struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
#define HIPCHK(x)                                                                \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess)                                                        \
      ::igamg::fail(IGAMG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Gauss-Legendre rule on [0,1], passed to kernels by value.
struct GaussRule {
  int q;
  double x[MAXQ];
  double w[MAXQ];
};

// One patch on one level, as the kernels see it.
struct PatchDev {
  double corners[8][3];
  int n[3];          // basis functions per direction (nel + p); 1 in unused directions
  int nel[3];        // elements per direction
  int stride[3];     // tensor strides (x fastest)
  long long off;     // offset of the patch tensor in the level vector
  int tab[3];        // offset of the direction's 1D element tables ([e][g][a] entries)
  int xp[3];         // prolongation rows from the coarser level: offset into lo / val tables
  int xr[3];         // restriction rows to the coarser level (on the coarse patch entry)
  int color;         // patch colour of the Gauss-Seidel ordering
  int p;             // spline degree of the patch
  double scms_scale; // tau / gamma_k
  double sigma;      // SCMS scaling 1/(delta h^2)
};

struct VolTile {
  int patch;
  int e0[3];
};

// Element tile of the 2D operator kernel with the fields of its patch (the
// tile record is the only load the kernel's data loads depend on).
struct OpTile2 {
  double corners[4][2];  // patch corners (x fastest)
  long long off;         // patch offset in the level vector
  int nx;                // unknowns per row of the patch tensor
  int nel[2];            // elements per direction
  int tab[2];            // 1D table offsets per direction
  int e0[2];             // first element of the tile
};

// Output tile of a transfer kernel (2D): up to 16 x 16 outputs of one patch
// and the window of input entries they read, all resolved at setup so that
// the kernel's loads depend on this record only.
// 2D transfer tiles (16 output rows): output columns per tile and the
// largest input window (columns x rows) each kernel form stages in LDS
constexpr int XFER_TX = 16, XFER_WX = 64;                        // any level
constexpr int XFER_R_TX = 32, XFER_R_WX = 72, XFER_R_WY = 40;  // restriction
constexpr int XFER_P_TX = 64, XFER_P_WX = 40, XFER_P_WY = 16;  // prolongation
struct XferTile {
  long long in_off, out_off;  // patch offsets in the input / output level vectors
  int in_nx, out_nx;          // x extents of the input / output patch tensors
  int o0[2], no[2];           // first output index and output count per direction
  int base[2];                // band-table row of the first output per direction
  int w0[2], wn[2];           // input window origin and extent per direction
};

// Gauss-Seidel tile with the fields of its patch that the kernel needs, so
// that the tile record is the only load the kernel's data loads depend on.
struct GsTile {
  long long off;     // patch offset in the level vector
  int nx, ny;        // patch tensor extents
  int i0[2];         // first unknown of the tile
  // cross-patch couplings of the tile rows, in slots of the level's flat
  // lists: cx_np passes of 64 slots (one per lane), cx_k entries per slot
  // (entry k of the slot in lane l of pass q at cx_off + (q cx_k + k) 64 + l;
  // padding: column -1), slot codes at cx_sl + 64 q + l (row | index of the
  // slot in its row << 16 | slots of the row << 24, or -1); the slots of a
  // row are consecutive lanes of one pass, at most cx_r of them
  int cx_off, cx_k;
  int cx_sl, cx_np;
  int cx_r;
  int mr_off, mr_n;  // conforming: copies in other patches of the tile's owned glued
                     // unknowns (mirror writes, in the level's flat lists)
  long long pad_off; // lane-per-right-hand-side operator: the patch's offset in the
                     // transposed copy with a halo of p zero rows and columns
};

// Gauss-Seidel tile of a 3D patch (2(p+1) unknowns per direction), with the
// fields of its patch that the kernels need (the cross-patch couplings of 3D
// levels are a CSR over the coupled rows, not per tile).
struct GsTile3 {
  long long off;     // patch offset in the level vector
  int n[3];          // patch tensor extents
  int i0[3];         // first unknown of the tile
  int mr_off, mr_n;  // conforming: mirror writes of the tile's owned glued unknowns
};

// Two chained products on a block of 16 rows (fast-diagonalization step of the
// subspace corrected mass smoother): Z = L[rows, :] M1, R = Z M2, then either
// O[rows, :] = R / (sigma + lam_r[row] + lam_c[col]) (lam_r != null) or
// O[rows, :] += scale R.  All operands are row-major with unit column stride;
// *_z is the element stride between right-hand sides of a batch (0 = shared).
template <typename T>
struct Fd2Item {
  const T *L;   // rows x K1, row stride l_r
  const T *M1;  // K1 x N, row stride m1_r
  const T *M2;  // N x N, row stride m2_r
  T *O;         // rows x N, row stride o_r
  long long l_r, m1_r, m2_r, o_r;
  long long m1_z, o_z;
  int rows, K1, N;
  const T *lam_r;
  const T *lam_c;
  T sigma;
  T scale;
};

// One product stage of the fast diagonalization on a batch: for every
// right-hand side z, C_z = A_z B_z (mode 0), C_z = A_z B_z ./ (sigma + lam_r[i]
// + lam_c[j]) (mode 1) or C_z += scale A_z B_z (mode 2).  Row-major operands;
// *_z is the element stride between right-hand sides (0 = shared operand).
template <typename T>
struct FdGemm {
  const T *A, *B;
  T *C;
  long long a_r, b_r, c_r;
  long long a_z, b_z, c_z;
  int M, N, K;
  int tn;  // 64-column tiles of C
  const T *lam_r, *lam_c;
  T sigma, scale;
  int mode;
};

// One product stage of the 2D fast diagonalization with the right-hand sides
// of a batch concatenated along the per-right-hand-side dimension:
//   left:  C_z[w][n] = sum_k S[w][k] X_z[k][n]    (X_z[k][n] at X + z x_z + k x_r + n)
//   right: C_z[i][w] = sum_k X_z[i][k] S[w][k]    (X_z[i][k] at X + z x_z + i x_r + k)
// S (the shared 1D factor, S[w][k] at S + w s_r + k) spans the wide dimension
// (`wide` <= 320 entries, one block covers all of it); the concatenated
// dimension runs over z * catn + (n or i).  C at C + z c_z + row c_r + col;
// mode 0: C = v, 1: C = v / (sigma + lam_r[row] + lam_c[col]), 2: C += scale v.
template <typename T>
struct FdWide {
  const T *S, *X;
  T *C;
  long long s_r, x_r, x_z, c_r, c_z;
  int wide, catn, K;
  const T *lam_r, *lam_c;
  T sigma, scale;
  int mode;
};

// Interface piece of the additive smoother (eq. Ldef): dense inverse of P^T A P.
struct PieceDev {
  long long inv_off;  // offset of the n x n inverse in the value array
  int n;
  int idx_off;        // gather indices (one torn index per piece unknown)
  int cp_off;         // scatter CSR row pointer offset (n+1 entries)
};

}  // namespace igamg
