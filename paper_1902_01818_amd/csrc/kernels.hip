// HIP kernels of the multigrid cycle for gfx950 (MI355X).
//
//  * volume operator: per-patch stiffness (Section 2, eq. model) applied
//    matrix-free by sum factorization over element tiles staged in LDS (2D
//    and 3D), the metric |det J| J^-1 J^-T recomputed from the patch corners
//    at every Gauss point, or from the stored stencil rows of the
//    Gauss-Seidel levels;
//  * interface terms of the SIPG form (Section 3, eq. model:discr2) as a
//    sparse row-gather over the unknowns next to interfaces, or in the
//    stored rows plus the cross-patch couplings (per tile in 2D, per coupled
//    row in 3D);
//  * multicolour Gauss-Seidel (Section 4): one wavefront per tile of a fixed
//    colour order in 2D, one block of eight wavefronts per tile in 3D;
//  * the subspace corrected mass smoother (Section 5, eq. Ldef): patch
//    interiors by fast diagonalization on the matrix cores (fused row-block
//    products or batched product stages; six mode-product stages in 3D),
//    interface pieces by dense inverses of P^T A P;
//  * canonical embedding / its transpose between dyadic levels (Section 4);
//  * direct coarse solve (float64) and deterministic reductions of the outer
//    conjugate gradient iteration;
//  * setup: stencil rows (sum factorization in 2D, element matrices and a
//    fixed-order gather in 3D), batched Gauss-Jordan inverses, and the L2
//    error against the manufactured solution.
// Cycle kernels are templates on the storage / arithmetic type (double or
// float) and process a batch of right-hand sides (a grid dimension) that
// share all operator data; vectors of the batch follow each other with
// stride Ntorn.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>

#include "geom.h"
#include "hostmath.h"
#include "kernels.h"

namespace igamg {

namespace {

constexpr int BS = 256;

// Gauss rules by number of points, computed once
const GaussRule &rule_of(int q) {
  static const std::vector<GaussRule> rules = [] {
    std::vector<GaussRule> v(MAXQ + 1);
    for (int n = 1; n <= MAXQ; ++n) v[n] = gauss_rule(n);
    return v;
  }();
  return rules[q];
}

inline unsigned nblocks(long long n, int bs = BS) {
  long long b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > 65535LL * 64) b = 65535LL * 64;
  return (unsigned)b;
}

// Event timing of one launch (or launch group) of a kernel family on a level,
// recorded on the launch stream when the family matches the context's filter.
struct TimeScope {
  Context &c;
  std::string key;
  bool on = false;
  hipEvent_t b = nullptr, e = nullptr;
  int n = 1;  // kernel launches covered by this event pair
  TimeScope(Context &c_, const char *f, int level) : c(c_) {
    if (!c.opt.timing) return;
    key = std::string(f) + "/" + std::to_string(level);
    on = c.timing_filter.empty() || key.rfind(c.timing_filter, 0) == 0;
    if (on) c.launch_begin(key.c_str(), &b, &e);
  }
  ~TimeScope() {
    if (on) c.launch_end(key.c_str(), b, e, n);
  }
};

// Cross-lane sums without LDS traffic: DPP row shifts (bound_ctrl: lanes
// without a source read 0) build an inclusive scan inside every row of 16
// lanes; lane 15 of a row then holds the row sum.
template <int CTRL>
__device__ inline double dpp_shift(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ inline float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <typename T>
__device__ inline T row16_scan(T v) {
  v += dpp_shift<0x111>(v);  // row_shr:1
  v += dpp_shift<0x112>(v);  // row_shr:2
  v += dpp_shift<0x114>(v);  // row_shr:4
  v += dpp_shift<0x118>(v);  // row_shr:8
  return v;
}

template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  using type = double2;
};
template <>
struct Pair2<float> {
  using type = float2;
};

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(T *x, T v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

// y = w .* x (w may be null), converted; zero[i] = 0 alongside when given;
// right-hand sides with active[j] == 0 are left alone.  grid.y = right-hand side
template <typename Ti, typename To>
__global__ void convert_kernel(const Ti *x, const To *w, To *y, long long n, To *zero,
                               const int *active) {
  const long long z = blockIdx.y;
  if (active && !active[z]) return;
  x += z * n;
  y += z * n;
  if (zero) zero += z * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    y[i] = w ? w[i] * (To)x[i] : (To)x[i];
    if (zero) zero[i] = 0;
  }
}

// ---------------------------------------------------------------------------
// setup: stencil (volume stiffness rows) assembly, gather form; rows padded
// to whole 16-lane groups (zero coefficients)
// ---------------------------------------------------------------------------
template <int D>
__global__ void stencil_kernel(const PatchDev *pd, int K, const double *tabB, const double *tabD,
                               GaussRule gr, int p, long long ntorn, double *st) {
  const int S1 = 2 * p + 1;
  int S = 1;
  for (int d = 0; d < D; ++d) S *= S1;
  const int SP = (S + 15) / 16 * 16;
  long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (tid >= ntorn * SP) return;
  long long t = tid / SP;
  int o = (int)(tid % SP);
  if (o >= S) {
    st[tid] = 0.0;
    return;
  }
  int k = 0;
  while (k + 1 < K && pd[k + 1].off <= t) ++k;
  const PatchDev &pt = pd[k];
  long long loc = t - pt.off;
  int i[3] = {0, 0, 0}, j[3] = {0, 0, 0};
  bool ok = true;
  int oo = o;
  for (int d = 0; d < D; ++d) {
    i[d] = (int)(loc % pt.n[d]);
    loc /= pt.n[d];
    j[d] = i[d] + (oo % S1) - p;
    oo /= S1;
    if (j[d] < 0 || j[d] >= pt.n[d]) ok = false;
  }
  st[tid] = ok ? vol_entry<D>(pt, tabB, tabD, gr, p, i, j) : 0.0;
}

// 3D stencil rows in two steps over a slab of element layers of one patch:
// (1) the element stiffness matrices, one block per element: the metric at the
// element's q^3 Gauss points and its 1D tables in LDS, then every entry
// (a, b) of the (p+1)^3 x (p+1)^3 matrix summed over the points;
// (2) every row entry (i, j) as the sum of K_e[i - e][j - e] over the common
// elements e in a fixed order (z, y, x), so the rows do not depend on the
// slab partition or on scheduling.
template <int P>
__global__ __launch_bounds__(256) void elem3d_kernel(const PatchDev *pd, int k, int ez0,
                                                     const double *tabB, const double *tabD,
                                                     GaussRule gr, double *Ke) {
  constexpr int P1 = P + 1, Q = P + 1, NB = P1 * P1 * P1, NQ = Q * Q * Q;
  __shared__ double sG[6][NQ];
  __shared__ double sB[3][Q][P1], sD[3][Q][P1];
  const PatchDev &pt = pd[k];
  const int nelx = pt.nel[0], nely = pt.nel[1];
  const long long le = blockIdx.x;
  const int el[3] = {(int)(le % nelx), (int)(le / nelx % nely), ez0 + (int)(le / ((long long)nelx * nely))};
  const int tid = threadIdx.x;
  for (int e = tid; e < 3 * Q * P1; e += 256) {
    const int g = e / (Q * P1), r = e % (Q * P1), qq = r / P1, a = r % P1;
    const size_t row = (size_t)pt.tab[g] + ((size_t)el[g] * Q + qq) * P1 + a;
    sB[g][qq][a] = tabB[row];
    sD[g][qq][a] = tabD[row];
  }
  for (int qi = tid; qi < NQ; qi += 256) {
    const int qx = qi % Q, qy = qi / Q % Q, qz = qi / (Q * Q);
    const int qd[3] = {qx, qy, qz};
    double xh[3], w = 1.0;
    for (int g = 0; g < 3; ++g) {
      xh[g] = ((double)el[g] + gr.x[qd[g]]) / (double)pt.nel[g];
      w *= gr.w[qd[g]] / (double)pt.nel[g];
    }
    double G[3][3];
    metric<3>(pt.corners, xh, w, G);
    sG[0][qi] = G[0][0];
    sG[1][qi] = G[0][1];
    sG[2][qi] = G[0][2];
    sG[3][qi] = G[1][1];
    sG[4][qi] = G[1][2];
    sG[5][qi] = G[2][2];
  }
  __syncthreads();
  double *out = Ke + le * (long long)(NB * NB);
  for (int ent = tid; ent < NB * NB; ent += 256) {
    const int a = ent / NB, b = ent % NB;
    const int ax = a % P1, ay = a / P1 % P1, az = a / (P1 * P1);
    const int bx = b % P1, by = b / P1 % P1, bz = b / (P1 * P1);
    double sum = 0.0;
    for (int qz = 0; qz < Q; ++qz)
      for (int qy = 0; qy < Q; ++qy)
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
          const int qi = (qz * Q + qy) * Q + qx;
          const double Bax = sB[0][qx][ax], Bay = sB[1][qy][ay], Baz = sB[2][qz][az];
          const double Bbx = sB[0][qx][bx], Bby = sB[1][qy][by], Bbz = sB[2][qz][bz];
          const double ga0 = sD[0][qx][ax] * Bay * Baz, ga1 = Bax * sD[1][qy][ay] * Baz,
                       ga2 = Bax * Bay * sD[2][qz][az];
          const double gb0 = sD[0][qx][bx] * Bby * Bbz, gb1 = Bbx * sD[1][qy][by] * Bbz,
                       gb2 = Bbx * Bby * sD[2][qz][bz];
          const double G00 = sG[0][qi], G01 = sG[1][qi], G02 = sG[2][qi];
          const double G11 = sG[3][qi], G12 = sG[4][qi], G22 = sG[5][qi];
          sum += ga0 * (G00 * gb0 + G01 * gb1 + G02 * gb2) + ga1 * (G01 * gb0 + G11 * gb1 + G12 * gb2) +
                 ga2 * (G02 * gb0 + G12 * gb1 + G22 * gb2);
        }
    out[ent] = sum;
  }
}

// Rows of patch k (degree P) in the level's layout: slots of the largest
// degree pm ((2pm+1)^3, row stride SP); offsets beyond P get no element
// (an empty range below) and hold zero.
template <int P>
__global__ __launch_bounds__(256) void gather3d_kernel(const PatchDev *pd, int k, int iz0, int iz1,
                                                       int ez0, const double *Ke, double *st,
                                                       int SP, int pm) {
  constexpr int P1 = P + 1, NB = P1 * P1 * P1;
  const int S1 = 2 * pm + 1, S = S1 * S1 * S1;
  const PatchDev &pt = pd[k];
  const int nx = pt.n[0], ny = pt.n[1], nz = pt.n[2];
  const int nelx = pt.nel[0], nely = pt.nel[1], nelz = pt.nel[2];
  const long long nrow = (long long)nx * ny * (iz1 - iz0);
  const long long tid = blockIdx.x * 256LL + threadIdx.x;
  if (tid >= nrow * SP) return;
  const long long rl = tid / SP;
  const int o = (int)(tid % SP);
  const int ix = (int)(rl % nx), iy = (int)(rl / nx % ny), iz = iz0 + (int)(rl / ((long long)nx * ny));
  const long long t = pt.off + ((long long)iz * ny + iy) * nx + ix;
  double sum = 0.0;
  if (o < S) {
    const int jx = ix + o % S1 - pm, jy = iy + o / S1 % S1 - pm, jz = iz + o / (S1 * S1) - pm;
    if (jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz) {
      const int zlo = max(max(iz, jz) - P, 0), zhi = min(min(iz, jz), nelz - 1);
      const int ylo = max(max(iy, jy) - P, 0), yhi = min(min(iy, jy), nely - 1);
      const int xlo = max(max(ix, jx) - P, 0), xhi = min(min(ix, jx), nelx - 1);
      for (int ez = zlo; ez <= zhi; ++ez)
        for (int ey = ylo; ey <= yhi; ++ey)
          for (int ex = xlo; ex <= xhi; ++ex) {
            const int a = ((iz - ez) * P1 + iy - ey) * P1 + ix - ex;
            const int b = ((jz - ez) * P1 + jy - ey) * P1 + jx - ex;
            const long long le = ((long long)(ez - ez0) * nely + ey) * nelx + ex;
            sum += Ke[le * NB * NB + a * NB + b];
          }
    }
  }
  st[t * SP + o] = sum;
}

// Stencil rows of the 2D volume stiffness on an RT x RT tile of rows by sum
// factorization, one element row at a time: for element row ey the metric
// at its Gauss points is evaluated once (as in the operator kernel), the
// x-direction is contracted into X_k[qy][row x][dx] for the four products
// of values/derivatives (g00 D D, g01 D B, g01 B D, g11 B B), and the
// y-direction accumulates into the rows' (2p+1)^2 entries held in registers.
template <int P, int RT>
__global__ __launch_bounds__(256) void stencil2d_kernel(const VolTile *tiles, const PatchDev *pd,
                                                        const double *tabB, const double *tabD,
                                                        GaussRule gr, double *st, int SP, int pm) {
  // Rows are laid out for the level's largest degree pm >= P: entry (dx, dy)
  // of this patch's (2P+1)^2 stencil sits at slot (dy + pm - P)(2pm + 1) +
  // dx + pm - P of a row of stride SP; every other slot is zero
  constexpr int Q = P + 1, P1 = P + 1, S1 = 2 * P + 1, S = S1 * S1;
  constexpr int NE = RT + P;                  // element columns touching the tile
  constexpr int NOUT = RT * RT * S;           // entries of the tile's rows
  constexpr int OPT = (NOUT + 255) / 256;     // entries per thread
  constexpr int NX = Q * RT * S1;             // stage-1 items per term
  __shared__ double sG[3][NE * Q][Q];         // metric of element row ey
  __shared__ double sX[4][Q][RT][S1];         // x-contracted products
  __shared__ double sBx[NE * Q][P1], sDx[NE * Q][P1], sBy[Q][P1], sDy[Q][P1];
  __shared__ double sC[4][3];
  const VolTile tl = tiles[blockIdx.x];
  const PatchDev &pt = pd[tl.patch];
  const int tid = threadIdx.x;
  const int x0 = tl.e0[0], y0 = tl.e0[1];     // first row of the tile (unknown indices)
  const int nx = pt.n[0], ny = pt.n[1], nelx = pt.nel[0], nely = pt.nel[1];
  const int ex0 = max(0, x0 - P), ex1 = min(nelx - 1, x0 + RT - 1);
  const int ey0 = max(0, y0 - P), ey1 = min(nely - 1, y0 + RT - 1);
  const double hx = 1.0 / nelx, hy = 1.0 / nely;
  if (tid < 12) sC[tid / 3][tid % 3] = pt.corners[tid / 3][tid % 3];
  for (int e = tid; e < NE * Q * P1; e += 256) {
    const int r = e / P1, a = e % P1;
    const int ex = ex0 + r / Q;
    const bool ok = ex <= ex1;
    const size_t row = (size_t)pt.tab[0] + ((size_t)ex * Q + r % Q) * P1 + a;
    sBx[r][a] = ok ? tabB[row] : 0.0;
    sDx[r][a] = ok ? tabD[row] : 0.0;
  }
  double acc[OPT];
#pragma unroll
  for (int u = 0; u < OPT; ++u) acc[u] = 0.0;
  for (int ey = ey0; ey <= ey1; ++ey) {
    __syncthreads();
    // metric at the Gauss points of element row ey, y tables of ey
    for (int e = tid; e < NE * Q * Q; e += 256) {
      const int c = e / Q, qy = e % Q;
      const int ex = ex0 + c / Q, qx = c % Q;
      double g00 = 0.0, g01 = 0.0, g11 = 0.0;
      if (ex <= ex1) {
        const double xe = ((double)ex + gr.x[qx]) * hx;
        const double ye = ((double)ey + gr.x[qy]) * hy;
        const double j00 = (1.0 - ye) * (sC[1][0] - sC[0][0]) + ye * (sC[3][0] - sC[2][0]);
        const double j10 = (1.0 - ye) * (sC[1][1] - sC[0][1]) + ye * (sC[3][1] - sC[2][1]);
        const double j01 = (1.0 - xe) * (sC[2][0] - sC[0][0]) + xe * (sC[3][0] - sC[1][0]);
        const double j11 = (1.0 - xe) * (sC[2][1] - sC[0][1]) + xe * (sC[3][1] - sC[1][1]);
        const double det = j00 * j11 - j01 * j10;
        const double sc = gr.w[qx] * hx * gr.w[qy] * hy / fabs(det);
        g00 = sc * (j11 * j11 + j01 * j01);
        g01 = -sc * (j11 * j10 + j01 * j00);
        g11 = sc * (j10 * j10 + j00 * j00);
      }
      sG[0][c][qy] = g00;
      sG[1][c][qy] = g01;
      sG[2][c][qy] = g11;
    }
    for (int e = tid; e < Q * P1; e += 256) {
      const size_t row = (size_t)pt.tab[1] + ((size_t)ey * Q + e / P1) * P1 + e % P1;
      sBy[e / P1][e % P1] = tabB[row];
      sDy[e / P1][e % P1] = tabD[row];
    }
    __syncthreads();
    // stage 1: X_k[qy][rx][dx] = sum over elements ex of both supports and qx
    for (int e = tid; e < NX; e += 256) {
      const int qy = e / (RT * S1), rem = e % (RT * S1), rx = rem / S1, dxi = rem % S1;
      const int ix = x0 + rx, jx = ix + dxi - P;
      double x00 = 0.0, x01 = 0.0, x10 = 0.0, x11 = 0.0;
      if (ix < nx && jx >= 0 && jx < nx) {
        const int elo = max(max(ix, jx) - P, ex0), ehi = min(min(ix, jx), ex1);
        for (int ex = elo; ex <= ehi; ++ex) {
          const int c0 = (ex - ex0) * Q;
#pragma unroll
          for (int qx = 0; qx < Q; ++qx) {
            const double bi = sBx[c0 + qx][ix - ex], di = sDx[c0 + qx][ix - ex];
            const double bj = sBx[c0 + qx][jx - ex], dj = sDx[c0 + qx][jx - ex];
            const double g00 = sG[0][c0 + qx][qy], g01 = sG[1][c0 + qx][qy];
            const double g11 = sG[2][c0 + qx][qy];
            x00 += g00 * di * dj;
            x01 += g01 * di * bj;
            x10 += g01 * bi * dj;
            x11 += g11 * bi * bj;
          }
        }
      }
      sX[0][qy][rx][dxi] = x00;
      sX[1][qy][rx][dxi] = x01;
      sX[2][qy][rx][dxi] = x10;
      sX[3][qy][rx][dxi] = x11;
    }
    __syncthreads();
    // stage 2: entries (ry, dy, rx, dx) of rows whose y-support holds ey
#pragma unroll
    for (int u = 0; u < OPT; ++u) {
      const int o = tid + 256 * u;
      if (o >= NOUT) continue;
      const int ry = o / (RT * S), rem = o % (RT * S), rx = rem / S, slot = rem % S;
      const int dyi = slot / S1, dxi = slot % S1;
      const int iy = y0 + ry, jy = iy + dyi - P;
      if (iy >= ny || jy < 0 || jy >= ny) continue;
      if (ey < max(iy, jy) - P || ey > min(iy, jy)) continue;
      const int ai = iy - ey, aj = jy - ey;
      double s = 0.0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        const double bi = sBy[qy][ai], di = sDy[qy][ai], bj = sBy[qy][aj], dj = sDy[qy][aj];
        s += sX[0][qy][rx][dxi] * bi * bj + sX[1][qy][rx][dxi] * bi * dj +
             sX[2][qy][rx][dxi] * di * bj + sX[3][qy][rx][dxi] * di * dj;
      }
      acc[u] += s;
    }
  }
  // rows of the tile in the level's layout; the other slots zero
  const int S1m = 2 * pm + 1, sh = pm - P;
#pragma unroll
  for (int u = 0; u < OPT; ++u) {
    const int o = tid + 256 * u;
    if (o >= NOUT) continue;
    const int ry = o / (RT * S), rem = o % (RT * S), rx = rem / S, slot = rem % S;
    const int ix = x0 + rx, iy = y0 + ry;
    if (ix >= nx || iy >= ny) continue;
    const int so = (slot / S1 + sh) * S1m + slot % S1 + sh;
    st[(pt.off + (long long)iy * nx + ix) * SP + so] = acc[u];
  }
  for (int e = tid; e < RT * RT * SP; e += 256) {
    const int r = e / SP, so = e % SP;
    const int dy = so / S1m - sh, dx = so % S1m - sh;
    if (so < S1m * S1m && dy >= 0 && dy < S1 && dx >= 0 && dx < S1) continue;  // an entry
    const int ix = x0 + r % RT, iy = y0 + r / RT;
    if (ix < nx && iy < ny) st[(pt.off + (long long)iy * nx + ix) * SP + so] = 0.0;
  }
}

__global__ void stencil_add_kernel(const int *rows, const int *slots, const double *vals, int n,
                                   double *st, int S) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) st[(long long)rows[i] * S + slots[i]] += vals[i];
}

__global__ void invdiag_kernel(const double *st, int S, int center, const unsigned char *mask,
                               double *invd, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) invd[i] = mask[i] ? 1.0 / st[i * S + center] : 0.0;
}

// (f, phi_i) for f = d pi^2 prod sin(pi x), gather over the support of phi_i
// Squared L2 error of u_h (torn coefficients) against prod sin(pi x) on
// element t: qe-point Gauss rule per direction, 1D tables of all basis values
// at those points (tab: offset of the element count's table per patch and
// direction, rows [e][g][a]).  el_off: first element of each patch.
template <int D>
__device__ double l2err_element(const PatchDev *pd, int K, const long long *el_off,
                                const int *tab, const double *tB, GaussRule gq, int p,
                                const double *ut, long long t) {
  int k = 0;
  while (k + 1 < K && el_off[k + 1] <= t) ++k;
  const PatchDev &pt = pd[k];
  long long loc = t - el_off[k];
  int e[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    e[d] = (int)(loc % pt.nel[d]);
    loc /= pt.nel[d];
  }
  const int q = gq.q, P1 = pt.p + 1;  // the patch's degree (p: unused, the largest)
  (void)p;
  double sum = 0.0;
  int g[3] = {0, 0, 0};
  for (;;) {
    double xh[D], w = 1.0;
    const double *row[3];
    for (int d = 0; d < D; ++d) {
      xh[d] = ((double)e[d] + gq.x[g[d]]) / (double)pt.nel[d];
      w *= gq.w[g[d]] / (double)pt.nel[d];
      row[d] = tB + (size_t)tab[k * 3 + d] + ((size_t)e[d] * q + g[d]) * P1;
    }
    double uh = 0.0;
    int a[3] = {0, 0, 0};
    for (;;) {
      double phi = 1.0;
      long long idx = pt.off;
      for (int d = 0; d < D; ++d) {
        phi *= row[d][a[d]];
        idx += (long long)(e[d] + a[d]) * pt.stride[d];
      }
      uh += phi * ut[idx];
      int d = 0;
      while (d < D && ++a[d] == P1) a[d++] = 0;
      if (d == D) break;
    }
    double J[D][D], Ji[D][D], X[D];
    multilinear_jac<D>(pt.corners, xh, J);
    const double det = inverse<D>(J, Ji);
    multilinear_map<D>(pt.corners, xh, X);
    double ex = 1.0;
    for (int d = 0; d < D; ++d) ex *= sin(M_PI * X[d]);
    sum += w * (det < 0 ? -det : det) * (uh - ex) * (uh - ex);
    int d = 0;
    while (d < D && ++g[d] == q) g[d++] = 0;
    if (d == D) break;
  }
  return sum;
}

// Each block sums its elements' contributions by a fixed tree and writes one
// partial (part[blockIdx.x]).
template <int D>
__global__ __launch_bounds__(256) void l2err_kernel(const PatchDev *pd, int K,
                                                    const long long *el_off, const int *tab,
                                                    const double *tB, GaussRule gq, int p,
                                                    const double *ut, double *part) {
  __shared__ double sp[256];
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const double sum = t < el_off[K] ? l2err_element<D>(pd, K, el_off, tab, tB, gq, p, ut, t) : 0.0;
  sp[threadIdx.x] = sum;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sp[threadIdx.x] += sp[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sp[0];
}

// sum of n values by one block in a fixed order (strided partial sums, then a
// tree over the 1024 partials)
__global__ __launch_bounds__(1024) void sum_fixed_kernel(const double *x, long long n,
                                                         double *out) {
  __shared__ double sp[1024];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) s += x[i];
  sp[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sp[threadIdx.x] += sp[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sp[0];
}

template <int D>
__global__ void load_kernel(const PatchDev *pd, int K, const double *tabB,
                            const GaussRule *rules, const unsigned char *mask, long long ntorn,
                            double *out) {
  long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= ntorn) return;
  int k = 0;
  while (k + 1 < K && pd[k + 1].off <= t) ++k;
  const PatchDev &pt = pd[k];
  // the patch's degree p and its (p+1)-point rule (the tables' rule)
  const int p = pt.p;
  const GaussRule &gr = rules[p + 1];
  long long loc = t - pt.off;
  int i[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    i[d] = (int)(loc % pt.n[d]);
    loc /= pt.n[d];
    lo[d] = i[d] - p < 0 ? 0 : i[d] - p;
    hi[d] = i[d] > pt.nel[d] - 1 ? pt.nel[d] - 1 : i[d];
  }
  if (!mask[t]) {
    out[t] = 0.0;
    return;
  }
  const int q = gr.q, P1 = p + 1;
  double sum = 0.0;
  int e[3] = {lo[0], lo[1], lo[2]};
  for (;;) {
    int g[3] = {0, 0, 0};
    for (;;) {
      double xh[D], w = 1.0, phi = 1.0;
      for (int d = 0; d < D; ++d) {
        xh[d] = ((double)e[d] + gr.x[g[d]]) / (double)pt.nel[d];
        w *= gr.w[g[d]] / (double)pt.nel[d];
        phi *= tabB[(size_t)pt.tab[d] + ((size_t)e[d] * q + g[d]) * P1 + (i[d] - e[d])];
      }
      double J[D][D], Ji[D][D], X[D];
      multilinear_jac<D>(pt.corners, xh, J);
      double det = inverse<D>(J, Ji);
      multilinear_map<D>(pt.corners, xh, X);
      double fx = D * M_PI * M_PI;
      for (int d = 0; d < D; ++d) fx *= sin(M_PI * X[d]);
      sum += w * (det < 0 ? -det : det) * fx * phi;
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
  out[t] = sum;
}

// ---------------------------------------------------------------------------
// interface terms: r = mask (beta fw.*f + alpha A_if u).  Blocks below nb_plain
// handle unknowns without interface couplings (one thread each); the others
// give 16 lanes to each unknown next to an interface.  grid.x = right-hand
// side (fastest, so that the right-hand sides of a row block share its
// operator data in cache), grid.y = row block.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void iface_kernel(long long n, int nb_plain,
                                                    const unsigned char *__restrict__ mask,
                                                    const unsigned char *__restrict__ has_if,
                                                    const int *__restrict__ rows, int nrows,
                                                    const int *__restrict__ ptr,
                                                    const int *__restrict__ col,
                                                    const T *__restrict__ val,
                                                    const T *__restrict__ u,
                                                    const T *__restrict__ f,
                                                    const T *__restrict__ fw, T beta, T alpha,
                                                    T *__restrict__ r) {
  const long long zo = (long long)blockIdx.x * n;
  u += zo;
  r += zo;
  if (f) f += zo;
  if ((int)blockIdx.y < nb_plain) {
    long long t = blockIdx.y * (long long)blockDim.x + threadIdx.x;
    if (t >= n || has_if[t]) return;
    T v = 0;
    if (mask[t] && f) v = beta * (fw ? fw[t] : (T)1) * f[t];
    r[t] = v;
    return;
  }
  const int g = ((int)blockIdx.y - nb_plain) * (blockDim.x / 16) + threadIdx.x / 16;
  const int lane = threadIdx.x % 16;
  const bool ok = g < nrows;
  const int t = ok ? rows[g] : 0;
  T s = 0;
  if (ok)
    for (int e = ptr[t] + lane; e < ptr[t + 1]; e += 16) s += val[e] * u[col[e]];
  s = row16_scan(s);
  if (ok && lane == 15) {
    T v = alpha * s;
    if (f) v += beta * (fw ? fw[t] : (T)1) * f[t];
    r[t] = v;
  }
}

// ---------------------------------------------------------------------------
// volume operator, 2D, sum factorization on a TE x TE element tile:
// r += alpha * A_vol u.  The tiles of one launch form one colour class whose
// output windows (TE + P unknowns per direction) do not overlap, so every
// output is read, added to and written by one thread, and the classes follow
// each other in a fixed order: the sums do not depend on scheduling.  The
// geometry (metric) is evaluated in float64 and rounded to T.
// grid.x = right-hand side (the batch shares the tile's tables in cache),
// grid.y = tile.
// ---------------------------------------------------------------------------
template <typename T, int P, int TE, int RC>
__global__ __launch_bounds__(256) void vol2d_kernel(const OpTile2 *tiles,
                                                    const double *tabB, const double *tabD,
                                                    GaussRule gr, const T *__restrict__ u,
                                                    T *__restrict__ r,
                                                    const unsigned char *__restrict__ mask,
                                                    T alpha, long long vs, int nrhs) {
  constexpr int Q = P + 1, P1 = P + 1;
  constexpr int ND = TE + P;   // unknowns per direction touched by the tile
  constexpr int NQ = TE * Q;   // Gauss points per direction in the tile
  constexpr int NG = RC > 1 ? NQ * NQ : 1;
  __shared__ T sU[ND * ND];
  __shared__ T sA0[ND * NQ], sA1[ND * NQ];
  __shared__ T sV0[NQ * NQ], sV1[NQ * NQ];
  __shared__ T sBx[NQ * P1], sDx[NQ * P1], sBy[NQ * P1], sDy[NQ * P1];
  __shared__ T sG[3][NG];  // metric at the tile's Gauss points (batches only)
  __shared__ double sC[4][2];
  const OpTile2 tl = tiles[blockIdx.y];
  const int tid = threadIdx.x;
  const int ex0 = tl.e0[0], ey0 = tl.e0[1];
  const int nex = min(TE, tl.nel[0] - ex0), ney = min(TE, tl.nel[1] - ey0);
  const int nx = tl.nx;
  const long long off = tl.off;
  // corners read through the record (a lane-indexed copy would live in scratch)
  if (tid < 8) sC[tid / 2][tid % 2] = tiles[blockIdx.y].corners[tid / 2][tid % 2];
  for (int i = tid; i < NQ * P1; i += blockDim.x) {
    int gq = i / P1;
    bool okx = gq < nex * Q, oky = gq < ney * Q;
    sBx[i] = okx ? (T)tabB[tl.tab[0] + (size_t)ex0 * Q * P1 + i] : (T)0;
    sDx[i] = okx ? (T)tabD[tl.tab[0] + (size_t)ex0 * Q * P1 + i] : (T)0;
    sBy[i] = oky ? (T)tabB[tl.tab[1] + (size_t)ey0 * Q * P1 + i] : (T)0;
    sDy[i] = oky ? (T)tabD[tl.tab[1] + (size_t)ey0 * Q * P1 + i] : (T)0;
  }
  const double hx = 1.0 / tl.nel[0], hy = 1.0 / tl.nel[1];
  // metric w |det J| J^-1 J^-T = (w / |det J|) adj(J) adj(J)^T at Gauss point
  // (gx, gy) of the tile: one division
  auto metric = [&](int gx, int gy, T &g00, T &g01, T &g11) {
    const int ex = gx / Q, ey = gy / Q;
    const int qx = gx - ex * Q, qy = gy - ey * Q;
    const double xe = ((double)(ex0 + ex) + gr.x[qx]) * hx;
    const double ye = ((double)(ey0 + ey) + gr.x[qy]) * hy;
    const double j00 = (1.0 - ye) * (sC[1][0] - sC[0][0]) + ye * (sC[3][0] - sC[2][0]);
    const double j10 = (1.0 - ye) * (sC[1][1] - sC[0][1]) + ye * (sC[3][1] - sC[2][1]);
    const double j01 = (1.0 - xe) * (sC[2][0] - sC[0][0]) + xe * (sC[3][0] - sC[1][0]);
    const double j11 = (1.0 - xe) * (sC[2][1] - sC[0][1]) + xe * (sC[3][1] - sC[1][1]);
    const double det = j00 * j11 - j01 * j10;
    const double sc = gr.w[qx] * hx * gr.w[qy] * hy / fabs(det);
    g00 = (T)(sc * (j11 * j11 + j01 * j01));
    g01 = (T)(-sc * (j11 * j10 + j01 * j00));
    g11 = (T)(sc * (j10 * j10 + j00 * j00));
  };
  if (RC > 1) {
    __syncthreads();  // corners
    for (int i = tid; i < NQ * NQ; i += blockDim.x) {
      T g00 = 0, g01 = 0, g11 = 0;
      if (i / NQ < ney * Q && i % NQ < nex * Q) metric(i % NQ, i / NQ, g00, g01, g11);
      sG[0][i % NG] = g00;
      sG[1][i % NG] = g01;
      sG[2][i % NG] = g11;
    }
  }
  // the right-hand sides of this block share the tables and the metric
  const int z0 = blockIdx.x * RC, z1 = min(nrhs, z0 + RC);  // RC = 1: z0 = blockIdx.x
  for (int z = z0; z < z1; ++z) {
    const T *uz = u + (long long)z * vs;
    T *rz = r + (long long)z * vs;
    if (z > z0) __syncthreads();  // previous right-hand side done with the LDS arrays
    for (int i = tid; i < ND * ND; i += blockDim.x) {
      int rr = i / ND, cc = i % ND;
      sU[i] = (rr < ney + P && cc < nex + P) ? uz[off + (long long)(ey0 + rr) * nx + ex0 + cc] : (T)0;
    }
    __syncthreads();
    // x-contraction: A0 = values, A1 = derivatives, rows = unknown rows
    for (int i = tid; i < ND * NQ; i += blockDim.x) {
      int rr = i / NQ, gx = i % NQ;
      int e = gx / Q;
      T a0 = 0, a1 = 0;
#pragma unroll
      for (int a = 0; a < P1; ++a) {
        T uv = sU[rr * ND + e + a];
        a0 += sBx[gx * P1 + a] * uv;
        a1 += sDx[gx * P1 + a] * uv;
      }
      sA0[i] = a0;
      sA1[i] = a1;
    }
    __syncthreads();
    // y-contraction + metric at the Gauss points
    for (int i = tid; i < NQ * NQ; i += blockDim.x) {
      int gy = i / NQ, gx = i % NQ;
      T v0 = 0, v1 = 0;
      if (gy < ney * Q && gx < nex * Q) {
        int ey = gy / Q;
        T ux = 0, uy = 0;
#pragma unroll
        for (int b = 0; b < P1; ++b) {
          ux += sBy[gy * P1 + b] * sA1[(ey + b) * NQ + gx];
          uy += sDy[gy * P1 + b] * sA0[(ey + b) * NQ + gx];
        }
        T g00, g01, g11;
        if (RC > 1) {
          g00 = sG[0][i % NG];
          g01 = sG[1][i % NG];
          g11 = sG[2][i % NG];
        } else {
          metric(gx, gy, g00, g01, g11);
        }
        v0 = g00 * ux + g01 * uy;
        v1 = g01 * ux + g11 * uy;
      }
      sV0[i] = v0;
      sV1[i] = v1;
    }
    __syncthreads();
    // transposed y-contraction: rows = output unknown rows
    for (int i = tid; i < ND * NQ; i += blockDim.x) {
      int rr = i / NQ, gx = i % NQ;
      T s1 = 0, s0 = 0;
      int elo = max(0, rr - P), ehi = min(ney - 1, rr);
      for (int e = elo; e <= ehi; ++e) {
        int a = rr - e;
#pragma unroll
        for (int g = 0; g < Q; ++g) {
          int gy = e * Q + g;
          s1 += sBy[gy * P1 + a] * sV0[gy * NQ + gx];
          s0 += sDy[gy * P1 + a] * sV1[gy * NQ + gx];
        }
      }
      sA1[i] = s1;
      sA0[i] = s0;
    }
    __syncthreads();
    // transposed x-contraction and accumulation
    for (int i = tid; i < ND * ND; i += blockDim.x) {
      int rr = i / ND, cc = i % ND;
      if (rr >= ney + P || cc >= nex + P) continue;
      T y = 0;
      int elo = max(0, cc - P), ehi = min(nex - 1, cc);
      for (int e = elo; e <= ehi; ++e) {
        int a = cc - e;
#pragma unroll
        for (int g = 0; g < Q; ++g) {
          int gx = e * Q + g;
          y += sDx[gx * P1 + a] * sA1[rr * NQ + gx] + sBx[gx * P1 + a] * sA0[rr * NQ + gx];
        }
      }
      long long t = off + (long long)(ey0 + rr) * nx + ex0 + cc;
      if (mask[t]) rz[t] += alpha * y;
    }
  }
}

// ---------------------------------------------------------------------------
// volume operator, 3D, sum factorization on a TE^3 element tile:
// r += alpha * A_vol u, one colour class of tiles with disjoint output
// windows per launch (as in 2D: a fixed order of the sums).  Stages
// (all in LDS): x-, y-, z-contractions of the u window with the value and
// derivative tables give the parameter gradient at the tile's Gauss points;
// the metric w |det J| J^-1 J^-T (float64 from the trilinear corners, rounded
// to T) multiplies it; the transposed z-, y-, x-contractions return to the
// unknowns.  grid.x = tile, grid.y = right-hand side.
// ---------------------------------------------------------------------------
template <typename T, int P, int TE>
__global__ __launch_bounds__(256) void vol3d_kernel(const VolTile *tiles, const PatchDev *pd,
                                                    const double *tabB, const double *tabD,
                                                    GaussRule gr, const T *__restrict__ u,
                                                    T *__restrict__ r,
                                                    const unsigned char *__restrict__ mask,
                                                    T alpha, long long vs) {
  constexpr int Q = P + 1, P1 = P + 1, ND = TE + P, NQ = TE * Q;
  constexpr int N2 = ND * ND, NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
  __shared__ T sU[ND * N2];         // u window [z][y][x]
  __shared__ T sA[2][N2 * NQ];      // [rz][ry][gx]
  __shared__ T sB[3][ND * NQ2];     // [rz][gy][gx]
  __shared__ T sV[3][NQ3];          // [gz][gy][gx]
  __shared__ T sTB[3][NQ][P1], sTD[3][NQ][P1];
  __shared__ double sC[8][3];
  const VolTile tl = tiles[blockIdx.x];
  const PatchDev &pt = pd[tl.patch];
  const int tid = threadIdx.x;
  const long long zo = (long long)blockIdx.y * vs;
  u += zo;
  r += zo;
  int ne[3], nel[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    nel[g] = pt.nel[g];
    ne[g] = min(TE, nel[g] - tl.e0[g]);
  }
  const int nx = pt.n[0], ny = pt.n[1];
  const long long off = pt.off;
  if (tid < 24) sC[tid / 3][tid % 3] = pt.corners[tid / 3][tid % 3];
  for (int i = tid; i < 3 * NQ * P1; i += 256) {
    // per-direction fields selected without indexing by a lane value
    const int g = i / (NQ * P1), gq = i / P1 % NQ, a = i % P1;
    const int neg = g == 0 ? ne[0] : (g == 1 ? ne[1] : ne[2]);
    const int e0g = g == 0 ? tl.e0[0] : (g == 1 ? tl.e0[1] : tl.e0[2]);
    const int tabg = g == 0 ? pt.tab[0] : (g == 1 ? pt.tab[1] : pt.tab[2]);
    const bool ok = gq < neg * Q;
    const size_t row = (size_t)tabg + ((size_t)e0g * Q + gq) * P1 + a;
    sTB[g][gq][a] = ok ? (T)tabB[row] : (T)0;
    sTD[g][gq][a] = ok ? (T)tabD[row] : (T)0;
  }
  for (int i = tid; i < ND * N2; i += 256) {
    const int rz = i / N2, ry = i / ND % ND, rx = i % ND;
    const bool ok = rz < ne[2] + P && ry < ne[1] + P && rx < ne[0] + P;
    sU[i] = ok ? u[off + ((long long)(tl.e0[2] + rz) * ny + tl.e0[1] + ry) * nx + tl.e0[0] + rx]
               : (T)0;
  }
  __syncthreads();
  // x: A0 = values, A1 = derivatives
  for (int i = tid; i < N2 * NQ; i += 256) {
    const int rzy = i / NQ, gx = i % NQ, ex = gx / Q;
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int a = 0; a < P1; ++a) {
      const T uv = sU[rzy * ND + ex + a];
      a0 += sTB[0][gx][a] * uv;
      a1 += sTD[0][gx][a] * uv;
    }
    sA[0][i] = a0;
    sA[1][i] = a1;
  }
  __syncthreads();
  // y: B0 = (val, val), B1 = (val, d), B2 = (d, val)
  for (int i = tid; i < ND * NQ2; i += 256) {
    const int rz = i / NQ2, gy = i / NQ % NQ, gx = i % NQ, ey = gy / Q;
    T b0 = 0, b1 = 0, b2 = 0;
#pragma unroll
    for (int b = 0; b < P1; ++b) {
      const int j = (rz * ND + ey + b) * NQ + gx;
      b0 += sTB[1][gy][b] * sA[0][j];
      b1 += sTD[1][gy][b] * sA[0][j];
      b2 += sTB[1][gy][b] * sA[1][j];
    }
    sB[0][i] = b0;
    sB[1][i] = b1;
    sB[2][i] = b2;
  }
  __syncthreads();
  // z: parameter gradient at the Gauss points, times the metric
  for (int i = tid; i < NQ3; i += 256) {
    const int gz = i / NQ2, gy = i / NQ % NQ, gx = i % NQ, ez = gz / Q;
    T v0 = 0, v1 = 0, v2 = 0;
    if (gx < ne[0] * Q && gy < ne[1] * Q && gz < ne[2] * Q) {
      T ux = 0, uy = 0, uz = 0;
#pragma unroll
      for (int c = 0; c < P1; ++c) {
        const int j = ((ez + c) * NQ + gy) * NQ + gx;
        ux += sTB[2][gz][c] * sB[2][j];
        uy += sTB[2][gz][c] * sB[1][j];
        uz += sTD[2][gz][c] * sB[0][j];
      }
      const int gq[3] = {gx, gy, gz};
      double xh[3], w = 1.0;
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        const int e = gq[g] / Q, q = gq[g] - e * Q;
        // Gauss node and weight selected without indexing by a lane value
        double xq = gr.x[0], wq = gr.w[0];
#pragma unroll
        for (int m = 1; m < Q; ++m)
          if (q == m) {
            xq = gr.x[m];
            wq = gr.w[m];
          }
        xh[g] = ((double)(tl.e0[g] + e) + xq) / (double)nel[g];
        w *= wq / (double)nel[g];
      }
      double G[3][3];
      metric<3>(sC, xh, w, G);
      v0 = (T)G[0][0] * ux + (T)G[0][1] * uy + (T)G[0][2] * uz;
      v1 = (T)G[1][0] * ux + (T)G[1][1] * uy + (T)G[1][2] * uz;
      v2 = (T)G[2][0] * ux + (T)G[2][1] * uy + (T)G[2][2] * uz;
    }
    sV[0][i] = v0;
    sV[1][i] = v1;
    sV[2][i] = v2;
  }
  __syncthreads();
  // transposed z (into sB): C0 -> (Dx, By), C1 -> (Bx, Dy), C2 -> (Bx, By)
  for (int i = tid; i < ND * NQ2; i += 256) {
    const int rz = i / NQ2, gyx = i % NQ2;
    T c0 = 0, c1 = 0, c2 = 0;
    const int elo = max(0, rz - P), ehi = min(ne[2] - 1, rz);
    for (int e = elo; e <= ehi; ++e) {
      const int a = rz - e;
#pragma unroll
      for (int g = 0; g < Q; ++g) {
        const int gz = e * Q + g, j = gz * NQ2 + gyx;
        c0 += sTB[2][gz][a] * sV[0][j];
        c1 += sTB[2][gz][a] * sV[1][j];
        c2 += sTD[2][gz][a] * sV[2][j];
      }
    }
    sB[0][i] = c0;
    sB[1][i] = c1;
    sB[2][i] = c2;
  }
  __syncthreads();
  // transposed y (into sA): E0 -> Dx, E1 -> Bx
  for (int i = tid; i < N2 * NQ; i += 256) {
    const int rz = i / (ND * NQ), ry = i / NQ % ND, gx = i % NQ;
    T e0 = 0, e1 = 0;
    const int elo = max(0, ry - P), ehi = min(ne[1] - 1, ry);
    for (int e = elo; e <= ehi; ++e) {
      const int a = ry - e;
#pragma unroll
      for (int g = 0; g < Q; ++g) {
        const int gy = e * Q + g, j = (rz * NQ + gy) * NQ + gx;
        e0 += sTB[1][gy][a] * sB[0][j];
        e1 += sTD[1][gy][a] * sB[1][j] + sTB[1][gy][a] * sB[2][j];
      }
    }
    sA[0][i] = e0;
    sA[1][i] = e1;
  }
  __syncthreads();
  // transposed x and accumulation
  for (int i = tid; i < ND * N2; i += 256) {
    const int rz = i / N2, ry = i / ND % ND, rx = i % ND;
    if (rz >= ne[2] + P || ry >= ne[1] + P || rx >= ne[0] + P) continue;
    T y = 0;
    const int elo = max(0, rx - P), ehi = min(ne[0] - 1, rx);
    for (int e = elo; e <= ehi; ++e) {
      const int a = rx - e;
#pragma unroll
      for (int g = 0; g < Q; ++g) {
        const int gx = e * Q + g, j = (rz * ND + ry) * NQ + gx;
        y += sTD[0][gx][a] * sA[0][j] + sTB[0][gx][a] * sA[1][j];
      }
    }
    const long long t = off + ((long long)(tl.e0[2] + rz) * ny + tl.e0[1] + ry) * nx + tl.e0[0] + rx;
    if (mask[t]) r[t] += alpha * y;
  }
}

// ---------------------------------------------------------------------------
// glue (conforming): y <- sum of copies on every copy; grid.y = right-hand side
// ---------------------------------------------------------------------------
template <typename T>
__global__ void glue_kernel(int ng, const int *ptr, const int *idx, T *y, long long vs) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  y += (long long)blockIdx.y * vs;
  T s = 0;
  for (int e = ptr[g]; e < ptr[g + 1]; ++e) s += y[idx[e]];
  for (int e = ptr[g]; e < ptr[g + 1]; ++e) y[idx[e]] = s;
}

// Conforming Gauss-Seidel levels: a distributed right-hand side gathered on
// the first copy of every glued unknown (the row the sweep updates); the
// other copies become 0, so the copies' sum, and with it the distributed
// form the residuals assume, is unchanged.  Fixed summation order.
template <typename T>
__global__ void glue_first_kernel(int ng, const int *ptr, const int *idx, T *y, long long vs) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  y += (long long)blockIdx.y * vs;
  T s = 0;
  for (int e = ptr[g]; e < ptr[g + 1]; ++e) s += y[idx[e]];
  y[idx[ptr[g]]] = s;
  for (int e = ptr[g] + 1; e < ptr[g + 1]; ++e) y[idx[e]] = (T)0;
}

// ---------------------------------------------------------------------------
// Cross-patch couplings of a Gauss-Seidel tile: sum_j a_ij u_j over the
// neighbouring patches' columns for every coupled row of the tile, in the
// slot layout of GsTile.  Every lane sums its slot's entries in order; the
// first lane of each row adds the sums of the row's slots in lane order
// (register shuffles) and hands the total to `apply(row, totals)` -- one
// call per row, so no two lanes update one row and the sums do not depend on
// scheduling.  NR right-hand sides (uz[r]) share the entry loads.  Called by
// all 64 lanes of a wavefront.
// ---------------------------------------------------------------------------
template <typename T, int NR, typename Apply>
__device__ __forceinline__ void tile_cross(const GsTile &tl, const int *__restrict__ slots,
                                           const int *__restrict__ cols,
                                           const T *__restrict__ vals, const T *const *uz,
                                           int lane, Apply apply) {
  for (int q = 0; q < tl.cx_np; ++q) {
    const int code = slots[tl.cx_sl + 64 * q + lane];
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = (T)0;
    const long long base = tl.cx_off + (long long)q * tl.cx_k * 64 + lane;
    for (int k0 = 0; k0 < tl.cx_k; k0 += 8) {
      int cc[8];
      T cv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = k0 + j < tl.cx_k;
        cc[j] = ok ? cols[base + 64 * (k0 + j)] : -1;
        cv[j] = ok ? vals[base + 64 * (k0 + j)] : (T)0;
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        T cu[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) cu[j] = cc[j] >= 0 ? uz[r][cc[j]] : (T)0;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[r] += cv[j] * cu[j];
      }
    }
    const int ns = (code >= 0 && ((code >> 16) & 0xff) == 0) ? code >> 24 : 0;
    T tot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tot[r] = (T)0;
    for (int s = 0; s < tl.cx_r; ++s) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const T v = __shfl(acc[r], (lane + s) & 63);
        if (s < ns) tot[r] += v;
      }
    }
    if (ns > 0) apply(code & 0xffff, tot);
  }
}

// Row stride of a Gauss-Seidel tile's u window in LDS by degree: the stride
// in [w, w + 64) that minimizes the LDS cycles of a chunk read (32 banks, 32
// lanes per cycle: the two row groups p+1 columns apart in a half-wavefront,
// each reading 16 consecutive stencil slots), from an enumeration of the
// strides; for p = 6, 52 takes 24 cycles per row where the unpadded 26 takes
// 44 (22 without conflicts).  0: unpadded.
__host__ __device__ constexpr int gs_window_stride(int p) {
  constexpr int tab[9] = {0, 0, 12, 43, 46, 51, 52, 55, 0};
  return p >= 0 && p <= 8 ? tab[p] : 0;
}

// ---------------------------------------------------------------------------
// Multicolour Gauss-Seidel, one wavefront per tile of 2(p+1) x 2(p+1)
// unknowns: the four unknowns of a colour class inside the tile are updated
// by four groups of 16 lanes; the row sum of each group comes out of a DPP
// scan in its last lane.  The u window's row stride in LDS is padded
// (gs_window_stride) so that the two groups of a half-wavefront, p+1
// columns apart, read nearly disjoint banks.  A single wavefront executes its LDS operations in
// program order, so a class reads what the previous class wrote without a
// barrier.  Stencil rows (padded to 16-lane groups) of the next D classes are
// prefetched into registers; f minus the cross-patch couplings (neighbouring
// patches carry another patch colour, so their values are constant during the
// launch) and 1/a_ii sit in LDS as one pair per unknown.
// A wavefront sweeps NR right-hand sides of a batch through its tile at once:
// every stencil row it loads serves the NR of them (their dot products and
// scans are independent, so they also overlap each other's latency).  A
// block holds RBW such wavefronts on the same tile, whose row loads meet in
// the CU's L1.  Blocks: (tile, group of RBW * NR right-hand sides) in an
// XCD-aware order (below).
// ---------------------------------------------------------------------------
template <typename T, int P, int RBW, int NR, bool BWD>
__global__ __launch_bounds__(64 * RBW) void gs2d_wave_kernel(const GsTile *tiles, int ntiles,
                                                       int ngroups,
                                                       const T *__restrict__ st,
                                                       const T *__restrict__ invd,
                                                       const int *__restrict__ cx_li,
                                                       const int *__restrict__ cx_col,
                                                       const T *__restrict__ cx_val,
                                                       const int *__restrict__ mr_li,
                                                       const int *__restrict__ mr_dst,
                                                       const T *__restrict__ f, T *u,
                                                       long long vs, int nrhs) {
  using T2 = typename Pair2<T>::type;
  constexpr int Q1 = P + 1, TT = 2 * Q1, W = TT + 2 * P;
  constexpr int S1 = 2 * P + 1, S = S1 * S1;
  constexpr int C = (S + 15) / 16;
  constexpr int SP = 16 * C;  // padded row length (zero coefficients beyond S)
  constexpr int NPH = Q1 * Q1;
  // window row stride: padded where the block's LDS stays within 64 KB.
  // A padded row holds K = WS / W windows side by side (right-hand side r
  // at plane r / K, columns (r % K) W ..): a read of one right-hand side
  // keeps the padded stride's bank pattern, and the padding is not wasted
  // LDS (at p = 6, two windows of 26 columns in a row of 52)
  constexpr int WS0 = gs_window_stride(P) > W ? gs_window_stride(P) : W;
  constexpr int K0 = WS0 / W, NPL0 = (NR + K0 - 1) / K0;
  constexpr bool WFIT =
      (size_t)RBW * (NPL0 * W * WS0 + NR * 2 * TT * TT) * sizeof(T) + 16 * C * 4 <= 65536;
  constexpr int WS = WFIT ? WS0 : W;
  constexpr int KW = WS / W, NPL = (NR + KW - 1) / KW;
  constexpr int WW = W * WS;  // one plane of windows
  // LDS offset of right-hand side r's window
  auto roff = [](int r) { return (r / KW) * WW + (r % KW) * W; };
  // rows prefetched D classes ahead (deeper prefetch measured slower: the
  // longer prologue outweighs the hidden latency; 3 to 8 classes ahead time
  // the same at p = 6)
  constexpr int D0 = (sizeof(T) == 8 ? 48 : 96) / C;
  constexpr int D = D0 < 1 ? 1 : (D0 > NPH ? NPH : D0);
  __shared__ T sUa[RBW][NPL * WW];
  __shared__ T2 sBDa[RBW][NR][TT * TT];
  __shared__ int sOff[C * 16];
  // XCD-aware order: block ids go round-robin over the 8 XCDs; XCD x takes
  // the x-th contiguous eighth of the (tile, group) list, groups fastest, so
  // the groups of a tile run back to back on one XCD, whose L2 serves their
  // repeated stencil-row reads (the grid is padded to a multiple of 8)
  const int per = gridDim.x >> 3;
  const int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int tix = lb / ngroups, gid = lb - tix * ngroups;
  if (tix >= ntiles) return;
  const GsTile tl = tiles[tix];
  const int wid = threadIdx.x >> 6;
  const int zw = (gid * RBW + wid) * NR;  // first right-hand side of this wave
  const int nx = tl.nx, ny = tl.ny;
  const int x0 = tl.i0[0], y0 = tl.i0[1];
  const int wx0 = x0 - P, wy0 = y0 - P;
  const long long off = tl.off;
  const int lane = threadIdx.x & 63, grp = lane >> 4, l16 = lane & 15;
  const int ax = (grp & 1) * Q1, ay = (grp >> 1) * Q1;
  // Prologue, per right-hand side: every global load that does not depend on
  // another one is issued before the first wait (u window, f, 1/a_ii -- zero
  // on Dirichlet unknowns by construction); the cross-patch couplings follow
  // for all NR right-hand sides at once.  Right-hand sides past the batch run
  // on column 0 and store nothing.
  constexpr int NW = (W * W + 63) / 64, NT = (TT * TT + 63) / 64;
  for (int r = 0; r < NR; ++r) {
    const int z = zw + r < nrhs ? zw + r : 0;
    const T *fz = f + (long long)z * vs;
    const T *uz = u + (long long)z * vs;
    T *sU = sUa[wid] + roff(r);
    T2 *sBD = sBDa[wid][r];
    T wv[NW], fv[NT], dv[NT];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int i = lane + 64 * j;
      const int gy = wy0 + i / W, gx = wx0 + i % W;
      const bool ok = i < W * W && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      wv[j] = ok ? uz[off + (long long)gy * nx + gx] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int i = lane + 64 * j;
      const int iy = y0 + i / TT, ix = x0 + i % TT;
      const bool ok = i < TT * TT && ix < nx && iy < ny;
      const long long t = off + (long long)iy * nx + ix;
      fv[j] = ok ? fz[t] : (T)0;
      dv[j] = ok ? invd[t] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int i = lane + 64 * j;
      if (i < W * W) sU[(i / W) * WS + i % W] = wv[j];
    }
#pragma unroll
    for (int j = 0; j < NT; ++j)
      if (lane + 64 * j < TT * TT) {
        T2 bd;
        bd.x = fv[j];
        bd.y = dv[j];
        sBD[lane + 64 * j] = bd;
      }
  }
  // f minus the cross-patch couplings (a single wavefront: its LDS stores
  // land in program order, so the corrections see the pairs written above)
  __builtin_amdgcn_wave_barrier();
  {
    const T *uzs[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) uzs[r] = u + (long long)(zw + r < nrhs ? zw + r : 0) * vs;
    tile_cross<T, NR>(tl, cx_li, cx_col, cx_val, uzs, lane, [&](int row, const T *tot) {
#pragma unroll
      for (int r = 0; r < NR; ++r) sBDa[wid][r][row].x -= tot[r];
    });
  }
  if (wid == 0)
    for (int o = lane; o < C * 16; o += 64) sOff[o] = o < S ? (o / S1 - P) * WS + (o % S1 - P) : 0;
  // row of this lane's group in class s: a compile-time offset from the
  // group's first row.  Rows of a ragged tile outside the patch fall on later
  // rows or on the zero padding past the level's end (never beyond it: at
  // most a tile height of rows plus a tile width past the patch) and are
  // not updated.
  const T *rowbase = st + (off + (long long)(y0 + ay) * nx + x0 + ax) * SP + l16;
  const long long nxSP = (long long)nx * SP;
  auto row_ptr = [&](int s) {
    const int ph = BWD ? NPH - 1 - s : s;
    return rowbase + (ph / Q1) * nxSP + (ph % Q1) * SP;
  };
  T buf[D][C];
#pragma unroll
  for (int s = 0; s < D; ++s) {
    const T *srow = row_ptr(s);
#pragma unroll
    for (int c = 0; c < C; ++c) buf[s][c] = srow[16 * c];
  }
  __syncthreads();
  // LDS addresses of this lane's slots at the group's first row (first
  // right-hand side; the others follow at compile-time offsets); a class
  // adds a compile-time offset
  const T *ub[C];
  const int wl = (ay + P) * WS + ax + P;
  const T *sU0 = sUa[wid];
#pragma unroll
  for (int c = 0; c < C; ++c) ub[c] = sU0 + wl + sOff[l16 + 16 * c];
  T *uw = sUa[wid] + wl;
  const T2 *bdl = sBDa[wid][0] + ay * TT + ax;
#pragma unroll
  for (int s = 0; s < NPH; ++s) {
    const int ph = BWD ? NPH - 1 - s : s;
    const int ix = x0 + ph % Q1 + ax, iy = y0 + ph / Q1 + ay;
    const int cw = (ph / Q1) * WS + ph % Q1, cl2 = (ph / Q1) * TT + ph % Q1;
    T uv[NR][C], uold[NR], acc[NR], ubd[NR], dinv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
      for (int c = 0; c < C; ++c) uv[r][c] = ub[c][roff(r) + cw];
      uold[r] = uw[roff(r) + cw];
      const T2 bd = bdl[r * TT * TT + cl2];
      // u + (b - a.u) d: every LDS value of the class is consumed before the
      // scans, so the reads go out as one batch and none is sunk past them
      ubd[r] = fma(bd.x, bd.y, uold[r]);
      dinv[r] = bd.y;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      // two independent partial sums halve the dependent multiply-add chain
      T acc0 = 0, acc1 = 0;
#pragma unroll
      for (int c = 0; c < C; c += 2) acc0 += buf[s % D][c] * uv[r][c];
#pragma unroll
      for (int c = 1; c < C; c += 2) acc1 += buf[s % D][c] * uv[r][c];
      acc[r] = acc0 + acc1;
      asm volatile("" : "+v"(acc[r]), "+v"(ubd[r]), "+v"(dinv[r]));
    }
    if (s + D < NPH) {
      const T *srow = row_ptr(s + D);
#pragma unroll
      for (int c = 0; c < C; ++c) buf[s % D][c] = srow[16 * c];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = row16_scan(acc[r]);
    if (l16 == 15 && ix < nx && iy < ny) {
#pragma unroll
      for (int r = 0; r < NR; ++r) uw[roff(r) + cw] = fma(-acc[r], dinv[r], ubd[r]);
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  }
  __syncthreads();
  for (int r = 0; r < NR; ++r) {
    const int z = zw + r;
    if (z >= nrhs) break;
    T *uz = u + (long long)z * vs;
    const T *sU = sUa[wid] + roff(r);
    for (int i = lane; i < TT * TT; i += 64) {
      int iy = y0 + i / TT, ix = x0 + i % TT;
      if (ix < nx && iy < ny) uz[off + (long long)iy * nx + ix] = sU[(iy - wy0) * WS + (ix - wx0)];
    }
    // conforming: the tile's owned glued unknowns into their copies in other
    // patches (those patches carry other colours: nothing else writes there)
    for (int e = lane; e < tl.mr_n; e += 64) {
      const int lt = mr_li[tl.mr_off + e];
      uz[mr_dst[tl.mr_off + e]] = sU[(lt / TT + P) * WS + lt % TT + P];
    }
  }
}

// ---------------------------------------------------------------------------
// Operator by the stored rows (levels that keep the Gauss-Seidel rows):
//   r = mask (beta fw.*f + alpha (S u + X u)),
// S = same-patch rows (volume + same-side interface terms, (2p+1)^2 per
// unknown), X = the cross-patch couplings of each tile's rows.  The matrix is
// the one the sum-factorized volume kernel and the interface kernel apply
// (assembled with the same quadrature); it is read once per group of RB
// right-hand sides instead of being recomputed for each of them.
// One block per (tile of the Gauss-Seidel partition, group of RB right-hand
// sides): the group's u windows sit in LDS and every 16-lane row group reads
// a stencil row once and applies it to the RB right-hand sides.  1D grid:
// consecutive block ids go to different XCDs (id mod 8), so the groups of one
// tile get ids of equal residue and share one XCD's L2.
// ---------------------------------------------------------------------------
template <typename T, int P, int RB>
__global__ __launch_bounds__(256) void sp2d_kernel(const GsTile *tiles, int ntiles, int ngroups,
                                                   int nrhs, const T *__restrict__ st,
                                                   const int *__restrict__ cx_li,
                                                   const int *__restrict__ cx_col,
                                                   const T *__restrict__ cx_val,
                                                   const unsigned char *__restrict__ mask,
                                                   const T *__restrict__ u,
                                                   const T *__restrict__ f,
                                                   const T *__restrict__ fw, T beta, T alpha,
                                                   T *__restrict__ r, long long vs) {
  constexpr int Q1 = P + 1, TT = 2 * Q1, W = TT + 2 * P, NT = TT * TT;
  constexpr int S1 = 2 * P + 1, S = S1 * S1;
  constexpr int C = (S + 15) / 16;
  constexpr int SP = 16 * C;
  __shared__ T sU[RB][W * W];
  __shared__ T sX[RB][NT];
  const int b = blockIdx.x;
  const int slot = b >> 3;
  const int tile = (slot / ngroups) * 8 + (b & 7);
  if (tile >= ntiles) return;
  const int z0 = (slot % ngroups) * RB;
  const int nz = min(RB, nrhs - z0);
  const GsTile tl = tiles[tile];
  const int nx = tl.nx, ny = tl.ny;
  const int x0 = tl.i0[0], y0 = tl.i0[1];
  const int wx0 = x0 - P, wy0 = y0 - P;
  const long long off = tl.off;
  const int tid = threadIdx.x;
  for (int i = tid; i < RB * W * W; i += 256) {
    const int z = i / (W * W), k = i - z * (W * W);
    const int gy = wy0 + k / W, gx = wx0 + k % W;
    const bool ok = z < nz && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    sU[z][k] = ok ? u[(long long)(z0 + z) * vs + off + (long long)gy * nx + gx] : (T)0;
  }
  for (int i = tid; i < RB * NT; i += 256) sX[i / NT][i % NT] = (T)0;
  __syncthreads();
  // cross-patch couplings: one wave per right-hand side (after the zeroing
  // above: a block barrier), one update per row
  const int wave = tid >> 6, lane = tid & 63;
  for (int z = wave; z < nz; z += 4) {
    const T *uzs[1] = {u + (long long)(z0 + z) * vs};
    tile_cross<T, 1>(tl, cx_li, cx_col, cx_val, uzs, lane,
                     [&](int row, const T *tot) { sX[z][row] += tot[0]; });
  }
  const int g = tid >> 4, l16 = tid & 15;
  int soff[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = l16 + 16 * c;
    soff[c] = k < S ? (k / S1 - P) * W + (k % S1 - P) : 0;
  }
  // rows outside the patch (ragged last tiles) read the tile origin's row
  // and are not written
  auto row_ptr = [&](int li) {
    const int ix = x0 + li % TT, iy = y0 + li / TT;
    const bool ok = ix < nx && iy < ny;
    const long long t = ok ? off + (long long)iy * nx + ix : off + (long long)y0 * nx + x0;
    return st + t * SP + l16;
  };
  T a[C], an[C];
  {
    const T *sr = row_ptr(g);
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = sr[16 * c];
  }
  __syncthreads();  // window and zeroed sums complete
  for (int li = g; li < NT; li += 16) {
    if (li + 16 < NT) {
      const T *sr = row_ptr(li + 16);
#pragma unroll
      for (int c = 0; c < C; ++c) an[c] = sr[16 * c];
    }
    const int ix = x0 + li % TT, iy = y0 + li / TT;
    if (ix < nx && iy < ny) {
      const int wi = (iy - wy0) * W + (ix - wx0);
#pragma unroll
      for (int z = 0; z < RB; ++z) {
        if (z >= nz) break;
        T acc0 = 0, acc1 = 0;
#pragma unroll
        for (int c = 0; c < C; c += 2) acc0 += a[c] * sU[z][wi + soff[c]];
#pragma unroll
        for (int c = 1; c < C; c += 2) acc1 += a[c] * sU[z][wi + soff[c]];
        const T acc = row16_scan(acc0 + acc1);
        if (l16 == 15) sX[z][li] += acc;
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = an[c];
  }
  __syncthreads();
  // coalesced write-back of the tile rows
  for (int i = tid; i < RB * NT; i += 256) {
    const int z = i / NT, li = i - z * NT;
    const int ix = x0 + li % TT, iy = y0 + li / TT;
    if (z >= nz || ix >= nx || iy >= ny) continue;
    const long long t = off + (long long)iy * nx + ix;
    const long long zo = (long long)(z0 + z) * vs;
    T v = alpha * sX[z][li];
    if (f) v += beta * (fw ? fw[t] : (T)1) * f[zo + t];
    r[zo + t] = mask[t] ? v : (T)0;
  }
}

// ---------------------------------------------------------------------------
// Operator by the stored rows for a batch of float32 right-hand sides, one
// right-hand side per lane (64 per wavefront):
//   r = mask (beta fw.*f + alpha S u)
// (S = the same-patch rows; the cross-patch couplings are added by a second
// kernel over the coupled rows).  u is first transposed to uT[t][64] so that
// the 64 values of a row are one contiguous line.  A wavefront takes BX
// consecutive rows of one patch line and walks the 2p+1 stencil lines b: it
// loads the BX + 2p values of line b once and applies them to all BX rows
// (each serves up to 2p+1 products); the coefficients of a (row, b) pair are
// the same for every lane: wave-uniform loads into scalar registers, used
// directly as the scalar operand of the products.  No LDS, no cross-lane
// reduction and no atomics: each lane owns its sums, summed in a fixed order
// (even and odd stencil lines apart, then added).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void transpose64_kernel(const float *__restrict__ u, int nrhs,
                                                          long long vs,
                                                          const long long *__restrict__ lines,
                                                          long long ptot,
                                                          float *__restrict__ ut) {
  // one patch line per block: its rows (torn offset lines[3 l], lines[3 l + 2]
  // of them) go to the padded copy at lines[3 l + 1], 64 rows x 64 right-hand
  // sides at a time through LDS (odd pitch), right-hand side group g at
  // g * ptot rows
  // the next 64 x 64 tile's loads are issued before the current tile's
  // stores
  __shared__ float tile[64][65];
  const long long tl0 = lines[3 * blockIdx.x], pl0 = lines[3 * blockIdx.x + 1];
  const int nx = (int)lines[3 * blockIdx.x + 2];
  const int z0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  float v[16];
  auto load = [&](int x0) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int zz = ty + 4 * m;
      v[m] = (z0 + zz < nrhs && x0 + tx < nx) ? u[(long long)(z0 + zz) * vs + tl0 + x0 + tx]
                                              : 0.0f;
    }
  };
  load(0);
  for (int x0 = 0; x0 < nx; x0 += 64) {
#pragma unroll
    for (int m = 0; m < 16; ++m) tile[ty + 4 * m][tx] = v[m];
    __syncthreads();
    if (x0 + 64 < nx) load(x0 + 64);
    for (int xx = ty; xx < 64 && x0 + xx < nx; xx += 4)
      ut[((long long)blockIdx.y * ptot + pl0 + x0 + xx) * 64 + tx] = tile[tx][xx];
    __syncthreads();
  }
}

// acc = c * w (Init) or acc += c * w, where c is read from lane A of this
// lane's 16-lane row (DPP row_newbcast): a register holding the 13
// coefficients of a stencil line in lanes 0..12 of every row serves all 64
// lanes.  The statements are volatile so that they keep the order written
// below (one offset for all rows of a strip, so no product waits on the one
// before it).  The leading s_nop of offset 0 keeps two wait states between any
// VALU write of the coefficient register and its first DPP read (it is
// written by LDS loads only).
template <int A, bool Init>
__device__ __forceinline__ void dpp_term(float &acc, float c, float w) {
  if constexpr (Init) {
    if constexpr (A == 0)
      asm volatile("s_nop 1\n\tv_mul_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf"
                   : "=v"(acc)
                   : "v"(c), "v"(w));
    else
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                   : "=v"(acc)
                   : "v"(c), "v"(w), "n"(A));
  } else {
    if constexpr (A == 0)
      asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf"
                   : "+v"(acc)
                   : "v"(c), "v"(w));
    else
      asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                   : "+v"(acc)
                   : "v"(c), "v"(w), "n"(A));
  }
}
// stencil offset A of one line for every row q of the strip: even offsets
// into ps[q], odd ones into ps[BX + q]; Init starts the sums (offsets 0, 1
// of the first line of a pair)
template <int A, bool Init, int... Qs>
__device__ __forceinline__ void dpp_offset(float *ps, const float *cf, const float *win,
                                           std::integer_sequence<int, Qs...>) {
  constexpr int BXN = sizeof...(Qs);
  (dpp_term<A, Init && (A < 2)>(ps[(A & 1) * BXN + Qs], cf[Qs], win[Qs + A]), ...);
}
template <int BX, bool Init, int... As>
__device__ __forceinline__ void dpp_line_offsets(float *ps, const float *cf, const float *win,
                                                 std::integer_sequence<int, As...>) {
  (dpp_offset<As, Init>(ps, cf, win, std::make_integer_sequence<int, BX>{}), ...);
}
template <int BX, int S1, bool Init>
__device__ __forceinline__ void dpp_line(float *ps, const float *cf, const float *win) {
  dpp_line_offsets<BX, Init>(ps, cf, win, std::make_integer_sequence<int, S1>{});
}

#ifndef SP_RHS_WAVES_PER_EU
#define SP_RHS_WAVES_PER_EU 3
#endif
template <int P, int BX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SP_RHS_WAVES_PER_EU))) void sp2d_rhs_kernel(const GsTile *tiles, int ntiles, int nrhs,
                                                       const float *__restrict__ st,
                                                       const unsigned char *__restrict__ mask,
                                                       const float *__restrict__ ut,
                                                       long long ptot,
                                                       const float *__restrict__ f,
                                                       const float *__restrict__ fw, float beta,
                                                       float alpha, float *__restrict__ r,
                                                       long long vs) {
  constexpr int S1 = 2 * P + 1, S = S1 * S1, SP = (S + 15) / 16 * 16;
  constexpr int WX = BX + 2 * P;
  const int w = threadIdx.x >> 6;
  // XCD-aware order: block ids go round-robin over the 8 XCDs, so XCD x
  // takes the x-th contiguous eighth of the strip list (its window lines
  // stay in that XCD's L2 from one line group to the next); the grid is
  // padded to a multiple of 8 blocks
  const int per = gridDim.x >> 3;
  const int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int item = lb * 4 + w;
  if (item >= ntiles) return;
  const GsTile tl = tiles[item];
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  const int zg = blockIdx.y;
  const int nx = tl.nx;
  const int x0 = tl.i0[0], y = tl.i0[1];
  const long long off = tl.off;
  // first row of the strip; rows of a ragged strip past the patch read the
  // rows that follow (the next line, or the zero padding past the level's
  // end: at most BX - 1 rows) and are not stored
  const float *row0 = st + (off + (long long)y * nx + x0) * SP;
  const int nq = nx - x0 < BX ? nx - x0 : BX;
  // Window of stencil line b: BX + 2p consecutive values of the padded copy
  // (zeros outside the patch), no conditions.  Beyond the padded line only
  // rows past the patch read (they are not stored).
  const int pw = nx + 2 * P;
  const float *ug = ut + ((long long)zg * ptot + tl.pad_off + (long long)y * pw + x0) * 64 + lane;
  auto load_line = [&](int b, float *win) {
    const float *lb = ug + (long long)b * pw * 64;
#pragma unroll
    for (int i = 0; i < WX; ++i) win[i] = lb[i * 64];
  };
  // the strip's BX rows of coefficients (contiguous) into this wavefront's
  // LDS slice, all loads in flight at once; the slice holds the strip's
  // results afterwards ([right-hand side][row], odd pitch BX + 1)
  constexpr int OP = BX + 1;
  constexpr int LW = BX * SP > 64 * OP ? BX * SP : 64 * OP;
  __shared__ float sC[4][LW];
  float *sc = sC[w];
  {
    constexpr int N4 = BX * SP / 4, PER = (N4 + 63) / 64;
    const float4 *src = reinterpret_cast<const float4 *>(row0);
    float4 v[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = lane + 64 * m;
      v[m] = e < N4 ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = lane + 64 * m;
      if (e < N4) reinterpret_cast<float4 *>(sc)[e] = v[m];
    }
    __builtin_amdgcn_wave_barrier();
  }
  // coefficients of stencil line b of the BX rows: lanes 0..12 of every
  // 16-lane row hold the line's S1 values, one register per row
  const int ka = l16 < S1 ? l16 : 0;
  auto load_coef = [&](int b, float *cf) {
    const float *cb = sc + b * S1 + ka;
#pragma unroll
    for (int q = 0; q < BX; ++q) cf[q] = cb[q * SP];
  };
  // Summation order (float32): the products of a pair of stencil lines go
  // into two partial sums per row (even and odd offsets, chains of at most
  // 14), added into the row's total once per pair (7 pairs) -- close to the
  // tree of the 16-lane row kernels (a single running sum of all (2p+1)^2
  // products loses enough accuracy to cost the float64 iterative refinement
  // an extra step)
  float tot[BX], ps[2 * BX];
#pragma unroll
  for (int q = 0; q < BX; ++q) tot[q] = 0.0f;
  float wa[WX], wb[WX], ca[BX], cb2[BX];
  load_line(0, wa);
  load_coef(0, ca);
  // stencil lines in pairs: even lines from (wa, ca), odd from (wb, cb2);
  // each pair's successor is loaded before its products
#pragma unroll 1
  for (int b = 0; b < S1; b += 2) {
    if (b + 1 < S1) {
      load_line(b + 1, wb);
      load_coef(b + 1, cb2);
    }
    dpp_line<BX, S1, true>(ps, ca, wa);
    if (b + 1 < S1) {
      if (b + 2 < S1) {
        load_line(b + 2, wa);
        load_coef(b + 2, ca);
      }
      dpp_line<BX, S1, false>(ps, cb2, wb);
    }
#pragma unroll
    for (int q = 0; q < BX; ++q) tot[q] += ps[q] + ps[BX + q];
  }
  // Results through LDS: lane z has the strip's BX totals of right-hand
  // side z; 16 lanes then take the rows of one right-hand side (four per
  // instruction), so that a load of f or a store of r covers the strip's
  // consecutive rows of four right-hand sides instead of one value in each
  // of 64 vectors
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < BX; ++q) sc[lane * OP + q] = alpha * tot[q];
  __builtin_amdgcn_wave_barrier();
  const int qq = lane & 15, zs = lane >> 4;
  if (qq >= nq) return;
  const long long t = off + (long long)y * nx + x0 + qq;
  const bool keep = mask[t] != 0;
  const float wf = f ? beta * (fw ? fw[t] : 1.0f) : 0.0f;
#pragma unroll 4
  for (int zz = 0; zz < 16; ++zz) {
    const int zl = zz * 4 + zs, zr = zg * 64 + zl;
    if (zr >= nrhs) break;
    float v = sc[zl * OP + qq];
    const long long zo = (long long)zr * vs;
    if (f) v += wf * f[zo + t];
    r[zo + t] = keep ? v : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// 3D patches.  A tile holds TT^3 unknowns (TT = 2(p+1)); its u window with a
// halo of p on every side sits in LDS.  Stencil rows ((2p+1)^3 entries padded
// to 16-lane groups) are read by one 16-lane group per row; slot k of a row
// is the neighbour (k mod S1 - p, k / S1 mod S1 - p, k / S1^2 - p).
// ---------------------------------------------------------------------------
template <int P>
struct Tile3 {
  static constexpr int Q1 = P + 1, TT = 2 * Q1, W = TT + 2 * P;
  static constexpr int NT = TT * TT * TT, NW = W * W * W;
  static constexpr int S1 = 2 * P + 1, S = S1 * S1 * S1;
  static constexpr int C = (S + 15) / 16, SP = 16 * C;
  static constexpr int NPH = Q1 * Q1 * Q1;
  // window offset of stencil slot k (0 for the zero padding slots)
  __device__ static int slot_off(int k) {
    return k < S ? ((k / (S1 * S1) - P) * W + (k / S1 % S1 - P)) * W + (k % S1 - P) : 0;
  }
};

// window of u (halo p, zero outside the patch) into LDS
template <typename T, int P>
__device__ inline void load_window3(const GsTile3 &tl, const T *u, T *sU, int tid, int nthr) {
  using G = Tile3<P>;
  const int wx0 = tl.i0[0] - P, wy0 = tl.i0[1] - P, wz0 = tl.i0[2] - P;
  for (int i = tid; i < G::NW; i += nthr) {
    const int gx = wx0 + i % G::W, gy = wy0 + i / G::W % G::W, gz = wz0 + i / (G::W * G::W);
    const bool ok = gx >= 0 && gx < tl.n[0] && gy >= 0 && gy < tl.n[1] && gz >= 0 && gz < tl.n[2];
    sU[i] = ok ? u[tl.off + ((long long)gz * tl.n[1] + gy) * tl.n[0] + gx] : (T)0;
  }
}

// Cross-patch couplings of 3D levels, one thread per coupled row r0 <= r < r1
// (CSR order, two partial sums): ADD = false stores s = X_row u (the
// Gauss-Seidel right-hand side correction of a patch colour), ADD = true adds
// alpha s to the masked output row (operator apply).  grid.y = right-hand side.
template <typename T, bool ADD>
__global__ __launch_bounds__(256) void cross3d_kernel(const int *__restrict__ rows,
                                                      const int *__restrict__ ptr,
                                                      const int *__restrict__ col,
                                                      const T *__restrict__ val, int r0, int r1,
                                                      const unsigned char *__restrict__ mask,
                                                      const T *__restrict__ u, T *out, T alpha,
                                                      long long vs) {
  const int r = r0 + blockIdx.x * 256 + threadIdx.x;
  if (r >= r1) return;
  const long long zo = (long long)blockIdx.y * vs;
  const int t = rows[r];
  int e = ptr[r];
  const int e1 = ptr[r + 1];
  T s0 = 0, s1 = 0;
#pragma unroll 4
  for (; e + 1 < e1; e += 2) {
    s0 += val[e] * u[zo + col[e]];
    s1 += val[e + 1] * u[zo + col[e + 1]];
  }
  if (e < e1) s0 += val[e] * u[zo + col[e]];
  const T sum = s0 + s1;
  if (ADD) {
    if (mask[t]) out[zo + t] += alpha * sum;
  } else {
    out[zo + t] = sum;
  }
}

// Sum over a wavefront, valid in lane 63: DPP scans inside the four rows of
// 16 lanes, then row_bcast:15 adds the last lane of rows 0 and 2 into rows 1
// and 3, and row_bcast:31 adds lane 31 into rows 2 and 3.  Lane 63 ends with
// (r3 + r2) + (r1 + r0), a fixed order, with no scalar round trip.
template <int CTRL, int ROWS>
__device__ inline double dpp_bcast(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWS, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWS>
__device__ inline float dpp_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <typename T>
__device__ inline T wave_sum_last(T v) {
  v = row16_scan(v);
  v += dpp_bcast<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_bcast<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

// Multicolour Gauss-Seidel on 3D tiles: one block of eight wavefronts per
// tile and right-hand side.  Phase s of the sweep updates the eight unknowns
// of the tile whose index mod (p+1) is (s mod Q1, s / Q1 mod Q1, s / Q1^2)
// -- one colour class of the ordering --, one unknown per wavefront, and a
// block barrier separates the phases.  A lane holds SP/64 slots of a row, so
// the rows of the next D phases fit in registers and their loads overlap the
// phases before them.  f - xs (xs = the cross-patch couplings applied to the
// neighbouring patches' values, another patch colour, constant during the
// patch colour's launches; zero on rows without couplings) and 1/a_ii sit in
// LDS.  grid.x = right-hand side, grid.y = tile.
template <typename T, int P, bool BWD>
__global__ __launch_bounds__(512) void gs3d_kernel(const GsTile3 *tiles, const T *__restrict__ st,
                                                   const T *__restrict__ invd,
                                                   const T *__restrict__ xs,
                                                   const int *__restrict__ mr_li,
                                                   const int *__restrict__ mr_dst,
                                                   const T *__restrict__ f, T *u, long long vs) {
  using G = Tile3<P>;
  constexpr int Q1 = G::Q1, TT = G::TT, W = G::W, SP = G::SP, NPH = G::NPH;
  constexpr int CL = (SP + 63) / 64;           // slots per lane
  constexpr int D = sizeof(T) == 8 ? 4 : 8;    // phases in flight
  __shared__ T sU[G::NW];
  __shared__ T sB[G::NT];
  __shared__ T sD[G::NT];
  const GsTile3 tl = tiles[blockIdx.y];
  f += (long long)blockIdx.x * vs;
  xs += (long long)blockIdx.x * vs;
  u += (long long)blockIdx.x * vs;
  const int tid = threadIdx.x;
  const int nx = tl.n[0], ny = tl.n[1], nz = tl.n[2];
  const int x0 = tl.i0[0], y0 = tl.i0[1], z0 = tl.i0[2];
  load_window3<T, P>(tl, u, sU, tid, 512);
  for (int i = tid; i < G::NT; i += 512) {
    const int ix = x0 + i % TT, iy = y0 + i / TT % TT, iz = z0 + i / (TT * TT);
    const bool ok = ix < nx && iy < ny && iz < nz;
    const long long t = tl.off + ((long long)iz * ny + iy) * nx + ix;
    sB[i] = ok ? f[t] - xs[t] : (T)0;
    sD[i] = ok ? invd[t] : (T)0;
  }
  const int w = tid >> 6, lane = tid & 63;
  const int ax = (w & 1) * Q1, ay = (w >> 1 & 1) * Q1, az = (w >> 2) * Q1;
  int soff[CL];
#pragma unroll
  for (int c = 0; c < CL; ++c) soff[c] = G::slot_off(lane + 64 * c);
  // row of this wavefront in phase s; rows outside the patch read the tile
  // origin's row and are not updated
  auto row_of = [&](int s, int &wi, int &li, bool &ok) {
    const int ph = BWD ? NPH - 1 - s : s;
    const int dx = ph % Q1 + ax, dy = ph / Q1 % Q1 + ay, dz = ph / (Q1 * Q1) + az;
    ok = x0 + dx < nx && y0 + dy < ny && z0 + dz < nz;
    wi = ((dz + P) * W + dy + P) * W + dx + P;
    li = (dz * TT + dy) * TT + dx;
    const long long t = ok ? tl.off + ((long long)(z0 + dz) * ny + y0 + dy) * nx + x0 + dx
                           : tl.off + ((long long)z0 * ny + y0) * nx + x0;
    return st + t * SP;
  };
  auto load_row = [&](int s, T *a) {
    int wi, li;
    bool ok;
    const T *sr = row_of(s, wi, li, ok);
#pragma unroll
    for (int c = 0; c < CL; ++c) {
      const int k = lane + 64 * c;
      a[c] = k < SP ? sr[k] : (T)0;
    }
  };
  T buf[D][CL];
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j < NPH) load_row(j, buf[j]);
  __syncthreads();
  // fully unrolled: the phase offsets are compile-time constants
#pragma unroll
  for (int s0 = 0; s0 < NPH; s0 += D) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int s = s0 + j;
      if (s < NPH) {
        int wi, li;
        bool ok;
        row_of(s, wi, li, ok);
        // every LDS value of the phase is read in one batch before the
        // reduction: u + (b - a.u) d = (u + b d) - (a.u) d
        T uv[CL];
#pragma unroll
        for (int c = 0; c < CL; ++c) uv[c] = sU[wi + soff[c]];
        const T uold = sU[wi], bb = sB[li];
        T dd = sD[li];
        T acc0 = 0, acc1 = 0;
#pragma unroll
        for (int c = 0; c < CL; c += 2) acc0 += buf[j][c] * uv[c];
#pragma unroll
        for (int c = 1; c < CL; c += 2) acc1 += buf[j][c] * uv[c];
        T ubd = fma(bb, dd, uold);
        T acc = acc0 + acc1;
        asm volatile("" : "+v"(acc), "+v"(ubd), "+v"(dd));
        if (s + D < NPH) load_row(s + D, buf[j]);
        acc = wave_sum_last(acc);
        if (lane == 63 && ok) sU[wi] = fma(-acc, dd, ubd);
        __syncthreads();
      }
    }
  }
  for (int i = tid; i < G::NT; i += 512) {
    const int dx = i % TT, dy = i / TT % TT, dz = i / (TT * TT);
    if (x0 + dx < nx && y0 + dy < ny && z0 + dz < nz)
      u[tl.off + ((long long)(z0 + dz) * ny + y0 + dy) * nx + x0 + dx] =
          sU[((dz + P) * W + dy + P) * W + dx + P];
  }
  // conforming: the tile's owned glued unknowns into their other copies
  for (int e = tid; e < tl.mr_n; e += 512) {
    const int lt = mr_li[tl.mr_off + e];
    const int dx = lt % TT, dy = lt / TT % TT, dz = lt / (TT * TT);
    u[mr_dst[tl.mr_off + e]] = sU[((dz + P) * W + dy + P) * W + dx + P];
  }
}

// Operator by the stored rows on 3D tiles: r = mask (beta fw.*f + alpha S u);
// the cross-patch part alpha X u follows in cross3d_kernel.  One block of 16
// row groups per tile and right-hand side.  grid.x = tile, grid.y = right-hand
// side.
template <typename T, int P>
__global__ __launch_bounds__(256) void sp3d_kernel(const GsTile3 *tiles, const T *__restrict__ st,
                                                   const unsigned char *__restrict__ mask,
                                                   const T *__restrict__ u,
                                                   const T *__restrict__ f,
                                                   const T *__restrict__ fw, T beta, T alpha,
                                                   T *__restrict__ r, long long vs) {
  using G = Tile3<P>;
  constexpr int TT = G::TT, W = G::W, C = G::C, SP = G::SP, NT = G::NT;
  __shared__ T sU[G::NW];
  __shared__ T sX[NT];
  const GsTile3 tl = tiles[blockIdx.x];
  const long long zo = (long long)blockIdx.y * vs;
  u += zo;
  const int tid = threadIdx.x;
  const int nx = tl.n[0], ny = tl.n[1], nz = tl.n[2];
  const int x0 = tl.i0[0], y0 = tl.i0[1], z0 = tl.i0[2];
  load_window3<T, P>(tl, u, sU, tid, 256);
  for (int i = tid; i < NT; i += 256) sX[i] = (T)0;
  const int g = tid >> 4, l16 = tid & 15;
  int soff[C];
#pragma unroll
  for (int c = 0; c < C; ++c) soff[c] = G::slot_off(l16 + 16 * c);
  auto row_ptr = [&](int li) {
    const int dx = li % TT, dy = li / TT % TT, dz = li / (TT * TT);
    const bool ok = x0 + dx < nx && y0 + dy < ny && z0 + dz < nz;
    const long long t = ok ? tl.off + ((long long)(z0 + dz) * ny + y0 + dy) * nx + x0 + dx
                           : tl.off + ((long long)z0 * ny + y0) * nx + x0;
    return st + t * SP + l16;
  };
  T a[C], an[C];
  {
    const T *sr = row_ptr(g);
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = sr[16 * c];
  }
  __syncthreads();  // window and zeroed sums complete
  for (int li = g; li < NT; li += 16) {
    if (li + 16 < NT) {
      const T *sr = row_ptr(li + 16);
#pragma unroll
      for (int c = 0; c < C; ++c) an[c] = sr[16 * c];
    }
    const int dx = li % TT, dy = li / TT % TT, dz = li / (TT * TT);
    if (x0 + dx < nx && y0 + dy < ny && z0 + dz < nz) {
      const int wi = ((dz + P) * W + dy + P) * W + dx + P;
      T acc0 = 0, acc1 = 0;
#pragma unroll
      for (int c = 0; c < C; c += 2) acc0 += a[c] * sU[wi + soff[c]];
#pragma unroll
      for (int c = 1; c < C; c += 2) acc1 += a[c] * sU[wi + soff[c]];
      const T acc = row16_scan(acc0 + acc1);
      if (l16 == 15) sX[li] += acc;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = an[c];
  }
  __syncthreads();
  for (int li = tid; li < NT; li += 256) {
    const int dx = li % TT, dy = li / TT % TT, dz = li / (TT * TT);
    if (x0 + dx >= nx || y0 + dy >= ny || z0 + dz >= nz) continue;
    const long long t = tl.off + ((long long)(z0 + dz) * ny + y0 + dy) * nx + x0 + dx;
    T v = alpha * sX[li];
    if (f) v += beta * (fw ? fw[t] : (T)1) * f[zo + t];
    r[zo + t] = mask[t] ? v : (T)0;
  }
}

// Transfer between dyadic 3D levels, one output entry per thread: the
// tensor product of the three 1D band rows (prolongation rows of the fine
// level's embedding, or its columns for the restriction) applied to the input
// patch tensor.  Restriction weights the fine input (consistent ->
// distributed) and writes the masked coarse result; prolongation adds into
// the free fine entries.  grid.y = right-hand side.
template <typename T, bool RESTRICT>
__global__ __launch_bounds__(256) void transfer3d_kernel(
    const PatchDev *__restrict__ pd_in, const PatchDev *__restrict__ pd_out,
    const PatchDev *__restrict__ pd_fine, int K, long long n_out, const int *__restrict__ lo,
    const T *__restrict__ val, int W, const T *__restrict__ in, const T *__restrict__ win,
    const unsigned char *__restrict__ mask_out, T *out, T *zero_out, long long vs_in,
    long long vs_out) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= n_out) return;
  in += (long long)blockIdx.y * vs_in;
  const long long to = (long long)blockIdx.y * vs_out + t;
  int k = 0, hi = K - 1;
  while (k < hi) {  // last patch with off <= t
    const int mid = (k + hi + 1) >> 1;
    if (pd_out[mid].off <= t)
      k = mid;
    else
      hi = mid - 1;
  }
  const PatchDev &po = pd_out[k], &pi = pd_in[k], &pf = pd_fine[k];
  long long loc = t - po.off;
  const int ox = (int)(loc % po.n[0]);
  loc /= po.n[0];
  const int oy = (int)(loc % po.n[1]), oz = (int)(loc / po.n[1]);
  if (!RESTRICT && !mask_out[t]) return;
  const int rx = (RESTRICT ? pf.xr[0] : pf.xp[0]) + ox;
  const int ry = (RESTRICT ? pf.xr[1] : pf.xp[1]) + oy;
  const int rz = (RESTRICT ? pf.xr[2] : pf.xp[2]) + oz;
  const int lx = lo[rx], ly = lo[ry], lz = lo[rz];
  T sum = 0;
  for (int c = 0; c < W; ++c) {
    const int jz = lz + c;
    const T vz = val[(long long)rz * W + c];
    if (jz >= pi.n[2] || vz == (T)0) continue;
    for (int b = 0; b < W; ++b) {
      const int jy = ly + b;
      const T vy = val[(long long)ry * W + b];
      if (jy >= pi.n[1] || vy == (T)0) continue;
      T sx = 0;
      for (int a = 0; a < W; ++a) {
        const int jx = lx + a;
        if (jx >= pi.n[0]) break;
        const long long j = pi.off + ((long long)jz * pi.n[1] + jy) * pi.n[0] + jx;
        T v = in[j];
        if (RESTRICT) v *= win[j];
        sx += val[(long long)rx * W + a] * v;
      }
      sum += vz * vy * sx;
    }
  }
  if (RESTRICT) {
    out[to] = mask_out[t] ? sum : (T)0;
    if (zero_out) zero_out[to] = 0;
  } else {
    out[to] += sum;
  }
}

// ---------------------------------------------------------------------------
// Fast-diagonalization step of the subspace corrected mass smoother on the
// matrix cores, fused form (Fd2Item): a block of 256 threads owns 16 rows of
// the output and computes Z = L[rows, :] M1 (Z kept in LDS), then R = Z M2,
// then the item's epilogue.  B operands are streamed through LDS in chunks
// of KC rows, the next chunk held in registers.  Wave w owns the 16-column
// tiles w, w+4, ...,
// w+4(NJ-1) of the block; a k-step issues one MFMA per tile, the A fragment
// shared by the tiles:
//   float64: v_mfma_f64_16x16x4f64 on the stored operands;
//   float32: v_mfma_f32_16x16x4f32 on the stored operands;
//   bf16:    v_mfma_f32_16x16x32_bf16 on operands rounded to bfloat16
//            (nearest even) with float32 accumulation.
// Fragments of a 16 x 16 tile, lane l = 16 q + c (c < 16): A row c, k-block
// q; B column c, k-block q; accumulator register r holds column c of row
// 4q + r (float32 results), or of row q + 4r (float64 results).
// LDS strides: A rows 2 (mod 32) words apart, so the 16 rows of a fragment
// read hit distinct banks; B rows WB + 16 apart, so the two k-rows that half
// a wave reads hit disjoint banks.
// ---------------------------------------------------------------------------
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_b8 __attribute__((ext_vector_type(8)));

template <typename T>
struct MfAcc;

// Global-memory views of pointers read from a work-item record: the compiler
// cannot tell such a pointer's address space and emits flat accesses, which
// count against the LDS wait counter as well as the vector-memory one, so a
// wait for LDS operands would also wait for every load still in flight.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T *p) {
  return (gptr<T>)p;
}
template <>
struct MfAcc<double> {
  using type = mf_d4;
};
template <>
struct MfAcc<float> {
  using type = mf_f4;
};

// row of accumulator register r in lane group q (layouts above)
template <typename T>
__device__ constexpr int mf_row(int q, int r) {
  return sizeof(T) == 8 ? q + 4 * r : 4 * q + r;
}

template <bool BF>
struct MfK {
  static constexpr int KS = BF ? 32 : 4;  // k per MFMA
};

template <int NJ, bool BF>
struct Fd2mShape {
  static constexpr int WB = 64 * NJ;  // columns of a block (tiles of all four waves)
  static constexpr int LDB = WB + 16;  // B row stride in LDS
  static constexpr int LDZ = WB + 2;   // Z row stride (A operand of the second product)
  // B rows per streamed chunk (a multiple of the MFMA k; short chunks keep
  // the registers of the next chunk few for wide blocks)
  static constexpr int KC = (BF || NJ <= 2) ? 32 : 16;
};

// acc[j] += A[0:16, ka:ka+kn] B[0:kn, tile j] with A in LDS (row stride lda)
// and B rows in LDS (stride LDB); tiles at or beyond ncols are skipped
// (their accumulators stay as they are)
template <typename T, bool BF, int NJ>
__device__ inline void mfma_rows(const T *sA, int lda, int ka, const T *sB, int kn, int ncols,
                                 typename MfAcc<T>::type acc[NJ]) {
  constexpr int KS = MfK<BF>::KS, LDB = Fd2mShape<NJ, BF>::LDB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, q = lane >> 4;
#pragma unroll 2
  for (int k = 0; k < kn; k += KS) {
    if constexpr (!BF) {
      const T a = sA[c * lda + ka + k + q];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int col = 16 * (w + 4 * j);
        if (col < ncols) {
          const T b = sB[(k + q) * LDB + col + c];
          if constexpr (sizeof(T) == 8)
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
          else
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
        }
      }
    } else {
      mf_b8 a;
#pragma unroll
      for (int t = 0; t < 8; ++t) a[t] = (__bf16)sA[c * lda + ka + k + 8 * q + t];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int col = 16 * (w + 4 * j);
        if (col < ncols) {
          mf_b8 b;
#pragma unroll
          for (int t = 0; t < 8; ++t) b[t] = (__bf16)sB[(k + 8 * q + t) * LDB + col + c];
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
      }
    }
  }
}

// acc += A[16 x K] B[K x N]: B streamed from global memory through LDS in
// chunks of KC rows, the next chunk held in registers while the current one
// is multiplied (measured faster than staging all of B at once, which leaves
// one block per CU).  Rows of B past K and columns past N are stored as zero;
// A must be zero in columns K..Kp-1.
template <typename T, bool BF, int NJ>
__device__ inline void rowblock_mfma(const T *sA, int lda, gptr<const T> B, long long b_r, int K,
                                     int N, T *sM, typename MfAcc<T>::type acc[NJ]) {
  constexpr int WB = Fd2mShape<NJ, BF>::WB, LDB = Fd2mShape<NJ, BF>::LDB, KS = MfK<BF>::KS;
  constexpr int KC = Fd2mShape<NJ, BF>::KC;
  constexpr int LPT = KC * WB / 256;
  const int tid = threadIdx.x;
  const int Kp = (K + KS - 1) / KS * KS;
  T pre[LPT];
  auto gload = [&](int k0) {
#pragma unroll
    for (int x = 0; x < LPT; ++x) {
      const int e = tid + 256 * x;
      const int kk = e / WB, col = e % WB;
      pre[x] = (k0 + kk < K && col < N) ? B[(long long)(k0 + kk) * b_r + col] : (T)0;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < Kp; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int x = 0; x < LPT; ++x) {
      const int e = tid + 256 * x;
      sM[(e / WB) * LDB + e % WB] = pre[x];
    }
    __syncthreads();
    if (k0 + KC < Kp) gload(k0 + KC);
    mfma_rows<T, BF, NJ>(sA, lda, k0, sM, min(KC, Kp - k0), N, acc);
  }
}

// Interface pieces run as extra blocks of the first fused SCMS launch (they
// read the same residual and write only piece unknowns, the first stage only
// its scratch): block (piece, 64-row block) of u[copies] += scale inv r.
template <typename T>
struct PieceArgs {
  const PieceDev *pieces;
  const int *idx, *cp, *cidx;
  const T *inv;
  const T *r;
  T *u;
  T scale;
  long long vs;
  int n_pieces;
};

// rows row0..row0+63 of one piece with 256 threads: wavefront w sums the
// columns j = w (mod 4) (lane = row), the four partial sums added in order;
// sm: dynamic LDS of at least n + 256 values
template <typename T>
__device__ inline void piece_rows256(const PieceArgs<T> &pa, int piece, int row0, T *sm) {
  const PieceDev pc = pa.pieces[piece];
  const int n = pc.n;
  if (row0 >= n) return;  // uniform over the block
  T *spart = sm + n;  // 4 x 64 partial sums after the gathered residual (dynamic LDS)
  const gptr<const T> r = gmem(pa.r) + (long long)blockIdx.x * pa.vs;
  const gptr<T> u = gmem(pa.u) + (long long)blockIdx.x * pa.vs;
  const gptr<const int> idx = gmem(pa.idx), cp = gmem(pa.cp), cidx = gmem(pa.cidx);
  for (int j = threadIdx.x; j < n; j += 256) sm[j] = r[idx[pc.idx_off + j]];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = row0 + lane;
  T s0 = 0, s1 = 0;
  if (i < n) {
    const gptr<const T> col = gmem(pa.inv) + pc.inv_off + i;
    int j = w;
    for (; j + 4 < n; j += 8) {
      s0 += col[(long long)j * n] * sm[j];
      s1 += col[(long long)(j + 4) * n] * sm[j + 4];
    }
    if (j < n) s0 += col[(long long)j * n] * sm[j];
  }
  spart[w * 64 + lane] = s0 + s1;
  __syncthreads();
  if (w == 0 && i < n) {
    const T y = (spart[lane] + spart[64 + lane]) + (spart[128 + lane] + spart[192 + lane]);
    for (int c = cp[pc.cp_off + i]; c < cp[pc.cp_off + i + 1]; ++c) u[cidx[c]] += pa.scale * y;
  }
}

template <typename T, bool BF, int NJ>
__global__ __launch_bounds__(256) void fd2m_kernel(const Fd2Item<T> *items, int n_items, int lda,
                                                   PieceArgs<T> pa) {
  using A4 = typename MfAcc<T>::type;
  constexpr int LDZ = Fd2mShape<NJ, BF>::LDZ;
  extern __shared__ char smraw[];
  T *sm = (T *)smraw;
  if ((int)blockIdx.z >= n_items) {
    piece_rows256<T>(pa, blockIdx.z - n_items, blockIdx.y * 64, sm);
    return;
  }
  const Fd2Item<T> it = items[blockIdx.z];
  const int i0 = blockIdx.y * 16;
  if (i0 >= it.rows) return;
  const gptr<const T> M1 = gmem(it.M1) + (long long)blockIdx.x * it.m1_z;
  const gptr<T> O = gmem(it.O) + (long long)blockIdx.x * it.o_z;
  const gptr<const T> L = gmem(it.L);
  T *sL = sm;             // 16 x lda, zero beyond K1
  T *sZ = sL + 16 * lda;  // 16 x LDZ
  T *sM = sZ + 16 * LDZ;  // rows of B
  const int tid = threadIdx.x;
  const int nrow = min(16, it.rows - i0);
  for (int e0 = 0; e0 < 16 * lda; e0 += 256 * 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + tid + 256 * j;
      const int i = e / lda, a = e % lda;
      v[j] = (e < 16 * lda && i < nrow && a < it.K1) ? L[(long long)(i0 + i) * it.l_r + a] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (e0 + tid + 256 * j < 16 * lda) sL[e0 + tid + 256 * j] = v[j];
  }
  A4 acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = A4{0, 0, 0, 0};
  rowblock_mfma<T, BF, NJ>(sL, lda, M1, it.m1_r, it.K1, it.N, sM, acc);
  const int lane = tid & 63, w = tid >> 6, c = lane & 15, q = lane >> 4;
  // Z (zero in the columns past N) becomes the A operand of the second product
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) sZ[mf_row<T>(q, r) * LDZ + 16 * (w + 4 * j) + c] = acc[j][r];
    acc[j] = A4{0, 0, 0, 0};
  }
  rowblock_mfma<T, BF, NJ>(sZ, LDZ, gmem(it.M2), it.m2_r, it.N, it.N, sM, acc);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int col = 16 * (w + 4 * j) + c;
    if (col >= it.N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = mf_row<T>(q, r);
      if (i >= nrow) continue;
      const T v = acc[j][r];
      const gptr<T> o = O + (long long)(i0 + i) * it.o_r + col;
      if (it.lam_r)
        *o = v / (it.sigma + gmem(it.lam_r)[i0 + i] + gmem(it.lam_c)[col]);
      else
        *o += it.scale * v;
    }
  }
}

// ---------------------------------------------------------------------------
// One product stage of the fast diagonalization over a batch (FdGemm): a
// block computes a 64 x 64 tile of C_z; its four waves own 32 x 32 quarters
// (2 x 2 MFMA tiles).  K is streamed in chunks of 32 through LDS, both
// operands stored k-contiguous (B transposed on the way in), the next chunk
// held in registers while the current one is multiplied.  Large batches
// read every per-right-hand-side operand once per tile row/column instead of
// once per 16-row block of the fused form.
// grid.x = right-hand side, grid.y = tile, grid.z = item (patch).
// ---------------------------------------------------------------------------
#ifndef FDG_BF_KC
#define FDG_BF_KC 32
#endif
#ifndef FDG_F_KC
#define FDG_F_KC 16
#endif

template <typename T, bool BF>
__global__ __launch_bounds__(256) void fdg_kernel(const FdGemm<T> *items) {
  using A4 = typename MfAcc<T>::type;
  // LDS operand type: bfloat16 fragments are rounded once, when staged
  using ST = typename std::conditional<BF, __bf16, T>::type;
  // K chunk: one bf16 MFMA step; 16 rows for float32, where the smaller
  // register footprint (7 instead of 4 waves per SIMD) was measured faster
  constexpr int KC = BF ? FDG_BF_KC : (sizeof(T) == 8 ? 32 : FDG_F_KC), KS = MfK<BF>::KS;
  // row strides: 16-byte rows for the 8-wide bf16 fragments, 2 (mod 32)
  // words for the single-value fragments (16 rows on distinct banks)
  constexpr int LDK = BF ? KC + 8 : KC + 2;
  constexpr int NL = 64 * KC / 256;  // loads per thread, operand and chunk
  __shared__ ST sA[64 * LDK], sB[64 * LDK];
  const FdGemm<T> g = items[blockIdx.z];
  const int tm = blockIdx.y / g.tn, tc = blockIdx.y - tm * g.tn;
  const int m0 = tm * 64, n0 = tc * 64;
  if (m0 >= g.M) return;
  const long long z = blockIdx.x;
  const gptr<const T> A = gmem(g.A) + z * g.a_z, B = gmem(g.B) + z * g.b_z;
  const gptr<T> C = gmem(g.C) + z * g.c_z;
  const gptr<const T> lam_r = gmem(g.lam_r), lam_c = gmem(g.lam_c);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, q = lane >> 4;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  T pa[NL], pb[NL];
  auto gload = [&](int k0) {
#pragma unroll
    for (int x = 0; x < NL; ++x) {
      const int e = tid + 256 * x;
      const int ar = e / KC, ak = e % KC;
      pa[x] = (m0 + ar < g.M && k0 + ak < g.K) ? A[(long long)(m0 + ar) * g.a_r + k0 + ak] : (T)0;
      const int bk = e / 64, bc = e % 64;
      pb[x] = (k0 + bk < g.K && n0 + bc < g.N) ? B[(long long)(k0 + bk) * g.b_r + n0 + bc] : (T)0;
    }
  };
  A4 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = A4{0, 0, 0, 0};
  gload(0);
  for (int k0 = 0; k0 < g.K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int x = 0; x < NL; ++x) {
      const int e = tid + 256 * x;
      sA[(e / KC) * LDK + e % KC] = (ST)pa[x];
      sB[(e % 64) * LDK + e / 64] = (ST)pb[x];
    }
    __syncthreads();
    if (k0 + KC < g.K) gload(k0 + KC);
#pragma unroll
    for (int k = 0; k < KC; k += KS) {
      if constexpr (!BF) {
        T a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) a[t] = sA[(wm + 16 * t + c) * LDK + k + q];
#pragma unroll
        for (int u = 0; u < 2; ++u) b[u] = sB[(wn + 16 * u + c) * LDK + k + q];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if constexpr (sizeof(T) == 8)
              acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
            else
              acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[u], acc[t][u], 0, 0, 0);
          }
      } else {
        mf_b8 a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) a[t] = *(const mf_b8 *)&sA[(wm + 16 * t + c) * LDK + k + 8 * q];
#pragma unroll
        for (int u = 0; u < 2; ++u) b[u] = *(const mf_b8 *)&sB[(wn + 16 * u + c) * LDK + k + 8 * q];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int u = 0; u < 2; ++u)
            acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[u], acc[t][u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = n0 + wn + 16 * u + c;
      if (j >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + 16 * t + mf_row<T>(q, r);
        if (i >= g.M) continue;
        const T v = acc[t][u][r];
        const gptr<T> o = C + (long long)i * g.c_r + j;
        if (g.mode == 0)
          *o = v;
        else if (g.mode == 1)
          *o = v / (g.sigma + lam_r[i] + lam_c[j]);
        else
          *o += g.scale * v;
      }
    }
}

// ---------------------------------------------------------------------------
// One product stage of the 2D fast diagonalization over a whole batch
// (FdWide): the right-hand sides are concatenated along the dimension that
// belongs to them, so it splits into exact 64-wide tiles, and a block covers
// the whole wide dimension of the shared factor S (NT MFMA tiles of 16, NT
// even, rows past the factor zero in LDS).  Only the wide dimension (to 32)
// and K (to 16) are padded (260 unknowns: 288 x 272 computed, where 64 x 64
// tiles of every right-hand side's product would compute 320 x 320).  Wave w owns the 16 concatenated indices
// 16w..16w+15 of the block and all wide tiles; a k-step reads one fragment
// of X and one of S per wide tile.  K streams through LDS in chunks of KC
// (both operands k-contiguous), the next chunk held in registers.
//   left:  MFMA A = S rows (wide), B = X columns (concatenated);
//   right: MFMA A = X rows (concatenated), B = S rows read as columns (wide);
// so the outputs' 16 lanes of a row run along the contiguous index of C.
// grid.x = 64-wide tile of the concatenated dimension, grid.y = item.
// ---------------------------------------------------------------------------
template <typename T, bool BF, bool RIGHT, int NT>
__global__ __launch_bounds__(256) void fdw_kernel(const FdWide<T> *items, int nrhs) {
  using A4 = typename MfAcc<T>::type;
  using ST = typename std::conditional<BF, __bf16, T>::type;
  constexpr int KC = BF ? 32 : 16, KS = MfK<BF>::KS;
  constexpr int LDK = BF ? KC + 8 : KC + 2;
  constexpr int WT = 16 * NT;                     // wide rows held (zero past g.wide)
  constexpr int NLS = WT * KC / 256, NLX = 64 * KC / 256;
  constexpr int RS = 256 / KC;                    // S rows (right: X rows) per load round
  __shared__ ST sS[WT * LDK], sX[64 * LDK];
  const FdWide<T> g = items[blockIdx.y];
  const int ncat = nrhs * g.catn;
  const int c0 = blockIdx.x * 64;
  if (c0 >= ncat) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = lane & 15, q = lane >> 4;
  // global loads, branch-free: clamped addresses, out-of-range values zeroed.
  // S entry (row tid / KC + RS x, k tid % KC); X entry: left, column
  // tid % 64 (one per thread) and k tid / 64 + 4 x; right, row tid / KC +
  // RS x and k tid % KC
  const int ks = tid % KC;
  gptr<const T> sbase[NLS];
  bool sok[NLS];
#pragma unroll
  for (int x = 0; x < NLS; ++x) {
    const int row = tid / KC + RS * x;
    sok[x] = row < g.wide;
    sbase[x] = gmem(g.S) + (long long)min(row, g.wide - 1) * g.s_r;
  }
  gptr<const T> xbase[NLX];
  bool xok[NLX];
#pragma unroll
  for (int x = 0; x < NLX; ++x) {
    const int cc = RIGHT ? tid / KC + RS * x : (tid & 63);
    const int cg = min(c0 + cc, ncat - 1);
    xok[x] = c0 + cc < ncat;
    const int z = cg / g.catn, n = cg - z * g.catn;
    xbase[x] = gmem(g.X) + (long long)z * g.x_z + (RIGHT ? (long long)n * g.x_r : (long long)n);
  }
  // raw values of the next chunk (zeroed out of range when stored to LDS,
  // so that no use of a load sits before the current chunk's products)
  T ps[NLS], px[NLX];
  auto gload = [&](int k0) {
    const int kSc = min(k0 + ks, g.K - 1);
#pragma unroll
    for (int x = 0; x < NLS; ++x) ps[x] = sbase[x][kSc];
#pragma unroll
    for (int x = 0; x < NLX; ++x) {
      const int kx = RIGHT ? k0 + ks : k0 + (tid >> 6) + 4 * x;
      const int kxc = min(kx, g.K - 1);
      px[x] = RIGHT ? xbase[x][kxc] : xbase[x][(long long)kxc * g.x_r];
    }
  };
  A4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = A4{0, 0, 0, 0};
  gload(0);
  for (int k0 = 0; k0 < g.K; k0 += KC) {
    __syncthreads();
    const bool kokS = k0 + ks < g.K;
#pragma unroll
    for (int x = 0; x < NLS; ++x)
      sS[(tid / KC + RS * x) * LDK + ks] = (ST)((sok[x] && kokS) ? ps[x] : (T)0);
#pragma unroll
    for (int x = 0; x < NLX; ++x) {
      const int cc = RIGHT ? tid / KC + RS * x : (tid & 63);
      const int kk = RIGHT ? ks : (tid >> 6) + 4 * x;
      sX[cc * LDK + kk] = (ST)((xok[x] && k0 + kk < g.K) ? px[x] : (T)0);
    }
    __syncthreads();
    if (k0 + KC < g.K) gload(k0 + KC);
#pragma unroll
    for (int k = 0; k < KC; k += KS) {
      if constexpr (!BF) {
        const T xf = sX[(16 * w + c) * LDK + k + q];
        T sf[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) sf[t] = sS[(16 * t + c) * LDK + k + q];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if constexpr (sizeof(T) == 8)
            acc[t] = RIGHT ? __builtin_amdgcn_mfma_f64_16x16x4f64(xf, sf[t], acc[t], 0, 0, 0)
                           : __builtin_amdgcn_mfma_f64_16x16x4f64(sf[t], xf, acc[t], 0, 0, 0);
          else
            acc[t] = RIGHT ? __builtin_amdgcn_mfma_f32_16x16x4f32(xf, sf[t], acc[t], 0, 0, 0)
                           : __builtin_amdgcn_mfma_f32_16x16x4f32(sf[t], xf, acc[t], 0, 0, 0);
        }
      } else {
        const mf_b8 xf = *(const mf_b8 *)&sX[(16 * w + c) * LDK + k + 8 * q];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const mf_b8 sf = *(const mf_b8 *)&sS[(16 * t + c) * LDK + k + 8 * q];
          acc[t] = RIGHT ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf, sf, acc[t], 0, 0, 0)
                         : __builtin_amdgcn_mfma_f32_16x16x32_bf16(sf, xf, acc[t], 0, 0, 0);
        }
      }
    }
  }
  // epilogue: accumulator (t, r) of lane (c, q) holds MFMA row mf_row(q, r)
  // and column c of tile t; the concatenated index of a lane does not
  // depend on t (left: column c; right: row mf_row(q, r))
  if constexpr (!RIGHT) {
    const int cg = c0 + 16 * w + c;
    if (cg >= ncat) return;
    const int z = cg / g.catn, n = cg - z * g.catn;
    const gptr<T> cb = gmem(g.C) + (long long)z * g.c_z + n;
    const gptr<const T> lam_r = gmem(g.lam_r), lam_c = gmem(g.lam_c);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int wide = 16 * t + mf_row<T>(q, r);
        if (wide >= g.wide) continue;
        const gptr<T> o = cb + (long long)wide * g.c_r;
        const T v = acc[t][r];
        if (g.mode == 0)
          *o = v;
        else if (g.mode == 1)
          *o = v / (g.sigma + lam_r[wide] + lam_c[n]);
        else
          *o += g.scale * v;
      }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cg = c0 + 16 * w + mf_row<T>(q, r);
      if (cg >= ncat) continue;
      const int z = cg / g.catn, n = cg - z * g.catn;
      const gptr<T> cb = gmem(g.C) + (long long)z * g.c_z + (long long)n * g.c_r;
      const gptr<const T> lam_c = gmem(g.lam_c);
      const T lr = g.mode == 1 ? g.sigma + gmem(g.lam_r)[n] : (T)0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int wide = 16 * t + c;
        if (wide >= g.wide) continue;
        const T v = acc[t][r];
        if (g.mode == 0)
          cb[wide] = v;
        else if (g.mode == 1)
          cb[wide] = v / (lr + lam_c[wide]);
        else
          cb[wide] += g.scale * v;
      }
    }
  }
}

// Rows row0..row0+63 of a dense symmetric matrix M (n x n, row-major) times
// the vector sr (LDS) with 1024 threads: wavefront w takes rows row0 + 4w ..
// row0 + 4w + 3, which are contiguous in M, its lanes striding along each row
// (every load one 256-byte segment); each row's 64 lane sums are added by a
// butterfly of fixed order.  spart: at least 64 values.
template <typename T>
__device__ inline T block_rows_matvec(const T *M, int n, int row0, const T *sr, T *spart) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const gptr<const T> Mg = gmem(M);
  gptr<const T> rowp[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) rowp[q] = Mg + (long long)min(row0 + 4 * w + q, n - 1) * n;
  T acc[4] = {0, 0, 0, 0};
#pragma unroll 2
  for (int j = lane; j < n; j += 64) {
    const T x = sr[j];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += rowp[q][j] * x;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T v = acc[q];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) spart[4 * w + q] = v;
  }
  __syncthreads();
  T y = 0;
  if (w == 0) y = spart[lane];
  return y;  // valid in wavefront 0 (rows past n: not to be stored)
}

// interface pieces: u[copies] += tau inv(P^T A P) r[piece];
// grid (right-hand side, piece, row block): the batch shares the inverse
template <typename T>
__global__ __launch_bounds__(1024) void piece_kernel(const PieceDev *pieces, const int *idx,
                                                     const int *cp, const int *cidx, const T *inv,
                                                     const T *r, T *u, T scale, long long vs) {
  extern __shared__ char smraw[];
  T *sm = (T *)smraw;
  __shared__ T spart[16 * 64];
  const PieceDev pc = pieces[blockIdx.y];
  const int n = pc.n;
  const int row0 = blockIdx.z * 64;
  if (row0 >= n) return;
  r += (long long)blockIdx.x * vs;
  u += (long long)blockIdx.x * vs;
  for (int j = threadIdx.x; j < n; j += blockDim.x) sm[j] = r[idx[pc.idx_off + j]];
  __syncthreads();
  const T y = block_rows_matvec<T>(inv + pc.inv_off, n, row0, sm, spart);
  const int i = row0 + (int)threadIdx.x;
  if (threadIdx.x < 64 && i < n)
    for (int c = cp[pc.cp_off + i]; c < cp[pc.cp_off + i + 1]; ++c) u[cidx[c]] += scale * y;
}

// Interface pieces of a float32 batch on the matrix cores: for each piece
// the products Y = inv R of its n x n inverse with the residual columns of
// 64 right-hand sides.  Block (64-row block, piece, group of 64 right-hand
// sides); k runs in chunks of PIECE_KC.  The chunk's rows of R are gathered
// through the piece's indices into LDS (row stride 65; thread t takes column
// t / 4 and rows t % 4 + 4m, every index and value load of the chunk in
// flight at once); wavefront w takes rows 16w.. of the block, its inverse
// operands for the chunk loaded straight into registers (one contiguous row
// segment per 16-lane row), and accumulates the four 16-column tiles of the
// group over k in a fixed order.  Each row then adds scale Y into its copies.
// Pieces of at most PIECE_MFMA_N unknowns (larger ones would gather R once
// per 64 rows).
constexpr int PIECE_MFMA_N = 1024, PIECE_KC = 120;
__global__ __launch_bounds__(256) void piece_mfma_kernel(const PieceDev *pieces, const int *idx,
                                                         const int *cp, const int *cidx,
                                                         const float *inv, const float *r,
                                                         float *u, float scale, long long vs,
                                                         int nrhs) {
  constexpr int LDR = 65, NJ = PIECE_KC / 4;
  __shared__ float sR[PIECE_KC * LDR];
  const PieceDev pc = pieces[blockIdx.y];
  const int n = pc.n;
  const int i0 = blockIdx.x * 64;
  if (i0 >= n) return;  // uniform over the block
  const int z0 = blockIdx.z * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = lane & 15, q = lane >> 4;
  const gptr<const int> gidx = gmem(idx) + pc.idx_off;
  const gptr<const float> gr = gmem(r);
  // this lane's inverse row (rows past n read row n - 1; their results are
  // not stored)
  const int arow = min(i0 + 16 * w + c, n - 1);
  const gptr<const float> ga = gmem(inv) + pc.inv_off + (long long)arow * n;
  const int gz = z0 + (tid >> 2), gj = tid & 3;  // gather column and first row
  const bool zok = gz < nrhs;
  const gptr<const float> grz = gr + (long long)(zok ? gz : 0) * vs;
  // scatter targets of this lane's four rows, loaded ahead of the products:
  // the copies e0 .. e1 - 1 of each row, the first one's torn index
  const gptr<const int> gcp = gmem(cp) + pc.cp_off, gcidx = gmem(cidx);
  int e0[4], e1[4], t0[4];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int i = i0 + 16 * w + mf_row<float>(q, rr);
    e0[rr] = i < n ? gcp[i] : 0;
    e1[rr] = i < n ? gcp[i + 1] : 0;
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) t0[rr] = e0[rr] < e1[rr] ? gcidx[e0[rr]] : -1;
  typename MfAcc<float>::type acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < n; k0 += PIECE_KC) {
    const int kn = min(PIECE_KC, n - k0);
    int ix[NJ];
    float rv[NJ], av[NJ];
#pragma unroll
    for (int m = 0; m < NJ; ++m) {
      const int jj = gj + 4 * m;
      ix[m] = gidx[k0 + min(jj, kn - 1)];
    }
#pragma unroll
    for (int m = 0; m < NJ; ++m) av[m] = ga[k0 + min(4 * m + q, kn - 1)];
#pragma unroll
    for (int m = 0; m < NJ; ++m) rv[m] = grz[ix[m]];
    __syncthreads();  // the previous chunk's R is consumed
#pragma unroll
    for (int m = 0; m < NJ; ++m) {
      const int jj = gj + 4 * m;
      sR[jj * LDR + (tid >> 2)] = (jj < kn && zok) ? rv[m] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NJ; ++m) {
      const float a = 4 * m + q < kn ? av[m] : 0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float b = sR[(4 * m + q) * LDR + 16 * t + c];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // first copies: every old value loaded before the stores (the rows and
  // right-hand sides of a block are distinct unknowns), then any further
  // copies of a row
  float uo[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int z = z0 + 16 * t + c;
    const gptr<float> uz = gmem(u) + (long long)(z < nrhs ? z : 0) * vs;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) uo[t][rr] = (z < nrhs && t0[rr] >= 0) ? uz[t0[rr]] : 0.0f;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int z = z0 + 16 * t + c;
    if (z >= nrhs) continue;
    const gptr<float> uz = gmem(u) + (long long)z * vs;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      if (t0[rr] < 0) continue;
      const float y = scale * acc[t][rr];
      uz[t0[rr]] = uo[t][rr] + y;
      for (int e = e0[rr] + 1; e < e1[rr]; ++e) uz[gcidx[e]] += y;
    }
  }
}

// Coarse solve in float64 whatever T: y = inv(A_0) g with g the sum of the
// copies of f, then y written to all copies.  The columns are split over
// gridDim.y blocks per row block (enough blocks to stream the dense inverse
// at full bandwidth); each writes its partial row sums, and the final kernel
// adds the splits in a fixed order (deterministic).
// grid (row block, column split, right-hand side)
template <typename T>
__global__ __launch_bounds__(1024) void coarse_partial_kernel(int n, const double *inv,
                                                              const int *cp, const int *cidx,
                                                              const T *f, double *part,
                                                              long long vs) {
  __shared__ double spart[16 * 64];
  extern __shared__ char smraw[];
  double *sm = (double *)smraw;  // gathered right-hand side of the column chunk
  const int nsplit = gridDim.y, split = blockIdx.y;
  const int chunk = (n + nsplit - 1) / nsplit;
  const int j0 = split * chunk, j1 = min(n, j0 + chunk);
  f += (long long)blockIdx.z * vs;
  for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) {
    double s = 0.0;
    for (int c = cp[j]; c < cp[j + 1]; ++c) s += (double)f[cidx[c]];
    sm[j - j0] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double s0 = 0.0, s1 = 0.0;
  if (i < n) {
    const double *col = inv + i;  // column i = row i (symmetric)
    int j = j0 + w;
    for (; j + 16 < j1; j += 32) {
      s0 += col[(long long)j * n] * sm[j - j0];
      s1 += col[(long long)(j + 16) * n] * sm[j + 16 - j0];
    }
    if (j < j1) s0 += col[(long long)j * n] * sm[j - j0];
  }
  spart[w * 64 + lane] = s0 + s1;
  __syncthreads();
  if (w == 0 && i < n) {
    double y = 0.0;
    for (int k = 0; k < 16; ++k) y += spart[k * 64 + lane];
    part[((long long)blockIdx.z * nsplit + split) * n + i] = y;
  }
}

template <typename T>
__global__ void coarse_final_kernel(int n, int nsplit, const double *part, const int *cp,
                                    const int *cidx, T *u, long long vs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  part += (long long)blockIdx.y * nsplit * n;
  u += (long long)blockIdx.y * vs;
  double y = 0.0;
  for (int k = 0; k < nsplit; ++k) y += part[(long long)k * n + i];
  for (int c = cp[i]; c < cp[i + 1]; ++c) u[cidx[c]] = (T)y;
}

// ---------------------------------------------------------------------------
// Transfers (2D), one output tile of 16 rows x TXO columns per block:
//   out[oy, ox] (+)= sum_a sum_b vy[oy][a] vx[ox][b] in[lo_y[oy] + a, lo_x[ox] + b]
// with the banded 1D factors (at most MAXW entries per output index).
// Restriction: in = w .* r on the fine patch, out = coarse residual (zero on
// Dirichlet rows), the band of coarse index j being column j of the 1D
// embedding; the coarse iterate is cleared alongside.  Prolongation: in = the
// coarse correction, out = fine iterate += (free rows only).  The tile's
// input window (at most WYM x WXM values) is staged in LDS in one round of
// loads over its actual extent (consecutive threads along its rows), then
// contracted in x and in y; a tile row of TXO outputs is one contiguous
// segment.  grid.x = right-hand side, grid.y = tile.
// ---------------------------------------------------------------------------
constexpr int MAXW = 12;
constexpr int XTY = 16;

template <typename T, bool RESTRICT, int TXO, int WXM, int WYM>
__global__ __launch_bounds__(256) void transfer2d_kernel(
    const XferTile *tiles, const int *__restrict__ lo, const T *__restrict__ val, int W,
    const T *__restrict__ in, const T *__restrict__ win, const unsigned char *__restrict__ mask_out,
    T *out, T *zero_out, long long vs_in, long long vs_out) {
  constexpr int NL = (WXM * WYM + 255) / 256;  // window loads per thread
  __shared__ T sIn[WYM * WXM];
  __shared__ T sX[WYM * TXO];
  // x band values [entry][output column]: the lanes of the x contraction
  // (consecutive columns) read consecutive banks
  __shared__ T sVx[MAXW][TXO], sVy[XTY][MAXW];
  __shared__ int sLox[TXO], sLoy[XTY];
  const XferTile tl = tiles[blockIdx.y];
  in += (long long)blockIdx.x * vs_in;
  out += (long long)blockIdx.x * vs_out;
  if (zero_out) zero_out += (long long)blockIdx.x * vs_out;
  const int tid = threadIdx.x;
  const int wxn = tl.wn[0], wyn = tl.wn[1], nwin = wxn * wyn;
  // one round of independent loads: window element e = (row e / wxn,
  // column e % wxn), band starts and values
  T wv[NL];
  int wo[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int e = tid + 256 * j, r = e / wxn, cc = e - r * wxn;
    const bool ok = e < nwin;
    const long long t = tl.in_off + (long long)(tl.w0[1] + r) * tl.in_nx + tl.w0[0] + cc;
    T v = ok ? in[t] : (T)0;
    if (RESTRICT && ok) v *= win[t];
    wv[j] = v;
    wo[j] = ok ? r * WXM + cc : -1;
  }
  // the tile's outputs of this thread: masks, and for the prolongation the
  // old values, loaded with the window
  constexpr int NO = XTY * TXO / 256;
  long long ot[NO];
  bool om[NO];
  T uo[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int e = tid + 256 * k, tx = e % TXO, ty = e / TXO;
    const bool in_tile = tx < tl.no[0] && ty < tl.no[1];
    ot[k] = in_tile ? tl.out_off + (long long)(tl.o0[1] + ty) * tl.out_nx + tl.o0[0] + tx : -1;
    om[k] = in_tile && mask_out[ot[k]];
    uo[k] = (!RESTRICT && om[k]) ? out[ot[k]] : (T)0;
  }
  if (tid < TXO + XTY) {
    // per-direction fields selected without indexing the record by a lane value
    const int g = tid < TXO ? 0 : 1, o = g ? tid - TXO : tid;
    const int no = g ? tl.no[1] : tl.no[0];
    const int row = (g ? tl.base[1] : tl.base[0]) + min(o, no - 1);
    const int l0 = lo[row] - (g ? tl.w0[1] : tl.w0[0]);
    if (g)
      sLoy[o] = l0;
    else
      sLox[o] = l0;
#pragma unroll
    for (int a = 0; a < MAXW; ++a) {
      const T v = (a < W && o < no) ? val[(long long)row * W + a] : (T)0;
      if (g)
        sVy[o][a] = v;
      else
        sVx[a][o] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < NL; ++j)
    if (wo[j] >= 0) sIn[wo[j]] = wv[j];
  __syncthreads();
  // contractions in groups of four band entries whose reads go out
  // together: band values are zero past each row's band and past the patch
  // (where the window is cut), so reads there are clamped into the window
  // and add exact zeros (the sums are those of the band entries in order)
  for (int e = tid; e < wyn * TXO; e += 256) {
    const int r = e / TXO, ox = e % TXO;
    const int b0 = sLox[ox];
    T sx = 0;
#pragma unroll
    for (int bc = 0; bc < MAXW; bc += 4)
      if (bc < W) {
        T cf[4], v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cf[j] = sVx[bc + j][ox];
          v[j] = sIn[r * WXM + min(b0 + bc + j, wxn - 1)];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) sx += cf[j] * v[j];
      }
    sX[r * TXO + ox] = sx;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int e = tid + 256 * k, tx = e % TXO, ty = e / TXO;
    if (ot[k] >= 0) {
      const int a0 = sLoy[ty];
      T sy = 0;
#pragma unroll
      for (int ac = 0; ac < MAXW; ac += 4)
        if (ac < W) {
          T cf[4], v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cf[j] = sVy[ty][ac + j];
            v[j] = sX[min(a0 + ac + j, wyn - 1) * TXO + tx];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) sy += cf[j] * v[j];
        }
      const long long t = ot[k];
      if (RESTRICT) {
        out[t] = om[k] ? sy : (T)0;
        if (zero_out) zero_out[t] = 0;
      } else if (om[k]) {
        out[t] = uo[k] + sy;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// compact <-> torn (grid.y = right-hand side)
// ---------------------------------------------------------------------------
__global__ void scatter_compact_kernel(const double *xc, long long N, const int *cp, const int *cidx,
                                       double *xt, long long nt) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= N) return;
  xc += (long long)blockIdx.y * N;
  xt += (long long)blockIdx.y * nt;
  double v = xc[i];
  for (int c = cp[i]; c < cp[i + 1]; ++c) xt[cidx[c]] = v;
}

__global__ void gather_compact_kernel(const double *xt, long long N, const int *cp, const int *cidx,
                                      int sum, double *xc, long long nt) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= N) return;
  xc += (long long)blockIdx.y * N;
  xt += (long long)blockIdx.y * nt;
  if (!sum) {
    xc[i] = xt[cidx[cp[i]]];
    return;
  }
  double s = 0.0;
  for (int c = cp[i]; c < cp[i + 1]; ++c) s += xt[cidx[c]];
  xc[i] = s;
}

// ---------------------------------------------------------------------------
// deterministic reductions: fixed grid, fixed-order trees.  Partials of
// right-hand side j sit at part[j * RED_BLOCKS ...]; the final kernels run
// one block per right-hand side.
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// vectors of type T (float64, or the float32 inner iteration of the
// refinement), sums in float64
template <typename T>
__global__ __launch_bounds__(256) void dot_partial_kernel(const T *a, const T *b,
                                                          const double *w, long long n,
                                                          double *part) {
  __shared__ double sh[256];
  a += (long long)blockIdx.y * n;
  b += (long long)blockIdx.y * n;
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    s += (w ? w[i] : 1.0) * (double)a[i] * (double)b[i];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// mode 0: scal[slot] = sum; 1: alpha = rz / sum; 2: beta = sum / rz, rz = sum
__global__ __launch_bounds__(256) void dot_final_kernel(const double *part, int nb, double *scal,
                                                        int slot, int mode) {
  __shared__ double sh[256];
  part += (long long)blockIdx.x * nb;
  scal += (long long)blockIdx.x * S_COUNT;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) {
    scal[slot] = t;
    if (mode == 1) scal[S_ALPHA] = scal[S_RZ] / t;
    if (mode == 2) {
      scal[S_BETA] = t / scal[S_RZ];
      scal[S_RZ] = t;
    }
  }
}

// flexible CG (Polak-Ribiere form): partial sums of (z, r) and (z, r_old)
__global__ __launch_bounds__(256) void dot2_partial_kernel(const double *z, const double *r,
                                                           const double *ro, const double *w,
                                                           long long n, double *part) {
  __shared__ double sh[256];
  const long long zo = (long long)blockIdx.y * n;
  double s1 = 0.0, s2 = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double zw = (w ? w[i] : 1.0) * z[zo + i];
    s1 += zw * r[zo + i];
    s2 += zw * ro[zo + i];
  }
  double t1 = block_sum(s1, sh);
  double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    const long long k = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * k] = t1;
    part[2 * k + 1] = t2;
  }
}

__global__ __launch_bounds__(256) void dot2_final_kernel(const double *part, int nb, double *scal) {
  __shared__ double sh[256];
  part += (long long)blockIdx.x * nb * 2;
  scal += (long long)blockIdx.x * S_COUNT;
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s1 += part[2 * i];
    s2 += part[2 * i + 1];
  }
  double t1 = block_sum(s1, sh);
  double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    scal[S_BETA] = (t1 - t2) / scal[S_RZ];
    scal[S_RZ] = t1;
    scal[S_ZRO] = t2;
  }
}

// x += alpha p, r -= alpha q on the right-hand sides still iterating (r_old
// keeps r before the update when given); ||r||_w^2 partials for all; z = 0.
// Vectors of type T, scalars and sums in float64 (each update rounded once).
template <typename T>
__global__ __launch_bounds__(256) void pcg_xr_kernel(T *x, T *r, const T *p, const T *q,
                                                     const double *w, long long n,
                                                     const double *scal, double *part,
                                                     T *z_zero, T *rold, const int *active) {
  __shared__ double sh[256];
  const int j = blockIdx.y;
  const long long zo = (long long)j * n;
  const bool act = active[j] != 0;
  const double alpha = scal[(long long)j * S_COUNT + S_ALPHA];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    z_zero[zo + i] = (T)0;
    double ri = r[zo + i];
    if (act) {
      if (rold) rold[zo + i] = (T)ri;
      x[zo + i] = (T)(x[zo + i] + alpha * p[zo + i]);
      ri = (double)(T)(ri - alpha * q[zo + i]);
      r[zo + i] = (T)ri;
    }
    s += (w ? w[i] : 1.0) * ri * ri;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[(long long)j * gridDim.x + blockIdx.x] = t;
}

template <typename T>
__global__ void pcg_p_kernel(T *p, const T *z, long long n, const double *scal,
                             const int *active) {
  const int j = blockIdx.y;
  if (!active[j]) return;
  const long long zo = (long long)j * n;
  const double beta = scal[(long long)j * S_COUNT + S_BETA];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[zo + i] = (T)(z[zo + i] + beta * p[zo + i]);
}

template <typename T>
__global__ void add_active_kernel(double *y, const T *x, long long n, const int *active) {
  const int j = blockIdx.y;
  if (!active[j]) return;
  const long long zo = (long long)j * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[zo + i] += x[zo + i];
}

// ---------------------------------------------------------------------------
// Setup: in-place inverse of a dense symmetric positive definite matrix by
// blocked Gauss-Jordan elimination without pivoting (the Schur complements of
// an SPD matrix stay SPD).  For pivot block k with P = inv(A_kk):
//   A_kj <- P A_kj,  A_ij <- A_ij - A_ik A_kj (new),  A_ik <- -A_ik P,  A_kk <- P
// (i, j outside block k); after the last block A holds inv(A).  Row-major
// n x n, leading dimension n.
// ---------------------------------------------------------------------------
constexpr int GJB = 32;

// Matrix z of a batch: A = base + offs[z] with order ns[z] (offs == null:
// one matrix of order n1 at base); false when step k0 is past its order.
__device__ inline bool gj_matrix(double *base, const long long *offs, const int *ns, int n1,
                                 int k0, double *&A, int &n, int &nb) {
  if (offs) {
    A = base + offs[blockIdx.z];
    n = ns[blockIdx.z];
  } else {
    A = base;
    n = n1;
  }
  nb = min(GJB, n - k0);
  return k0 < n;
}

// scalar Gauss-Jordan on the diagonal block (1024 threads = 32 x 32)
__global__ __launch_bounds__(1024) void gj_diag_kernel(double *base, const long long *offs,
                                                       const int *ns, int n1, int k0,
                                                       int *bad) {
  double *A;
  int n, nb;
  if (!gj_matrix(base, offs, ns, n1, k0, A, n, nb)) return;
  __shared__ double S[GJB][GJB + 1];
  const int c = threadIdx.x % GJB, r = threadIdx.x / GJB;
  const bool in = r < nb && c < nb;
  S[r][c] = in ? A[(long long)(k0 + r) * n + k0 + c] : (r == c ? 1.0 : 0.0);
  __syncthreads();
  for (int t = 0; t < nb; ++t) {
    const double att = S[t][t];
    if (threadIdx.x == 0 && !(att > 0.0)) bad[0] = 1;
    const double piv = 1.0 / att;
    const double art = S[r][t], atc = S[t][c], arc = S[r][c];
    __syncthreads();
    double v;
    if (r == t && c == t)
      v = piv;
    else if (r == t)
      v = atc * piv;
    else if (c == t)
      v = -art * piv;
    else
      v = arc - art * atc * piv;
    S[r][c] = v;
    __syncthreads();
  }
  if (in) A[(long long)(k0 + r) * n + k0 + c] = S[r][c];
}

// A_kj <- P A_kj for every column j outside the block (one thread per column)
__global__ __launch_bounds__(256) void gj_row_kernel(double *base, const long long *offs,
                                                     const int *ns, int n1, int k0) {
  double *A;
  int n, nb;
  if (!gj_matrix(base, offs, ns, n1, k0, A, n, nb)) return;
  if (blockIdx.x * blockDim.x >= (unsigned)n) return;
  __shared__ double P[GJB][GJB];
  for (int e = threadIdx.x; e < GJB * GJB; e += blockDim.x) {
    const int r = e / GJB, c = e % GJB;
    P[r][c] = (r < nb && c < nb) ? A[(long long)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + nb)) return;
  double col[GJB];
#pragma unroll
  for (int t = 0; t < GJB; ++t) col[t] = t < nb ? A[(long long)(k0 + t) * n + j] : 0.0;
#pragma unroll 4
  for (int r = 0; r < nb; ++r) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < GJB; ++t) s += P[r][t] * col[t];
    A[(long long)(k0 + r) * n + j] = s;
  }
}

// A_ij <- A_ij - A_ik A_kj for i, j outside the block: 64 x 64 tiles, each
// thread 4 x 4 entries, inner dimension nb <= 32 staged in LDS
__global__ __launch_bounds__(256) void gj_update_kernel(double *base, const long long *offs,
                                                        const int *ns, int n1, int k0) {
  double *A;
  int n, nb;
  if (!gj_matrix(base, offs, ns, n1, k0, A, n, nb)) return;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  if (i0 >= n || j0 >= n) return;
  __shared__ double Ci[64][GJB + 1];  // A_ik rows of the tile
  __shared__ double Rj[GJB][64 + 1];  // A_kj columns of the tile
  for (int e = threadIdx.x; e < 64 * GJB; e += blockDim.x) {
    const int a = e / GJB, t = e % GJB;
    const int i = i0 + a;
    Ci[a][t] = (i < n && t < nb) ? A[(long long)i * n + k0 + t] : 0.0;
    const int t2 = e / 64, b = e % 64;
    const int j = j0 + b;
    Rj[t2][b] = (j < n && t2 < nb) ? A[(long long)(k0 + t2) * n + j] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int t = 0; t < nb; ++t) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Ci[ty + 16 * u][t];
      b[u] = Rj[t][tx + 16 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= n || (i >= k0 && i < k0 + nb)) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j >= n || (j >= k0 && j < k0 + nb)) continue;
      A[(long long)i * n + j] -= acc[u][v];
    }
  }
}

// A_ik <- -A_ik P for every row i outside the block (one thread per row)
__global__ __launch_bounds__(256) void gj_col_kernel(double *base, const long long *offs,
                                                     const int *ns, int n1, int k0) {
  double *A;
  int n, nb;
  if (!gj_matrix(base, offs, ns, n1, k0, A, n, nb)) return;
  if (blockIdx.x * blockDim.x >= (unsigned)n) return;
  __shared__ double P[GJB][GJB];
  for (int e = threadIdx.x; e < GJB * GJB; e += blockDim.x) {
    const int r = e / GJB, c = e % GJB;
    P[r][c] = (r < nb && c < nb) ? A[(long long)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (i >= k0 && i < k0 + nb)) return;
  double row[GJB];
#pragma unroll
  for (int t = 0; t < GJB; ++t) row[t] = t < nb ? A[(long long)i * n + k0 + t] : 0.0;
#pragma unroll 4
  for (int c = 0; c < nb; ++c) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < GJB; ++t) s += row[t] * P[t][c];
    A[(long long)i * n + k0 + c] = -s;
  }
}

__global__ void gather_rows_kernel(const double *st, int SP, const int *rows, int nrows,
                                   double *out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)nrows * SP) return;
  const int r = (int)(e / SP), o = (int)(e % SP);
  out[e] = st[(long long)rows[r] * SP + o];
}

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
template <typename T>
void k_fill(T *x, T v, long long n, hipStream_t s) {
  fill_kernel<T><<<std::min<unsigned>(nblocks(n), 4096), BS, 0, s>>>(x, v, n);
}
template void k_fill<double>(double *, double, long long, hipStream_t);
template void k_fill<float>(float *, float, long long, hipStream_t);
template void k_fill<int>(int *, int, long long, hipStream_t);

template <typename Ti, typename To>
void k_convert(const Ti *x, const To *w, To *y, long long n, int nrhs, hipStream_t s, To *zero,
               const int *active) {
  dim3 grid(std::min<unsigned>(nblocks(n), 2048), nrhs);
  convert_kernel<Ti, To><<<grid, BS, 0, s>>>(x, w, y, n, zero, active);
}
template void k_convert<double, double>(const double *, const double *, double *, long long, int,
                                        hipStream_t, double *, const int *);
template void k_convert<double, float>(const double *, const float *, float *, long long, int,
                                       hipStream_t, float *, const int *);
template void k_convert<float, double>(const float *, const double *, double *, long long, int,
                                       hipStream_t, double *, const int *);
template void k_convert<float, float>(const float *, const float *, float *, long long, int,
                                      hipStream_t, float *, const int *);

int stencil_tile_2d(int p) { return p <= 3 ? 8 : 4; }

template <int P, int RT>
static void launch_stencil2d(Context &c, LevelData &L, double *out, int first, int count,
                             int SP) {
  stencil2d_kernel<P, RT><<<count, 256, 0, c.stream>>>(L.d_stiles + first, L.d_pd, L.d_tabB,
                                                       L.d_tabD, rule_of(P + 1), out, SP, c.p);
}

// element matrices of at most this many bytes at a time (z slabs of a patch)
constexpr size_t ASSEMBLE3D_SCRATCH = (size_t)2 << 30;

// rows of the patches of degree P (element matrices with P+1 Gauss points
// per direction), written in the level's layout of row stride SP
template <int P>
static void assemble3d(Context &c, LevelData &L, double *out, int SP) {
  constexpr int P1 = P + 1, NB = P1 * P1 * P1;
  const size_t per_el = (size_t)NB * NB * sizeof(double);
  // rows per slab: the slab's element layers (rows + P) fit the scratch
  std::vector<int> rows_per(L.K);
  size_t cap = 0;
  for (int k = 0; k < L.K; ++k) {
    const PatchDev &pt = L.pd[k];
    if (pt.p != P) continue;
    const size_t layer = (size_t)pt.nel[0] * pt.nel[1] * per_el;
    const int fit = (int)std::max<size_t>(1, ASSEMBLE3D_SCRATCH / layer);
    const int R = std::max(1, fit - P);
    rows_per[k] = R;
    cap = std::max(cap, (size_t)std::min(pt.nel[2], R + P) * layer);
  }
  DeviceScratch ke;
  double *Ke = ke.alloc<double>(cap / sizeof(double));
  if (cap == 0) return;
  for (int k = 0; k < L.K; ++k) {
    const PatchDev &pt = L.pd[k];
    if (pt.p != P) continue;
    for (int iz0 = 0; iz0 < pt.n[2]; iz0 += rows_per[k]) {
      const int iz1 = std::min(pt.n[2], iz0 + rows_per[k]);
      const int ez0 = std::max(0, iz0 - P), ez1 = std::min(pt.nel[2] - 1, iz1 - 1);
      const long long nel = (long long)pt.nel[0] * pt.nel[1] * (ez1 - ez0 + 1);
      elem3d_kernel<P><<<(unsigned)nel, 256, 0, c.stream>>>(L.d_pd, k, ez0, L.d_tabB, L.d_tabD,
                                                            rule_of(P + 1), Ke);
      const long long n = (long long)pt.n[0] * pt.n[1] * (iz1 - iz0) * SP;
      gather3d_kernel<P><<<nblocks(n), 256, 0, c.stream>>>(L.d_pd, k, iz0, iz1, ez0, Ke, out, SP,
                                                           c.p);
    }
  }
  HIPCHK(hipStreamSynchronize(c.stream));  // the scratch is freed at scope exit
}

void k_stencil_assemble(Context &c, LevelData &L, double *out) {
  int S = 1;
  for (int d = 0; d < c.d; ++d) S *= (2 * c.p + 1);
  const int SP = (S + 15) / 16 * 16;  // row stride: the level's largest degree
  long long tot = L.Ntorn * SP;
  if (c.d == 2) {
    // one launch per patch degree (tiles grouped by degree)
    for (const auto &g : L.sgroups) {
      switch (g[0]) {
        case 1: launch_stencil2d<1, 8>(c, L, out, g[1], g[2], SP); break;
        case 2: launch_stencil2d<2, 8>(c, L, out, g[1], g[2], SP); break;
        case 3: launch_stencil2d<3, 8>(c, L, out, g[1], g[2], SP); break;
        case 4: launch_stencil2d<4, 4>(c, L, out, g[1], g[2], SP); break;
        case 5: launch_stencil2d<5, 4>(c, L, out, g[1], g[2], SP); break;
        case 6: launch_stencil2d<6, 4>(c, L, out, g[1], g[2], SP); break;
        case 7: launch_stencil2d<7, 4>(c, L, out, g[1], g[2], SP); break;
        case 8: launch_stencil2d<8, 4>(c, L, out, g[1], g[2], SP); break;
        default: fail(IGAMG_EUNSUPPORTED, "degree out of range");
      }
    }
  } else if (c.arena.region || c.p > 4) {
    // inside a lent region (no scratch allocation): per-entry quadrature
    if (c.mixed) fail(IGAMG_EUNSUPPORTED, "3D rows of mixed degrees inside a lent region");
    stencil_kernel<3><<<nblocks(tot), BS, 0, c.stream>>>(L.d_pd, L.K, L.d_tabB, L.d_tabD, c.gr, c.p,
                                                         L.Ntorn, out);
  } else {
    // one pass per degree present (each over its patches)
    assemble3d<1>(c, L, out, SP);
    assemble3d<2>(c, L, out, SP);
    assemble3d<3>(c, L, out, SP);
    assemble3d<4>(c, L, out, SP);
  }
  HIPCHK(hipGetLastError());
}

void k_stencil_add(const int *rows, const int *slots, const double *vals, int n, double *stencil,
                   int S, hipStream_t s) {
  if (n == 0) return;
  stencil_add_kernel<<<nblocks(n), BS, 0, s>>>(rows, slots, vals, n, stencil, S);
}

void k_invdiag(const double *stencil, int S, int center, const unsigned char *mask, double *invd,
               long long n, hipStream_t s) {
  invdiag_kernel<<<nblocks(n), BS, 0, s>>>(stencil, S, center, mask, invd, n);
}

void k_load_manufactured(Context &c, LevelData &L, double *out) {
  if (c.d == 2)
    load_kernel<2><<<nblocks(L.Ntorn), BS, 0, c.stream>>>(L.d_pd, L.K, L.d_tabB, c.d_rules,
                                                          L.d_mask, L.Ntorn, out);
  else
    load_kernel<3><<<nblocks(L.Ntorn), BS, 0, c.stream>>>(L.d_pd, L.K, L.d_tabB, c.d_rules,
                                                          L.d_mask, L.Ntorn, out);
}

long long l2_error_partials(long long nel) { return (nel + BS - 1) / BS; }

void k_l2_error(Context &c, LevelData &L, const double *ut, const long long *el_off,
                const int *tab, const double *tB, const GaussRule &gq, double *part,
                long long nel, double *out) {
  const long long nb = l2_error_partials(nel);
  if (nb > 65535LL * 64) fail(IGAMG_EUNSUPPORTED, "too many elements for the L2 error kernel");
  if (c.d == 2)
    l2err_kernel<2><<<(unsigned)nb, BS, 0, c.stream>>>(L.d_pd, L.K, el_off, tab, tB, gq, c.p, ut,
                                                       part);
  else
    l2err_kernel<3><<<(unsigned)nb, BS, 0, c.stream>>>(L.d_pd, L.K, el_off, tab, tB, gq, c.p, ut,
                                                       part);
  sum_fixed_kernel<<<1, 1024, 0, c.stream>>>(part, nb, out);
  HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free entry points (igamg_l2_error_noalloc):
// one array per GPU, held until the process ends.  In host code the array's
// name is a host-side stand-in, not a device address; host code uses only
// the address hipGetSymbolAddress returns for the current device, looked up
// once per device and kept in noalloc_addr.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex noalloc_mu;
std::map<int, void *> noalloc_addr;
}  // namespace

void *noalloc_scratch_init() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(noalloc_mu);
  auto it = noalloc_addr.find(dev);
  if (it != noalloc_addr.end()) return it->second;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    fail(IGAMG_EHIP, std::string("hipGetSymbolAddress of the device scratch failed: ") +
                         hipGetErrorString(e));
  noalloc_addr[dev] = ptr;
  return ptr;
}

void *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(noalloc_mu);
  auto it = noalloc_addr.find(device);
  return it == noalloc_addr.end() ? nullptr : it->second;
}

template <typename T>
void k_iface_apply(Context &c, LevelData &L, const T *u, const T *f, const T *fw, T beta, T alpha,
                   T *r, int nrhs) {
  TimeScope ts(c, "iface_apply", L.l);
  const int nb_plain = (int)nblocks(L.Ntorn);
  const int nb_rows = (L.n_if_rows + 15) / 16;
  dim3 grid(nrhs, nb_plain + nb_rows);
  iface_kernel<T><<<grid, BS, 0, c.stream>>>(L.Ntorn, nb_plain, L.d_mask, L.d_has_if, L.d_if_rows,
                                             L.n_if_rows, L.d_if_ptr, L.d_if_col,
                                             L.arr<T>().if_val, u, f, fw, beta, alpha, r);
}
template void k_iface_apply<double>(Context &, LevelData &, const double *, const double *,
                                    const double *, double, double, double *, int);
template void k_iface_apply<float>(Context &, LevelData &, const float *, const float *,
                                   const float *, float, float, float *, int);

int vol_tile_2d(int p) { return p <= 4 ? 8 : (p <= 6 ? 6 : 4); }

// one right-hand side per block, the metric evaluated on the fly (measured
// faster for batches too than sharing a stored metric across several
// right-hand sides per block, which costs parallelism)
template <typename T, int P, int TE>
static void launch_vol2d(Context &c, LevelData &L, const T *u, T *r, T alpha, int nrhs, int first,
                         int count) {
  vol2d_kernel<T, P, TE, 1><<<dim3(nrhs, count), 256, 0, c.stream>>>(
      L.d_optiles + first, L.d_tabB, L.d_tabD, rule_of(P + 1), u, r, L.d_mask, alpha, L.Ntorn,
      nrhs);
}

template <typename T, int P>
static void launch_vol3d(Context &c, LevelData &L, const T *u, T *r, T alpha, int nrhs, int first,
                         int count) {
  vol3d_kernel<T, P, VOL3D_TILE><<<dim3(count, nrhs), 256, 0, c.stream>>>(
      L.d_vtiles + first, L.d_pd, L.d_tabB, L.d_tabD, rule_of(P + 1), u, r, L.d_mask, alpha,
      L.Ntorn);
}

template <typename T>
void k_vol_apply(Context &c, LevelData &L, const T *u, T *r, T alpha, int nrhs) {
  TimeScope ts(c, "vol_apply", L.l);
  // one launch per (patch degree, colour class of tiles): the outputs of one
  // launch are disjoint, the classes run in a fixed order on the stream
  if (c.d == 3) {
    for (const auto &g : L.vgroups) switch (g[0]) {
        case 1: launch_vol3d<T, 1>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
        case 2: launch_vol3d<T, 2>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
        case 3: launch_vol3d<T, 3>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
        case 4: launch_vol3d<T, 4>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
        default: fail(IGAMG_EUNSUPPORTED, "3D degree out of range 1..4");
      }
    return;
  }
  for (const auto &g : L.vgroups) {
    switch (g[0]) {
      case 1: launch_vol2d<T, 1, 8>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 2: launch_vol2d<T, 2, 8>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 3: launch_vol2d<T, 3, 8>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 4: launch_vol2d<T, 4, 8>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 5: launch_vol2d<T, 5, 6>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 6: launch_vol2d<T, 6, 6>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 7: launch_vol2d<T, 7, 4>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      case 8: launch_vol2d<T, 8, 4>(c, L, u, r, alpha, nrhs, g[1], g[2]); break;
      default: fail(IGAMG_EUNSUPPORTED, "degree out of range");
    }
  }
}
template void k_vol_apply<double>(Context &, LevelData &, const double *, double *, double, int);
template void k_vol_apply<float>(Context &, LevelData &, const float *, float *, float, int);

template <typename T>
void k_glue_sum(LevelData &L, T *y, int nrhs, hipStream_t s) {
  if (L.n_glue == 0) return;
  dim3 grid(nblocks(L.n_glue), nrhs);
  glue_kernel<T><<<grid, BS, 0, s>>>(L.n_glue, L.d_glue_ptr, L.d_glue_idx, y, L.Ntorn);
}
template void k_glue_sum<double>(LevelData &, double *, int, hipStream_t);
template void k_glue_sum<float>(LevelData &, float *, int, hipStream_t);

template <typename T, int P, int RBW, int NR, bool BWD>
static void launch_gs2d_dir(Context &c, LevelData &L, const GsClass &cl, int nrhs) {
  LevelArrays<T> &A = L.arr<T>();
  const int ngroups = (nrhs + RBW * NR - 1) / (RBW * NR);
  const long long nblk = ((long long)ngroups * cl.count + 7) / 8 * 8;
  gs2d_wave_kernel<T, P, RBW, NR, BWD><<<(unsigned)nblk, 64 * RBW, 0, c.stream>>>(
      cl.tiles, cl.count, ngroups, A.stencil, A.invdiag, L.d_gcx_li, L.d_gcx_col, A.gcx_val,
      L.d_mr_li, L.d_mr_dst, A.f, A.u, L.Ntorn, nrhs);
}

// the sweep direction is a template parameter: the unrolled class steps then
// address their rows with compile-time offsets
#ifndef GS2D_NR
#define GS2D_NR 2
#endif
#ifndef GS2D_RBW
#define GS2D_RBW 2
#endif
template <typename T, int P>
static void launch_gs2d(Context &c, LevelData &L, const GsClass &cl, bool backward, int nrhs) {
  // one right-hand side: one wavefront per tile; batches: GS2D_NR right-hand
  // sides per wavefront, GS2D_RBW wavefronts of a tile per block
  if (nrhs == 1) {
    if (backward)
      launch_gs2d_dir<T, P, 1, 1, true>(c, L, cl, nrhs);
    else
      launch_gs2d_dir<T, P, 1, 1, false>(c, L, cl, nrhs);
  } else {
    if (backward)
      launch_gs2d_dir<T, P, GS2D_RBW, GS2D_NR, true>(c, L, cl, nrhs);
    else
      launch_gs2d_dir<T, P, GS2D_RBW, GS2D_NR, false>(c, L, cl, nrhs);
  }
}

template <typename T, int P>
static void launch_gs3d(Context &c, LevelData &L, const GsClass &cl, bool backward, int nrhs) {
  LevelArrays<T> &A = L.arr<T>();
  if (backward)
    gs3d_kernel<T, P, true><<<dim3(nrhs, cl.count), 512, 0, c.stream>>>(
        cl.tiles3, A.stencil, A.invdiag, A.xsum, L.d_mr_li, L.d_mr_dst, A.f, A.u, L.Ntorn);
  else
    gs3d_kernel<T, P, false><<<dim3(nrhs, cl.count), 512, 0, c.stream>>>(
        cl.tiles3, A.stencil, A.invdiag, A.xsum, L.d_mr_li, L.d_mr_dst, A.f, A.u, L.Ntorn);
}

// couplings of the coupled rows r0 .. r1 (CSR order): xs = X u, or out +=
// alpha mask X u
template <typename T>
static void launch_cross3d(Context &c, LevelData &L, const T *val, int r0, int r1, const T *u,
                           T *out, bool add, T alpha, int nrhs) {
  if (r1 <= r0) return;
  dim3 grid((unsigned)((r1 - r0 + 255) / 256), nrhs);
  if (add)
    cross3d_kernel<T, true><<<grid, 256, 0, c.stream>>>(L.d_x_rows, L.d_x_ptr, L.d_x_col, val, r0,
                                                        r1, L.d_mask, u, out, alpha, L.Ntorn);
  else
    cross3d_kernel<T, false><<<grid, 256, 0, c.stream>>>(L.d_x_rows, L.d_x_ptr, L.d_x_col, val, r0,
                                                         r1, L.d_mask, u, out, alpha, L.Ntorn);
}

template <typename T>
void k_gs_sweep(Context &c, LevelData &L, bool backward, int nrhs) {
  // one event pair around the sweep (its class launches run back to back)
  TimeScope ts(c, "gauss_seidel", L.l);
  ts.n = 0;
  if (c.opt.discretization == IGAMG_CONFORMING && L.n_glue > 0) {
    glue_first_kernel<T><<<dim3(nblocks(L.n_glue), nrhs), BS, 0, c.stream>>>(
        L.n_glue, L.d_glue_ptr, L.d_glue_idx, L.arr<T>().f, L.Ntorn);
    ++ts.n;
  }
  int nc = (int)L.gs.size();
  for (int ii = 0; ii < nc; ++ii) {
    const int ci = backward ? nc - 1 - ii : ii;
    const GsClass &cl = L.gs[ci];
    if (c.d == 3 && ci % 8 == (backward ? 7 : 0)) {
      // first class of a patch colour: its rows' cross couplings
      LevelArrays<T> &A = L.arr<T>();
      const int colr = ci / 8;
      launch_cross3d<T>(c, L, A.x_val, L.x_cptr[colr], L.x_cptr[colr + 1], A.u, A.xsum, false,
                        (T)0, nrhs);
    }
    if (cl.count == 0) continue;
    ++ts.n;
    if (c.d == 3) {
      switch (c.p) {
        case 1: launch_gs3d<T, 1>(c, L, cl, backward, nrhs); break;
        case 2: launch_gs3d<T, 2>(c, L, cl, backward, nrhs); break;
        case 3: launch_gs3d<T, 3>(c, L, cl, backward, nrhs); break;
        case 4: launch_gs3d<T, 4>(c, L, cl, backward, nrhs); break;
        default: fail(IGAMG_EUNSUPPORTED, "3D degree out of range 1..4");
      }
      continue;
    }
    switch (c.p) {
      case 1: launch_gs2d<T, 1>(c, L, cl, backward, nrhs); break;
      case 2: launch_gs2d<T, 2>(c, L, cl, backward, nrhs); break;
      case 3: launch_gs2d<T, 3>(c, L, cl, backward, nrhs); break;
      case 4: launch_gs2d<T, 4>(c, L, cl, backward, nrhs); break;
      case 5: launch_gs2d<T, 5>(c, L, cl, backward, nrhs); break;
      case 6: launch_gs2d<T, 6>(c, L, cl, backward, nrhs); break;
      case 7: launch_gs2d<T, 7>(c, L, cl, backward, nrhs); break;
      case 8: launch_gs2d<T, 8>(c, L, cl, backward, nrhs); break;
      default: fail(IGAMG_EUNSUPPORTED, "degree out of range");
    }
  }
}
template void k_gs_sweep<double>(Context &, LevelData &, bool, int);
template void k_gs_sweep<float>(Context &, LevelData &, bool, int);

template <typename T, int P, int RB>
static void launch_sp2d(Context &c, LevelData &L, const LevelArrays<T> &A, const T *u, const T *f,
                        const T *fw, T beta, T alpha, T *r, int nrhs) {
  const int ng = (nrhs + RB - 1) / RB;
  const long long nblk = (long long)((L.n_atiles + 7) / 8) * 8 * ng;
  sp2d_kernel<T, P, RB><<<(unsigned)nblk, 256, 0, c.stream>>>(
      L.d_atiles, L.n_atiles, ng, nrhs, A.stencil, L.d_gcx_li, L.d_gcx_col, A.gcx_val, L.d_mask,
      u, f, fw, beta, alpha, r, L.Ntorn);
}

// the strip width of the lane-per-right-hand-side operator: a Gauss-Seidel
// tile width 2(p+1); 0 = none (a stencil line of 2p+1 > 16 coefficients does
// not fit the 16-lane broadcast)
template <int P>
constexpr int sp_rhs_bx_of() {
  return 2 * P + 1 <= 16 ? 2 * (P + 1) : 0;
}

template <int P>
static void launch_sp2d_rhs(Context &c, LevelData &L, const LevelArrays<float> &A, const float *u,
                            const float *f, const float *fw, float beta, float alpha, float *r,
                            int nrhs) {
  constexpr int BX = sp_rhs_bx_of<P>();
  if constexpr (BX == 0) {
    fail(IGAMG_EUNSUPPORTED, "no lane-per-right-hand-side operator for this degree");
  } else {
  const int ng = (nrhs + 63) / 64;
  transpose64_kernel<<<dim3((unsigned)L.n_plines, ng), 256, 0, c.stream>>>(
      u, nrhs, L.Ntorn, L.d_plines, L.pad_tot, L.ut);
  dim3 grid((unsigned)(((L.n_sptiles + 3) / 4 + 7) / 8 * 8), ng);
  {
    // the row kernel alone (without the transposition and the cross-patch
    // couplings of the same apply): the family of its roofline entry
    TimeScope ts(c, "stencil_rows", L.l);
    sp2d_rhs_kernel<P, BX><<<grid, 256, 0, c.stream>>>(L.d_sptiles, L.n_sptiles, nrhs, A.stencil,
                                                      L.d_mask, L.ut, L.pad_tot, f, fw, beta,
                                                      alpha, r, L.Ntorn);
  }
  launch_cross3d<float>(c, L, A.x_val, 0, L.x_n, u, r, true, alpha, nrhs);
  }
}

// one right-hand side per block, or groups of 4 (float64) / 8 (float32);
// float32 batches of 32 and more: one right-hand side per lane
template <typename T, int P>
static void launch_sp2d_rb(Context &c, LevelData &L, const LevelArrays<T> &A, const T *u,
                           const T *f, const T *fw, T beta, T alpha, T *r, int nrhs) {
  constexpr int RBB = sizeof(T) == 8 ? 4 : 8;
  if constexpr (sizeof(T) == 4) {
    if (sp_rhs_bx_of<P>() > 0 && nrhs >= SP_RHS_MIN && L.d_sptiles && L.ut) {
      launch_sp2d_rhs<P>(c, L, A, u, f, fw, beta, alpha, r, nrhs);
      return;
    }
  }
  if (nrhs == 1)
    launch_sp2d<T, P, 1>(c, L, A, u, f, fw, beta, alpha, r, nrhs);
  else
    launch_sp2d<T, P, RBB>(c, L, A, u, f, fw, beta, alpha, r, nrhs);
}

int sp_rhs_bx(int p) {
  switch (p) {
    case 1: return sp_rhs_bx_of<1>();
    case 2: return sp_rhs_bx_of<2>();
    case 3: return sp_rhs_bx_of<3>();
    case 4: return sp_rhs_bx_of<4>();
    case 5: return sp_rhs_bx_of<5>();
    case 6: return sp_rhs_bx_of<6>();
    case 7: return sp_rhs_bx_of<7>();
    case 8: return sp_rhs_bx_of<8>();
    default: return 0;
  }
}

template <typename T, int P>
static void launch_sp3d(Context &c, LevelData &L, const LevelArrays<T> &A, const T *u, const T *f,
                        const T *fw, T beta, T alpha, T *r, int nrhs) {
  sp3d_kernel<T, P><<<dim3(L.n_atiles, nrhs), 256, 0, c.stream>>>(
      L.d_atiles3, A.stencil, L.d_mask, u, f, fw, beta, alpha, r, L.Ntorn);
  launch_cross3d<T>(c, L, A.x_val, 0, L.x_n, u, r, true, alpha, nrhs);
}

template <typename T>
void k_stencil_apply(Context &c, LevelData &L, const LevelArrays<T> &A, const T *u, const T *f,
                     const T *fw, T beta, T alpha, T *r, int nrhs) {
  // the float64 operator of a float32-cycle solve is its own family
  TimeScope ts(c, sizeof(T) == 8 && c.fp32() ? "outer_apply" : "stencil_apply", L.l);
  if (c.d == 3) {
    if (!A.stencil || !L.d_atiles3 || L.n_atiles == 0)
      fail(IGAMG_EUNSUPPORTED, "no stored operator rows on this level");
    switch (c.p) {
      case 1: launch_sp3d<T, 1>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
      case 2: launch_sp3d<T, 2>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
      case 3: launch_sp3d<T, 3>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
      case 4: launch_sp3d<T, 4>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
      default: fail(IGAMG_EUNSUPPORTED, "3D degree out of range 1..4");
    }
    return;
  }
  if (c.d != 2 || !A.stencil || !L.d_atiles || L.n_atiles == 0)
    fail(IGAMG_EUNSUPPORTED, "no stored operator rows on this level");
  switch (c.p) {
    case 1: launch_sp2d_rb<T, 1>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 2: launch_sp2d_rb<T, 2>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 3: launch_sp2d_rb<T, 3>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 4: launch_sp2d_rb<T, 4>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 5: launch_sp2d_rb<T, 5>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 6: launch_sp2d_rb<T, 6>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 7: launch_sp2d_rb<T, 7>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    case 8: launch_sp2d_rb<T, 8>(c, L, A, u, f, fw, beta, alpha, r, nrhs); break;
    default: fail(IGAMG_EUNSUPPORTED, "degree out of range");
  }
}
template void k_stencil_apply<double>(Context &, LevelData &, const LevelArrays<double> &,
                                      const double *, const double *, const double *, double,
                                      double, double *, int);
template void k_stencil_apply<float>(Context &, LevelData &, const LevelArrays<float> &,
                                     const float *, const float *, const float *, float, float,
                                     float *, int);

template <typename T, bool BF, int NJ>
static void launch_fd2m(Context &c, LevelData &L, int stage, int nrhs) {
  constexpr int LDB = Fd2mShape<NJ, BF>::LDB, LDZ = Fd2mShape<NJ, BF>::LDZ;
  constexpr int KC = Fd2mShape<NJ, BF>::KC;
  const int lda = (L.fd_K1 + 31) / 32 * 32 + 2;
  const size_t lds = (size_t)(16 * lda + 16 * LDZ + KC * LDB) * sizeof(T);
  if (lds > 160 * 1024) fail(IGAMG_EUNSUPPORTED, "patch too large for the SCMS kernel");
  static const hipError_t lds_set =
      hipFuncSetAttribute((const void *)fd2m_kernel<T, BF, NJ>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  HIPCHK(lds_set);
  // the first stage also runs the interface pieces (extra blocks along z)
  PieceArgs<T> pa{};
  int gy = (L.fd_rows + 15) / 16, gz = L.n_fd;
  size_t shm = lds;
  if (stage == 0 && L.n_pieces > 0) {
    LevelArrays<T> &A = L.arr<T>();
    pa = PieceArgs<T>{L.d_pieces, L.d_piece_idx, L.d_piece_cp, L.d_piece_cidx, A.piece_inv, A.r,
                      A.u, (T)c.opt.damping_tau, L.Ntorn, L.n_pieces};
    gy = std::max(gy, (L.max_piece + 63) / 64);
    gz += L.n_pieces;
    shm = std::max(shm, (size_t)(L.max_piece + 4 * 64) * sizeof(T));
    if (shm > 160 * 1024) fail(IGAMG_EUNSUPPORTED, "interface piece too large for the SCMS kernel");
  }
  dim3 grid(nrhs, gy, gz);
  fd2m_kernel<T, BF, NJ><<<grid, 256, shm, c.stream>>>(L.arr<T>().fd[stage], L.n_fd, lda, pa);
}

#ifndef FD_STAGED_MIN
#define FD_STAGED_MIN 5.0e6
#endif

template <typename T, bool BF>
static void scms_staged(Context &c, LevelData &L, int nrhs) {
  dim3 grid(nrhs, L.fg_tiles, L.n_fd);
  for (int st = 0; st < 4; ++st)
    fdg_kernel<T, BF><<<grid, 256, 0, c.stream>>>(L.arr<T>().fg[st]);
}

// the four stages with the batch concatenated (FdWide): left, right, left, right
template <typename T, bool BF, int NT>
static void launch_fdw(Context &c, LevelData &L, int nrhs) {
  const dim3 grid((unsigned)((nrhs * (long long)L.fw_cat + 63) / 64), L.n_fd);
  for (int st = 0; st < 4; ++st) {
    if (st % 2)
      fdw_kernel<T, BF, true, NT><<<grid, 256, 0, c.stream>>>(L.arr<T>().fw[st], nrhs);
    else
      fdw_kernel<T, BF, false, NT><<<grid, 256, 0, c.stream>>>(L.arr<T>().fw[st], nrhs);
  }
}

// wide tiles rounded up to an even count (at most one zero tile computed)
template <typename T, bool BF>
static void scms_wide(Context &c, LevelData &L, int nrhs) {
  switch ((L.fw_wide + 31) / 32) {
    case 1: launch_fdw<T, BF, 2>(c, L, nrhs); break;
    case 2: launch_fdw<T, BF, 4>(c, L, nrhs); break;
    case 3: launch_fdw<T, BF, 6>(c, L, nrhs); break;
    case 4: launch_fdw<T, BF, 8>(c, L, nrhs); break;
    case 5: launch_fdw<T, BF, 10>(c, L, nrhs); break;
    case 6: launch_fdw<T, BF, 12>(c, L, nrhs); break;
    case 7: launch_fdw<T, BF, 14>(c, L, nrhs); break;
    case 8: launch_fdw<T, BF, 16>(c, L, nrhs); break;
    case 9: launch_fdw<T, BF, 18>(c, L, nrhs); break;
    case 10: launch_fdw<T, BF, 20>(c, L, nrhs); break;
    default: fail(IGAMG_EUNSUPPORTED, "patch too large for the SCMS kernel");
  }
}

template <typename T, bool BF>
static void scms_mfma(Context &c, LevelData &L, int nrhs) {
  const int nj = (L.fd_N + 63) / 64;
  for (int st = 0; st < 2; ++st) {
    switch (nj) {
      case 1: launch_fd2m<T, BF, 1>(c, L, st, nrhs); break;
      case 2: launch_fd2m<T, BF, 2>(c, L, st, nrhs); break;
      case 3: launch_fd2m<T, BF, 3>(c, L, st, nrhs); break;
      case 4: launch_fd2m<T, BF, 4>(c, L, st, nrhs); break;
      case 5: launch_fd2m<T, BF, 5>(c, L, st, nrhs); break;
      default: fail(IGAMG_EUNSUPPORTED, "patch too large for the SCMS kernel");
    }
  }
}

// patch interiors of the subspace corrected mass smoother: two launches of
// chained products on the matrix cores (bfloat16 operands when the options
// ask for them, float32 cycles only)
// 3D: six stages, each with its own item count and tile range
template <typename T, bool BF>
static void scms_staged3(Context &c, LevelData &L, int nrhs) {
  for (int st = 0; st < 6; ++st) {
    if (L.fg_n[st] == 0) continue;
    dim3 grid(nrhs, L.fg_t[st], L.fg_n[st]);
    fdg_kernel<T, BF><<<grid, 256, 0, c.stream>>>(L.arr<T>().fg[st]);
  }
}

template <typename T>
bool k_scms_interior(Context &c, LevelData &L, int nrhs) {
  TimeScope ts(c, "scms", L.l);
  if (L.n_fd == 0) return false;
  if (c.d == 3) {
    if constexpr (sizeof(T) == 4) {
      if (c.bf16_scms()) {
        scms_staged3<float, true>(c, L, nrhs);
        return false;
      }
    }
    scms_staged3<T, false>(c, L, nrhs);
    return false;
  }
  // the fused form re-reads each right-hand side's operand once per 16-row
  // block; past this much re-read work the four-stage form is faster.  The
  // fused form runs the interface pieces in its first launch (returns true).
  const bool staged = (double)L.fd_work * nrhs >= FD_STAGED_MIN;
  if constexpr (sizeof(T) == 4) {
    if (c.bf16_scms()) {
      if (staged)
        scms_wide<float, true>(c, L, nrhs);
      else
        scms_mfma<float, true>(c, L, nrhs);
      return !staged;
    }
  }
  // float64 keeps the per-right-hand-side tiles (fdg_kernel): the batched
  // form's float64 instantiation is switched off
  if (staged) {
    if constexpr (sizeof(T) == 4)
      scms_wide<T, false>(c, L, nrhs);
    else
      scms_staged<T, false>(c, L, nrhs);
  } else
    scms_mfma<T, false>(c, L, nrhs);
  return !staged;
}
template bool k_scms_interior<double>(Context &, LevelData &, int);
template bool k_scms_interior<float>(Context &, LevelData &, int);

// float32 batches of at least this many right-hand sides take the matrix-core
// form of the interface pieces
constexpr int PIECE_MFMA_MIN = 16;

template <typename T>
void k_pieces(Context &c, LevelData &L, int nrhs) {
  TimeScope ts(c, "pieces", L.l);
  if (L.n_pieces == 0) return;
  LevelArrays<T> &A = L.arr<T>();
  // dynamic LDS: the piece's residual; static: 16 x 64 partial sums
  const size_t shm = (size_t)L.max_piece * sizeof(T);
  if (shm + 16 * 64 * sizeof(T) > 160 * 1024)
    fail(IGAMG_EUNSUPPORTED, "interface piece too large for the piece kernel's LDS");
  static const hipError_t lds_set = hipFuncSetAttribute(
      (const void *)piece_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
      160 * 1024 - 16 * 64 * (int)sizeof(T));
  HIPCHK(lds_set);
  if constexpr (sizeof(T) == 4) {
    if (nrhs >= PIECE_MFMA_MIN && L.max_piece <= PIECE_MFMA_N) {
      dim3 g4((unsigned)((L.max_piece + 63) / 64), L.n_pieces, (nrhs + 63) / 64);
      piece_mfma_kernel<<<g4, 256, 0, c.stream>>>(L.d_pieces, L.d_piece_idx, L.d_piece_cp,
                                                   L.d_piece_cidx, A.piece_inv, A.r, A.u,
                                                   (T)c.opt.damping_tau, L.Ntorn, nrhs);
      return;
    }
  }
  dim3 grid(nrhs, L.n_pieces, (L.max_piece + 63) / 64);
  piece_kernel<T><<<grid, 1024, shm, c.stream>>>(
      L.d_pieces, L.d_piece_idx, L.d_piece_cp, L.d_piece_cidx, A.piece_inv, A.r, A.u,
      (T)c.opt.damping_tau, L.Ntorn);
}
template void k_pieces<double>(Context &, LevelData &, int);
template void k_pieces<float>(Context &, LevelData &, int);

template <typename T>
void k_restrict(Context &c, LevelData &F, LevelData &C, const T *rf, T *rc, T *uc_zero, int nrhs) {
  TimeScope ts(c, "restrict", F.l);
  if (c.d == 3) {
    transfer3d_kernel<T, true><<<dim3(nblocks(C.Ntorn), nrhs), 256, 0, c.stream>>>(
        F.d_pd, C.d_pd, F.d_pd, F.K, C.Ntorn, F.d_R_lo, F.arr<T>().R_val, F.RW, rf,
        F.arr<T>().weight, C.d_mask, rc, uc_zero, F.Ntorn, C.Ntorn);
    return;
  }
  dim3 grid(nrhs, F.n_rtiles);
  if (F.r_wide)
    transfer2d_kernel<T, true, XFER_R_TX, XFER_R_WX, XFER_R_WY><<<grid, 256, 0, c.stream>>>(
        F.d_rtiles, F.d_R_lo, F.arr<T>().R_val, F.RW, rf, F.arr<T>().weight, C.d_mask, rc,
        uc_zero, F.Ntorn, C.Ntorn);
  else
    transfer2d_kernel<T, true, XFER_TX, XFER_WX, XFER_WX><<<grid, 256, 0, c.stream>>>(
        F.d_rtiles, F.d_R_lo, F.arr<T>().R_val, F.RW, rf, F.arr<T>().weight, C.d_mask, rc,
        uc_zero, F.Ntorn, C.Ntorn);
}
template void k_restrict<double>(Context &, LevelData &, LevelData &, const double *, double *,
                                 double *, int);
template void k_restrict<float>(Context &, LevelData &, LevelData &, const float *, float *, float *,
                                int);

template <typename T>
void k_prolong_add(Context &c, LevelData &F, LevelData &C, const T *ec, T *uf, int nrhs) {
  TimeScope ts(c, "prolong", F.l);
  if (c.d == 3) {
    transfer3d_kernel<T, false><<<dim3(nblocks(F.Ntorn), nrhs), 256, 0, c.stream>>>(
        C.d_pd, F.d_pd, F.d_pd, F.K, F.Ntorn, F.d_P_lo, F.arr<T>().P_val, F.PW, ec, nullptr,
        F.d_mask, uf, nullptr, C.Ntorn, F.Ntorn);
    return;
  }
  dim3 grid(nrhs, F.n_ptiles);
  if (F.p_wide)
    transfer2d_kernel<T, false, XFER_P_TX, XFER_P_WX, XFER_P_WY><<<grid, 256, 0, c.stream>>>(
        F.d_ptiles, F.d_P_lo, F.arr<T>().P_val, F.PW, ec, nullptr, F.d_mask, uf, nullptr,
        C.Ntorn, F.Ntorn);
  else
    transfer2d_kernel<T, false, XFER_TX, XFER_WX, XFER_WX><<<grid, 256, 0, c.stream>>>(
        F.d_ptiles, F.d_P_lo, F.arr<T>().P_val, F.PW, ec, nullptr, F.d_mask, uf, nullptr,
        C.Ntorn, F.Ntorn);
}
template void k_prolong_add<double>(Context &, LevelData &, LevelData &, const double *, double *,
                                    int);
template void k_prolong_add<float>(Context &, LevelData &, LevelData &, const float *, float *, int);

template <typename T>
void k_coarse_solve(Context &c, const T *f0, T *u0, int nrhs) {
  TimeScope ts(c, "coarse", 0);
  const int rb = (c.N0 + 63) / 64;
  const int ns = c.coarse_splits;
  const int chunk = (c.N0 + ns - 1) / ns;
  coarse_partial_kernel<T><<<dim3(rb, ns, nrhs), 1024, (size_t)chunk * sizeof(double), c.stream>>>(
      c.N0, c.d_A0inv, c.d_c0_cp, c.d_c0_cidx, f0, c.d_coarse_part, c.lv[0].Ntorn);
  coarse_final_kernel<T><<<dim3((c.N0 + 255) / 256, nrhs), 256, 0, c.stream>>>(
      c.N0, ns, c.d_coarse_part, c.d_c0_cp, c.d_c0_cidx, u0, c.lv[0].Ntorn);
}
template void k_coarse_solve<double>(Context &, const double *, double *, int);
template void k_coarse_solve<float>(Context &, const float *, float *, int);

void k_gather_rows(const double *st, int SP, const int *rows, int nrows, double *out,
                   hipStream_t s) {
  if (nrows <= 0) return;
  gather_rows_kernel<<<nblocks((long long)nrows * SP), BS, 0, s>>>(st, SP, rows, nrows, out);
}

// one launch of each kernel per block step for the whole batch (offs/ns
// device arrays of nmat entries; offs == null: one matrix of order nmax)
static void gj_batch(double *base, const long long *offs, const int *ns, int nmat, int nmax,
                     int *bad, hipStream_t s) {
  if (nmax <= 0 || nmat <= 0) return;
  const unsigned nbl = (unsigned)((nmax + 255) / 256);
  const unsigned nt = (unsigned)((nmax + 63) / 64);
  for (int k0 = 0; k0 < nmax; k0 += GJB) {
    gj_diag_kernel<<<dim3(1, 1, nmat), 1024, 0, s>>>(base, offs, ns, nmax, k0, bad);
    if (nmax > GJB) {
      gj_row_kernel<<<dim3(nbl, 1, nmat), 256, 0, s>>>(base, offs, ns, nmax, k0);
      gj_update_kernel<<<dim3(nt, nt, nmat), 256, 0, s>>>(base, offs, ns, nmax, k0);
      gj_col_kernel<<<dim3(nbl, 1, nmat), 256, 0, s>>>(base, offs, ns, nmax, k0);
    }
  }
}

void k_spd_inverse(double *A, int n, int *bad, hipStream_t s) {
  gj_batch(A, nullptr, nullptr, 1, n, bad, s);
}

void k_spd_inverse_batch(double *base, const long long *offs, const int *ns, int nmat, int nmax,
                         int *bad, hipStream_t s) {
  gj_batch(base, offs, ns, nmat, nmax, bad, s);
}

void k_scatter_compact(const double *xc, long long N, const int *cp, const int *cidx, double *xt,
                       long long Ntorn, int nrhs, hipStream_t s) {
  dim3 grid(nblocks(N), nrhs);
  scatter_compact_kernel<<<grid, BS, 0, s>>>(xc, N, cp, cidx, xt, Ntorn);
}

void k_gather_compact(const double *xt, long long N, const int *cp, const int *cidx, int sum,
                      double *xc, long long Ntorn, int nrhs, hipStream_t s) {
  dim3 grid(nblocks(N), nrhs);
  gather_compact_kernel<<<grid, BS, 0, s>>>(xt, N, cp, cidx, sum, xc, Ntorn);
}

// Weights of the finest level's inner products: 1 on every unknown's
// representative copy, 0 on the other copies and on Dirichlet entries (held
// at zero in every vector the sums read).  Without glued copies the free
// unknowns are all representatives, so the weights are dropped (same sums,
// one vector read fewer per right-hand side).
static const double *dot_weights(const Context &c) {
  const LevelData &L = c.lv.back();
  return L.n_glue > 0 ? L.a64.weight : nullptr;
}

template <typename T>
static void dot_any(Context &c, const T *a, const T *b, long long n, int slot, int mode,
                    int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dot_partial_kernel<T><<<dim3(RED_BLOCKS, nrhs), 256, 0, c.stream>>>(a, b, dot_weights(c), n,
                                                                       c.d_red);
  dot_final_kernel<<<nrhs, 256, 0, c.stream>>>(c.d_red, RED_BLOCKS, c.d_scal, slot, mode);
}
void k_dot(Context &c, const double *a, const double *b, long long n, int slot, int mode, int nrhs) {
  dot_any(c, a, b, n, slot, mode, nrhs);
}
void k_dot(Context &c, const float *a, const float *b, long long n, int slot, int mode, int nrhs) {
  dot_any(c, a, b, n, slot, mode, nrhs);
}

void k_dot_fcg(Context &c, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dot2_partial_kernel<<<dim3(RED_BLOCKS, nrhs), 256, 0, c.stream>>>(c.z, c.rr, c.rold,
                                                                     dot_weights(c), n, c.d_red);
  dot2_final_kernel<<<nrhs, 256, 0, c.stream>>>(c.d_red, RED_BLOCKS, c.d_scal);
}

void k_pcg_update_xr(Context &c, long long n, int nrhs, bool keep_rold) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  pcg_xr_kernel<double><<<dim3(RED_BLOCKS, nrhs), 256, 0, c.stream>>>(
      c.x, c.rr, c.pp, c.qq, dot_weights(c), n, c.d_scal, c.d_red, c.z,
      keep_rold ? c.rold : nullptr, c.d_active);
  dot_final_kernel<<<nrhs, 256, 0, c.stream>>>(c.d_red, RED_BLOCKS, c.d_scal, S_RR, 0);
}

void k_pcg_update_xr(Context &c, float *x, float *r, const float *p, const float *q,
                     float *z_zero, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  pcg_xr_kernel<float><<<dim3(RED_BLOCKS, nrhs), 256, 0, c.stream>>>(
      x, r, p, q, dot_weights(c), n, c.d_scal, c.d_red, z_zero, nullptr, c.d_active);
  dot_final_kernel<<<nrhs, 256, 0, c.stream>>>(c.d_red, RED_BLOCKS, c.d_scal, S_RR, 0);
}

void k_add_active(Context &c, double *y, const double *x, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dim3 grid(std::min<unsigned>(nblocks(n), 2048), nrhs);
  add_active_kernel<double><<<grid, BS, 0, c.stream>>>(y, x, n, c.d_active);
}

void k_add_active(Context &c, double *y, const float *x, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dim3 grid(std::min<unsigned>(nblocks(n), 2048), nrhs);
  add_active_kernel<float><<<grid, BS, 0, c.stream>>>(y, x, n, c.d_active);
}

void k_pcg_update_p(Context &c, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dim3 grid(std::min<unsigned>(nblocks(n), 2048), nrhs);
  pcg_p_kernel<double><<<grid, BS, 0, c.stream>>>(c.pp, c.z, n, c.d_scal, c.d_active);
}

void k_pcg_update_p(Context &c, float *p, const float *z, long long n, int nrhs) {
  TimeScope ts(c, "blas1", (int)c.lv.size() - 1);
  dim3 grid(std::min<unsigned>(nblocks(n), 2048), nrhs);
  pcg_p_kernel<float><<<grid, BS, 0, c.stream>>>(p, z, n, c.d_scal, c.d_active);
}

}  // namespace igamg
