// Multigrid cycle (Algorithms 1 and 2) and outer iterations (Section 4:
// multigrid used directly, or as preconditioner of conjugate gradients,
// stopped at ||f - A u|| / ||f|| <= tol).
//
// Vector conventions on every level (torn layout = all patch-local
// coefficients, Dirichlet entries held at zero):
//  * iterates u and residuals r are consistent: every copy of a glued
//    (conforming) unknown holds its value;
//  * right-hand sides f of the cycle are distributed: the copies of a glued
//    unknown sum to its value (restriction of a weighted residual produces
//    exactly this form).  In the SIPG space every unknown has one copy and
//    both forms coincide.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "context.h"
#include "kernels.h"

namespace igamg {

// r = f - A u on level l (f distributed, result consistent)
static void residual(Context &c, int l, const double *u, const double *f, double *r) {
  LevelData &L = c.lv[l];
  k_iface_apply(c, L, u, f, nullptr, 1.0, -1.0, r);
  k_vol_apply(c, L, u, r, -1.0);
  k_glue_sum(L, r, c.stream);
}

void apply_torn(Context &c, int l, const double *u, const double *f, const double *fw, double *r,
                double alpha) {
  LevelData &L = c.lv[l];
  k_iface_apply(c, L, u, f, fw, 1.0, alpha, r);
  k_vol_apply(c, L, u, r, alpha);
  k_glue_sum(L, r, c.stream);
}

// one step of the additive piece smoother (eq. Ldef): u += tau sum_T P_T L_T^-1 P_T^T r
static void scms_step(Context &c, int l) {
  LevelData &L = c.lv[l];
  residual(c, l, L.u, L.f, L.r);
  k_scms_interior(c, L);
  k_pieces(c, L, L.r, L.u);
}

static void mg(Context &c, int l) {
  LevelData &L = c.lv[l];
  if (l == 0) {
    k_coarse_solve(c, L.f, L.u);
    return;
  }
  const int sm = c.opt.smoother;
  // pre-smoothing
  if (sm == IGAMG_SMOOTHER_GS) {
    for (int i = 0; i < c.opt.nu; ++i) k_gs_sweep(c, L, false);
  } else {
    if (sm == IGAMG_SMOOTHER_HYBRID) k_gs_sweep(c, L, false);
    for (int i = 0; i < c.opt.nu; ++i) scms_step(c, l);
  }
  // coarse-grid correction
  LevelData &C = c.lv[l - 1];
  const int reps = (l == 1) ? 1 : c.opt.mu;
  for (int rep = 0; rep < reps; ++rep) {
    residual(c, l, L.u, L.f, L.r);
    k_restrict(c, L, C, L.r, C.f, l == 1 ? nullptr : C.u);
    if (l == 1)
      k_coarse_solve(c, C.f, C.u);
    else
      mg(c, l - 1);
    k_prolong_add(c, L, C, C.u, L.u);
  }
  // post-smoothing
  if (sm == IGAMG_SMOOTHER_GS) {
    for (int i = 0; i < c.opt.nu; ++i) k_gs_sweep(c, L, true);
  } else {
    for (int i = 0; i < c.opt.nu; ++i) scms_step(c, l);
    if (sm == IGAMG_SMOOTHER_HYBRID) k_gs_sweep(c, L, true);
  }
}

void vcycle_torn(Context &c, int l) { mg(c, l); }

// z = MG(L, r, 0) on the finest level.  z is the finest level's iterate L.u
// (c.z aliases it); it must be zero on entry.  In the SIPG space the
// distributed right-hand side equals r itself, so the cycle reads r directly.
static void precondition(Context &c, double *r) {
  LevelData &L = c.lv.back();
  double *f_saved = L.f;
  if (L.n_glue > 0)
    k_copy_weighted(r, L.d_weight, L.f, L.Ntorn, c.stream);
  else
    L.f = r;
  mg(c, (int)c.lv.size() - 1);
  L.f = f_saved;
}

static double read_scalar(Context &c, int slot) {
  HIPCHK(hipMemcpyAsync(c.h_scal + slot, c.d_scal + slot, sizeof(double), hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return c.h_scal[slot];
}

int solve_compact(Context &c, const double *rhs, double *u, double tol, int maxit, int use_x0,
                  igamg_solve_info *info) {
  auto t0 = std::chrono::steady_clock::now();
  LevelData &L = c.lv.back();
  const int top = (int)c.lv.size() - 1;
  const long long nt = L.Ntorn;
  k_fill(c.ff, 0.0, nt, c.stream);
  k_scatter_compact(rhs, L.N, c.d_fin_cp, c.d_fin_cidx, c.ff, c.stream);
  k_fill(c.x, 0.0, nt, c.stream);
  if (use_x0) {
    k_scatter_compact(u, L.N, c.d_fin_cp, c.d_fin_cidx, c.x, c.stream);
    apply_torn(c, top, c.x, c.ff, L.d_weight, c.rr, -1.0);  // r = f - A x
  } else {
    HIPCHK(hipMemcpyAsync(c.rr, c.ff, nt * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
  }
  k_dot(c, c.ff, c.ff, nt, S_FF, 0);
  const double ff = read_scalar(c, S_FF);
  const double nf = std::sqrt(ff);
  k_dot(c, c.rr, c.rr, nt, S_RR, 0);
  double res = nf > 0 ? std::sqrt(read_scalar(c, S_RR)) / nf : 0.0;
  int it = 0;
  if (info && info->history) info->history[0] = res;
  if (nf > 0 && res > tol) {
    if (c.opt.outer == IGAMG_OUTER_MG) {
      for (it = 1; it <= maxit; ++it) {
        k_copy_weighted(c.ff, L.d_weight, L.f, nt, c.stream);
        HIPCHK(hipMemcpyAsync(L.u, c.x, nt * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
        mg(c, top);
        HIPCHK(hipMemcpyAsync(c.x, L.u, nt * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
        apply_torn(c, top, c.x, c.ff, L.d_weight, c.rr, -1.0);
        k_dot(c, c.rr, c.rr, nt, S_RR, 0);
        res = std::sqrt(read_scalar(c, S_RR)) / nf;
        if (info && info->history) info->history[it] = res;
        if (res <= tol) break;
      }
    } else {
      k_fill(c.z, 0.0, nt, c.stream);
      precondition(c, c.rr);
      k_dot(c, c.rr, c.z, nt, S_RZ, 0);
      HIPCHK(hipMemcpyAsync(c.pp, c.z, nt * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
      for (it = 1; it <= maxit; ++it) {
        apply_torn(c, top, c.pp, nullptr, nullptr, c.qq, 1.0);  // q = A p
        k_dot(c, c.pp, c.qq, nt, S_PQ, 1);              // alpha = rz / pq
        k_pcg_update_xr(c, nt);                         // x += alpha p, r -= alpha q, rr
        res = std::sqrt(read_scalar(c, S_RR)) / nf;
        if (info && info->history) info->history[it] = res;
        if (res <= tol) break;
        precondition(c, c.rr);                          // z zeroed by the update above
        k_dot(c, c.rr, c.z, nt, S_RZNEW, 2);            // beta = rz_new / rz
        k_pcg_update_p(c, nt);                          // p = z + beta p
      }
    }
  }
  if (it > maxit) it = maxit;
  k_gather_compact(c.x, L.N, c.d_fin_cp, c.d_fin_cidx, 0, u, c.stream);
  // true residual in float64
  apply_torn(c, top, c.x, c.ff, L.d_weight, c.qq, -1.0);
  k_dot(c, c.qq, c.qq, nt, S_TMP, 0);
  double tres = nf > 0 ? std::sqrt(read_scalar(c, S_TMP)) / nf : 0.0;
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iterations = it;
    info->rel_residual = res;
    info->true_rel_residual = tres;
    info->seconds = std::chrono::duration<double>(t1 - t0).count();
  }
  return res <= tol || nf == 0 ? IGAMG_OK : IGAMG_ENOCONV;
}

}  // namespace igamg
