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
// Every vector holds a batch of right-hand sides ([nrhs][Ntorn]).  The cycle
// runs in the context's arithmetic T (float64 or float32); the outer
// iteration, its residuals and the convergence test are float64 always.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "context.h"
#include "kernels.h"

namespace igamg {

namespace {

// r = f - A u on level L (f distributed, result consistent)
template <typename T>
void residual(Context &c, LevelData &L, const T *u, const T *f, T *r, int nb) {
  if (L.st_apply) {
    k_stencil_apply<T>(c, L, L.arr<T>(), u, f, nullptr, (T)1, (T)-1, r, nb);
    return;
  }
  k_iface_apply<T>(c, L, u, f, nullptr, (T)1, (T)-1, r, nb);
  k_vol_apply<T>(c, L, u, r, (T)-1, nb);
  k_glue_sum<T>(L, r, nb, c.stream);
}

// one step of the additive piece smoother (eq. Ldef): u += tau sum_T P_T L_T^-1 P_T^T r
template <typename T>
void scms_step(Context &c, LevelData &L, int nb) {
  LevelArrays<T> &A = L.arr<T>();
  residual<T>(c, L, A.u, A.f, A.r, nb);
  if (!k_scms_interior<T>(c, L, nb)) k_pieces<T>(c, L, nb);
}

template <typename T>
void mg(Context &c, int l, int nb) {
  LevelData &L = c.lv[l];
  LevelArrays<T> &A = L.arr<T>();
  if (l == 0) {
    k_coarse_solve<T>(c, A.f, A.u, nb);
    return;
  }
  const int sm = c.opt.smoother;
  // pre-smoothing
  if (sm == IGAMG_SMOOTHER_GS) {
    for (int i = 0; i < c.opt.nu; ++i) k_gs_sweep<T>(c, L, false, nb);
  } else {
    if (sm == IGAMG_SMOOTHER_HYBRID) k_gs_sweep<T>(c, L, false, nb);
    for (int i = 0; i < c.opt.nu; ++i) scms_step<T>(c, L, nb);
  }
  // coarse-grid correction
  LevelData &C = c.lv[l - 1];
  LevelArrays<T> &AC = C.arr<T>();
  const int reps = (l == 1) ? 1 : c.opt.mu;
  for (int rep = 0; rep < reps; ++rep) {
    residual<T>(c, L, A.u, A.f, A.r, nb);
    k_restrict<T>(c, L, C, A.r, AC.f, l == 1 ? nullptr : AC.u, nb);
    if (l == 1)
      k_coarse_solve<T>(c, AC.f, AC.u, nb);
    else
      mg<T>(c, l - 1, nb);
    k_prolong_add<T>(c, L, C, AC.u, A.u, nb);
  }
  // post-smoothing
  if (sm == IGAMG_SMOOTHER_GS) {
    for (int i = 0; i < c.opt.nu; ++i) k_gs_sweep<T>(c, L, true, nb);
  } else {
    for (int i = 0; i < c.opt.nu; ++i) scms_step<T>(c, L, nb);
    if (sm == IGAMG_SMOOTHER_HYBRID) k_gs_sweep<T>(c, L, true, nb);
  }
}

void mg_top(Context &c, int nb) {
  if (c.fp32())
    mg<float>(c, (int)c.lv.size() - 1, nb);
  else
    mg<double>(c, (int)c.lv.size() - 1, nb);
}

// Finest cycle input from a float64 torn vector: f = w .* x (consistent ->
// distributed) in the cycle arithmetic; zero_u also clears the iterate.
void set_cycle_rhs(Context &c, const double *x, int nb, bool zero_u) {
  LevelData &L = c.lv.back();
  const long long nt = L.Ntorn;
  if (c.fp32()) {
    k_convert<double, float>(x, L.a32.weight, L.a32.f, nt, nb, c.stream,
                             zero_u ? L.a32.u : nullptr);
  } else {
    k_convert<double, double>(x, L.a64.weight, L.a64.f, nt, nb, c.stream,
                              zero_u ? L.a64.u : nullptr);
  }
}

// z = MG(L, r, 0) on the finest level (z = c.z).  In float64 z is the finest
// iterate itself and must be zero on entry (the outer update clears it).
void precondition_launches(Context &c, const double *r, int nb) {
  LevelData &L = c.lv.back();
  const long long nt = L.Ntorn;
  if (c.fp32()) {
    set_cycle_rhs(c, r, nb, true);
    mg<float>(c, (int)c.lv.size() - 1, nb);
    k_convert<float, double>(L.a32.u, nullptr, c.z, nt, nb, c.stream);
    return;
  }
  // In the SIPG space the distributed right-hand side equals r itself, so the
  // cycle reads r directly.
  double *f_saved = L.a64.f;
  if (L.n_glue > 0)
    set_cycle_rhs(c, r, nb, false);
  else
    L.a64.f = const_cast<double *>(r);
  mg<double>(c, (int)c.lv.size() - 1, nb);
  L.a64.f = f_saved;
}

// z = MG(L, r, 0) from a float32 residual (the refinement's inner
// iteration): z is the finest float32 iterate itself and must be zero on
// entry; in the SIPG space the cycle reads r directly.
void precondition_launches(Context &c, const float *r, int nb) {
  LevelData &L = c.lv.back();
  float *f_saved = L.a32.f;
  if (L.n_glue > 0)
    k_convert<float, float>(r, L.a32.weight, L.a32.f, L.Ntorn, nb, c.stream);
  else
    L.a32.f = const_cast<float *>(r);
  mg<float>(c, (int)c.lv.size() - 1, nb);
  L.a32.f = f_saved;
}

// The same cycle as one graph launch (option graphs).  Its launches read
// the device mask of active right-hand sides, so one graph serves every
// iteration; pointers and the batch size are fixed in it, hence one graph
// per (r, nb).  The first use runs launch by launch (one-time host work such
// as kernel attributes happens there), the second is captured on the
// context's private stream and replayed on c.stream from then on.  The
// cycle issues kernels only (no memset, allocation or host wait).
template <typename R>
void precondition_any(Context &c, const R *r, int nb) {
  if (!c.opt.graphs || c.opt.timing) {
    precondition_launches(c, r, nb);
    return;
  }
  Context::CycleGraph *g = nullptr;
  for (auto &e : c.graphs)
    if (e.r == r && e.nb == nb) g = &e;
  if (!g) {
    constexpr size_t MAX_GRAPHS = 8;
    if (c.graphs.size() >= MAX_GRAPHS) {
      precondition_launches(c, r, nb);
      return;
    }
    c.graphs.push_back(Context::CycleGraph{r, nb, 0, nullptr});
    g = &c.graphs.back();
  }
  if (g->exec) {
    HIPCHK(hipGraphLaunch(g->exec, c.stream));
    return;
  }
  if (++g->uses < 2) {
    precondition_launches(c, r, nb);
    return;
  }
  if (!c.cap_stream) HIPCHK(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
  hipStream_t user = c.stream;
  c.stream = c.cap_stream;
  HIPCHK(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    precondition_launches(c, r, nb);
  } catch (...) {
    c.stream = user;
    if (hipStreamEndCapture(c.cap_stream, &graph) == hipSuccess && graph)
      (void)hipGraphDestroy(graph);
    throw;
  }
  c.stream = user;
  HIPCHK(hipStreamEndCapture(c.cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(e);
  g->exec = exec;
  HIPCHK(hipGraphLaunch(exec, c.stream));
}

void precondition(Context &c, const double *r, int nb) { precondition_any(c, r, nb); }
void precondition(Context &c, const float *r, int nb) { precondition_any(c, r, nb); }

// q = A p on the finest level, float32 vectors in and out
void apply_inner(Context &c, const float *p, float *q, int nb) {
  LevelData &L = c.lv.back();
  LevelArrays<float> &A = L.a32;
  if (L.st_apply) {
    k_stencil_apply<float>(c, L, A, p, nullptr, nullptr, 0.0f, 1.0f, q, nb);
  } else {
    k_iface_apply<float>(c, L, p, nullptr, nullptr, 0.0f, 1.0f, q, nb);
    k_vol_apply<float>(c, L, p, q, 1.0f, nb);
    k_glue_sum<float>(L, q, nb, c.stream);
  }
}

// q = A p on the finest level, float64 vectors in and out
void apply_inner(Context &c, const double *p, double *q, int nb) {
  apply64(c, p, nullptr, nullptr, q, 1.0, nb);
}

void read_scalars(Context &c, int nb) {
  HIPCHK(hipMemcpyAsync(c.h_scal, c.d_scal, (size_t)nb * S_COUNT * sizeof(double),
                        hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
}

void upload_active(Context &c, int nb) {
  HIPCHK(hipMemcpyAsync(c.d_active, c.h_active, (size_t)nb * sizeof(int),
                        hipMemcpyHostToDevice, c.stream));
}

}  // namespace

void apply64(Context &c, const double *u, const double *f, const double *fw, double *r,
             double alpha, int nb) {
  LevelData &L = c.lv.back();
  if (c.apply64_rows) {
    k_stencil_apply<double>(c, L, L.a64, u, f, fw, 1.0, alpha, r, nb);
    return;
  }
  k_iface_apply<double>(c, L, u, f, fw, 1.0, alpha, r, nb);
  k_vol_apply<double>(c, L, u, r, alpha, nb);
  k_glue_sum<double>(L, r, nb, c.stream);
}

void vcycle_compact(Context &c, const double *f, double *u, int nb) {
  LevelData &L = c.lv.back();
  const long long nt = L.Ntorn;
  k_fill(c.ff, 0.0, nt * nb, c.stream);
  k_scatter_compact(f, L.N, c.d_fin_cp, c.d_fin_cidx, c.ff, nt, nb, c.stream);
  k_fill(c.x, 0.0, nt * nb, c.stream);
  k_scatter_compact(u, L.N, c.d_fin_cp, c.d_fin_cidx, c.x, nt, nb, c.stream);
  set_cycle_rhs(c, c.ff, nb, false);
  if (c.fp32())
    k_convert<double, float>(c.x, nullptr, L.a32.u, nt, nb, c.stream);
  else
    k_convert<double, double>(c.x, nullptr, L.a64.u, nt, nb, c.stream);
  mg_top(c, nb);
  if (c.fp32())
    k_convert<float, double>(L.a32.u, nullptr, c.x, nt, nb, c.stream);
  else
    k_convert<double, double>(L.a64.u, nullptr, c.x, nt, nb, c.stream);
  k_gather_compact(c.x, L.N, c.d_fin_cp, c.d_fin_cidx, 0, u, nt, nb, c.stream);
}

int solve_batch(Context &c, const double *rhs, double *u, int nb, double tol, int maxit,
                int use_x0, igamg_solve_info *info) {
  auto t0 = std::chrono::steady_clock::now();
  LevelData &L = c.lv.back();
  const long long nt = L.Ntorn;
  const size_t bytes = (size_t)nt * nb * sizeof(double);
  k_fill(c.ff, 0.0, nt * nb, c.stream);
  k_scatter_compact(rhs, L.N, c.d_fin_cp, c.d_fin_cidx, c.ff, nt, nb, c.stream);
  k_fill(c.x, 0.0, nt * nb, c.stream);
  if (use_x0) {
    k_scatter_compact(u, L.N, c.d_fin_cp, c.d_fin_cidx, c.x, nt, nb, c.stream);
    apply64(c, c.x, c.ff, L.a64.weight, c.rr, -1.0, nb);  // r = f - A x
  } else {
    HIPCHK(hipMemcpyAsync(c.rr, c.ff, bytes, hipMemcpyDeviceToDevice, c.stream));
  }
  k_dot(c, c.ff, c.ff, nt, S_FF, 0, nb);
  k_dot(c, c.rr, c.rr, nt, S_RR, 0, nb);
  read_scalars(c, nb);
  std::vector<double> nf(nb), res(nb);
  std::vector<int> its(nb, 0);
  int n_active = 0;
  for (int j = 0; j < nb; ++j) {
    const double *sc = c.h_scal + (size_t)j * S_COUNT;
    nf[j] = std::sqrt(sc[S_FF]);
    res[j] = nf[j] > 0 ? std::sqrt(sc[S_RR]) / nf[j] : 0.0;
    if (info && info[j].history) info[j].history[0] = res[j];
    c.h_active[j] = (nf[j] > 0 && res[j] > tol) ? 1 : 0;
    n_active += c.h_active[j];
  }
  upload_active(c, nb);
  // host-side convergence bookkeeping after an update of S_RR (the host
  // mirror must hold the scalars of iteration it)
  std::vector<double> res_prev(nb, 0.0);  // relative residual one step before res
  auto tally = [&](int it) {
    bool changed = false;
    for (int j = 0; j < nb; ++j) {
      if (!c.h_active[j]) continue;
      res_prev[j] = res[j];
      res[j] = std::sqrt(c.h_scal[(size_t)j * S_COUNT + S_RR]) / nf[j];
      its[j] = it;
      if (info && info[j].history) info[j].history[it] = res[j];
      if (res[j] <= tol) {
        c.h_active[j] = 0;
        --n_active;
        changed = true;
      }
    }
    if (changed && n_active > 0) upload_active(c, nb);
  };
  auto check = [&](int it) {
    read_scalars(c, nb);
    tally(it);
  };
  if (n_active > 0) {
    if (c.opt.outer == IGAMG_OUTER_MG) {
      for (int it = 1; it <= maxit && n_active > 0; ++it) {
        set_cycle_rhs(c, c.ff, nb, false);
        if (c.fp32())
          k_convert<double, float>(c.x, nullptr, L.a32.u, nt, nb, c.stream);
        else
          k_convert<double, double>(c.x, nullptr, L.a64.u, nt, nb, c.stream);
        mg_top(c, nb);
        // converged right-hand sides keep their iterate
        if (c.fp32())
          k_convert<float, double>(L.a32.u, nullptr, c.x, nt, nb, c.stream, nullptr, c.d_active);
        else
          k_convert<double, double>(L.a64.u, nullptr, c.x, nt, nb, c.stream, nullptr, c.d_active);
        apply64(c, c.x, c.ff, L.a64.weight, c.rr, -1.0, nb);
        k_dot(c, c.rr, c.rr, nt, S_RR, 0, nb);
        check(it);
      }
    } else if (c.opt.outer == IGAMG_OUTER_IR) {
      // iterative refinement: inner PCG in the cycle arithmetic on the
      // float64 residual, to a fixed relative reduction or, when that is
      // more than the tolerance still needs, to half the remaining gap
      // (||r_in|| <= max(1e-4 ||r||, tol ||f|| / 2): the last step does not
      // over-solve); x += d; the float64 residual decides convergence
      constexpr double INNER_REDUCTION = 1e-4, LAST_STEP_MARGIN = 0.5;
      double *x_out = c.x, *r_out = c.rr;
      std::vector<int> outer_active(c.h_active, c.h_active + nb);
      std::vector<int> total(nb, 0);
      std::vector<double> ref(nb);
      for (int step = 1; step <= maxit && n_active > 0; ++step) {
        for (int j = 0; j < nb; ++j) ref[j] = res[j] * nf[j];
        int inner_active = n_active;
        // after an inner update of S_RR: stop the right-hand sides whose
        // inner residual met its target; false once none is left
        auto inner_continue = [&]() {
          read_scalars(c, nb);
          bool changed = false;
          for (int j = 0; j < nb; ++j) {
            if (!c.h_active[j]) continue;
            ++total[j];
            const double rin = std::sqrt(c.h_scal[(size_t)j * S_COUNT + S_RR]);
            const double target = std::max(INNER_REDUCTION * ref[j], LAST_STEP_MARGIN * tol * nf[j]);
            if (rin <= target || total[j] >= maxit) {
              c.h_active[j] = 0;
              --inner_active;
              changed = true;
            }
          }
          if (inner_active == 0) return false;
          if (changed) upload_active(c, nb);
          return true;
        };
        if (c.fp32()) {
          // float32 cycle: the inner PCG runs in float32 vectors (sums in
          // float64); z is the finest float32 iterate, cleared by each update
          float *z32 = L.a32.u;
          const size_t bytes32 = (size_t)nt * nb * sizeof(float);
          k_convert<double, float>(r_out, nullptr, c.r32, nt, nb, c.stream);
          k_fill(c.d32, 0.0f, nt * nb, c.stream);
          k_fill(z32, 0.0f, nt * nb, c.stream);
          precondition(c, c.r32, nb);
          k_dot(c, c.r32, z32, nt, S_RZ, 0, nb);
          HIPCHK(hipMemcpyAsync(c.p32, z32, bytes32, hipMemcpyDeviceToDevice, c.stream));
          for (;;) {
            apply_inner(c, c.p32, c.q32, nb);                          // q = A p
            k_dot(c, c.p32, c.q32, nt, S_PQ, 1, nb);                   // alpha = rz / pq
            k_pcg_update_xr(c, c.d32, c.r32, c.p32, c.q32, z32, nt, nb);  // z = 0
            if (!inner_continue()) break;
            precondition(c, c.r32, nb);
            k_dot(c, c.r32, z32, nt, S_RZNEW, 2, nb);  // beta = rz_new / rz
            k_pcg_update_p(c, c.p32, z32, nt, nb);     // p = z + beta p
          }
          for (int j = 0; j < nb; ++j) c.h_active[j] = outer_active[j];
          upload_active(c, nb);
          k_add_active(c, c.x, c.d32, nt, nb);  // x += d
        } else {
          HIPCHK(hipMemcpyAsync(c.rin, r_out, bytes, hipMemcpyDeviceToDevice, c.stream));
          k_fill(c.dd, 0.0, nt * nb, c.stream);
          c.x = c.dd;
          c.rr = c.rin;
          k_fill(c.z, 0.0, nt * nb, c.stream);
          precondition(c, c.rr, nb);
          k_dot(c, c.rr, c.z, nt, S_RZ, 0, nb);
          HIPCHK(hipMemcpyAsync(c.pp, c.z, bytes, hipMemcpyDeviceToDevice, c.stream));
          for (;;) {
            apply_inner(c, c.pp, c.qq, nb);          // q = A p
            k_dot(c, c.pp, c.qq, nt, S_PQ, 1, nb);    // alpha = rz / pq
            k_pcg_update_xr(c, nt, nb, false);       // d += alpha p, r -= alpha q; z = 0
            if (!inner_continue()) break;
            precondition(c, c.rr, nb);
            k_dot(c, c.rr, c.z, nt, S_RZNEW, 2, nb);  // beta = rz_new / rz
            k_pcg_update_p(c, nt, nb);                  // p = z + beta p
          }
          c.x = x_out;
          c.rr = r_out;
          for (int j = 0; j < nb; ++j) c.h_active[j] = outer_active[j];
          upload_active(c, nb);
          k_add_active(c, c.x, c.dd, nt, nb);  // x += d
        }
        apply64(c, c.x, c.ff, L.a64.weight, c.rr, -1.0, nb);  // r = f - A x (float64)
        k_dot(c, c.rr, c.rr, nt, S_RR, 0, nb);
        read_scalars(c, nb);
        bool changed = false;
        for (int j = 0; j < nb; ++j) {
          if (!outer_active[j]) continue;
          res[j] = std::sqrt(c.h_scal[(size_t)j * S_COUNT + S_RR]) / nf[j];
          its[j] = total[j];
          if (info && info[j].history) info[j].history[step] = res[j];
          if (res[j] <= tol || total[j] >= maxit) {
            outer_active[j] = 0;
            c.h_active[j] = 0;
            --n_active;
            changed = true;
          }
        }
        if (changed && n_active > 0) upload_active(c, nb);
      }
    } else {
      const bool fcg = c.opt.outer == IGAMG_OUTER_FCG;
      if (!c.fp32()) k_fill(c.z, 0.0, nt * nb, c.stream);
      precondition(c, c.rr, nb);
      k_dot(c, c.rr, c.z, nt, S_RZ, 0, nb);
      HIPCHK(hipMemcpyAsync(c.pp, c.z, bytes, hipMemcpyDeviceToDevice, c.stream));
      for (int it = 1; it <= maxit; ++it) {
        apply64(c, c.pp, nullptr, nullptr, c.qq, 1.0, nb);  // q = A p
        k_dot(c, c.pp, c.qq, nt, S_PQ, 1, nb);               // alpha = rz / pq
        k_pcg_update_xr(c, nt, nb, fcg);  // x += alpha p, r -= alpha q, rr; z = 0
        HIPCHK(hipMemcpyAsync(c.h_scal, c.d_scal, (size_t)nb * S_COUNT * sizeof(double),
                              hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipEventRecord(c.ev_scal, c.stream));
        // The next step's preconditioner is queued before the convergence
        // test waits, so the device does not idle during it, unless this
        // step is predicted to converge (residual times its last reduction
        // within 3 tol for some right-hand side), where a queued cycle would
        // only delay the return.  It writes only z and p: the iterate and
        // residual of a right-hand side that has converged at this step stay
        // as they are (the updated mask freezes them from the next update on).
        bool ahead = it < maxit;
        for (int j = 0; j < nb && ahead; ++j) {
          if (!c.h_active[j]) continue;
          const double rate = res_prev[j] > 0 ? res[j] / res_prev[j] : 1.0;
          if (res[j] * rate <= 3.0 * tol) ahead = false;
        }
        if (ahead) {
          precondition(c, c.rr, nb);
          if (fcg)
            k_dot_fcg(c, nt, nb);  // beta = (z, r - r_old) / rz
          else
            k_dot(c, c.rr, c.z, nt, S_RZNEW, 2, nb);  // beta = rz_new / rz
          k_pcg_update_p(c, nt, nb);                  // p = z + beta p
        }
        HIPCHK(hipEventSynchronize(c.ev_scal));
        tally(it);
        if (n_active == 0) break;
        if (!ahead && it < maxit) {
          precondition(c, c.rr, nb);
          if (fcg)
            k_dot_fcg(c, nt, nb);
          else
            k_dot(c, c.rr, c.z, nt, S_RZNEW, 2, nb);
          k_pcg_update_p(c, nt, nb);
        }
      }
    }
  }
  k_gather_compact(c.x, L.N, c.d_fin_cp, c.d_fin_cidx, 0, u, nt, nb, c.stream);
  // true residual in float64
  apply64(c, c.x, c.ff, L.a64.weight, c.qq, -1.0, nb);
  k_dot(c, c.qq, c.qq, nt, S_TMP, 0, nb);
  read_scalars(c, nb);
  auto t1 = std::chrono::steady_clock::now();
  int status = IGAMG_OK;
  for (int j = 0; j < nb; ++j) {
    const bool ok = nf[j] == 0 || res[j] <= tol;
    if (!ok) status = IGAMG_ENOCONV;
    if (info) {
      info[j].iterations = its[j];
      info[j].rel_residual = res[j];
      info[j].true_rel_residual =
          nf[j] > 0 ? std::sqrt(c.h_scal[(size_t)j * S_COUNT + S_TMP]) / nf[j] : 0.0;
      info[j].seconds = std::chrono::duration<double>(t1 - t0).count();
    }
  }
  // leave every right-hand side active for the next call's kernels (the
  // stream was synchronized above, so no copy still reads the mirror)
  for (int j = 0; j < nb; ++j) c.h_active[j] = 1;
  upload_active(c, nb);
  return status;
}

}  // namespace igamg
