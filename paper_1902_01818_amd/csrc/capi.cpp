// extern "C" boundary of the library (declarations and contracts: include/igamg.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "context.h"
#include "hostmath.h"
#include "kernels.h"

struct igamg_ctx {
  igamg::Context c;
};

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace igamg {
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace igamg

namespace {

template <typename F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const igamg::Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return IGAMG_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return IGAMG_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return IGAMG_EINVAL;
  }
}

void flush_timers(igamg::Context &c) {
  HIPCHK(hipStreamSynchronize(c.stream));
  for (auto &kv : c.timers) {
    for (auto &pe : kv.second.pending) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pe.first, pe.second));
      kv.second.ms += ms;
      kv.second.pool.push_back(pe);
    }
    kv.second.pending.clear();
  }
}

// Host tables of the L2 error: the (p+3)-point rule, per distinct element
// count the basis values at its points, per patch and direction the table
// offset, and the first element of every patch.
struct L2Tables {
  igamg::GaussRule gq;
  std::vector<double> tB;
  std::vector<int> tab;
  std::vector<long long> el_off{0};
  long long nel = 0;
  // (p+3)-point rule with p the largest degree, on every patch
  explicit L2Tables(const igamg::Context &c) : gq(igamg::gauss_rule(c.p + 3)) {
    const igamg::LevelData &L = c.lv.back();
    tab.assign(3 * L.K, 0);
    std::map<std::pair<int, int>, int> tab_of;
    for (int k = 0; k < L.K; ++k) {
      long long ne = 1;
      for (int g = 0; g < c.d; ++g) {
        const int n = L.pd[k].nel[g];
        ne *= n;
        auto it = tab_of.find({n, L.pd[k].p});
        if (it == tab_of.end()) {
          std::vector<double> B, D;
          igamg::element_tables(n, L.pd[k].p, gq, B, D);
          it = tab_of.emplace(std::make_pair(n, L.pd[k].p), (int)tB.size()).first;
          tB.insert(tB.end(), B.begin(), B.end());
        }
        tab[3 * k + g] = it->second;
      }
      el_off.push_back(el_off.back() + ne);
    }
    nel = el_off.back();
  }
};

// device arrays of one L2 error evaluation (scratch owned by the caller)
struct L2Buffers {
  double *tB = nullptr;
  int *tab = nullptr;
  long long *el_off = nullptr;
  double *part = nullptr;  // l2_error_partials(nel) block sums
  double *out = nullptr;   // one value
};

// Upload the tables, scatter u to the torn layout (context work vector x),
// sum the squared error in a fixed order, read it back (synchronizes).
double l2_error_run(igamg::Context &c, const L2Tables &t, const L2Buffers &b, const double *u) {
  igamg::LevelData &L = c.lv.back();
  HIPCHK(hipMemcpyAsync(b.tB, t.tB.data(), t.tB.size() * sizeof(double), hipMemcpyHostToDevice,
                        c.stream));
  HIPCHK(hipMemcpyAsync(b.tab, t.tab.data(), t.tab.size() * sizeof(int), hipMemcpyHostToDevice,
                        c.stream));
  HIPCHK(hipMemcpyAsync(b.el_off, t.el_off.data(), t.el_off.size() * sizeof(long long),
                        hipMemcpyHostToDevice, c.stream));
  const long long nt = L.Ntorn;
  igamg::k_fill(c.x, 0.0, nt, c.stream);
  igamg::k_scatter_compact(u, L.N, c.d_fin_cp, c.d_fin_cidx, c.x, nt, 1, c.stream);
  igamg::k_l2_error(c, L, c.x, b.el_off, b.tab, b.tB, t.gq, b.part, t.nel, b.out);
  double e2 = 0.0;
  HIPCHK(hipMemcpyAsync(&e2, b.out, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return std::sqrt(e2);
}
}  // namespace

extern "C" {

void igamg_default_options(igamg_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->discretization = IGAMG_SIPG;
  o->smoother = IGAMG_SMOOTHER_HYBRID;
  o->mu = 1;
  o->nu = 1;
  o->damping_tau = 0.25;
  o->scaling_delta = 0.1;
  o->precision = IGAMG_FP64;
  o->outer = IGAMG_OUTER_PCG;
  o->gs_tile = 0;
  o->coarse_min = 0;
  o->timing = 0;
  o->max_rhs = 0;
  o->operator_apply = IGAMG_APPLY_AUTO;
  o->graphs = 0;
}

int igamg_footprint(const igamg_patches *patches, int degree, const igamg_options *o, int nrhs,
                    size_t *bytes) {
  return guarded([&] {
    if (!bytes || !o || nrhs < 0) igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg_options oo = *o;
    if (nrhs > 0) oo.max_rhs = nrhs;
    *bytes = igamg::estimate_footprint(patches, degree, &oo);
    return IGAMG_OK;
  });
}

int igamg_setup(const igamg_patches *patches, int degree, double penalty_sigma,
                const igamg_options *o, void *stream, igamg_ctx **out) {
  return guarded([&] {
    if (!out) igamg::fail(IGAMG_EINVAL, "null output pointer");
    *out = nullptr;
    igamg_ctx *ctx = new igamg_ctx();
    try {
      igamg::build_context(ctx->c, patches, degree, penalty_sigma, o, (hipStream_t)stream);
      // device scratch of the allocation-free entry points: its address on
      // this device, looked up once per device
      igamg::noalloc_scratch_init();
    } catch (...) {
      (void)hipStreamSynchronize((hipStream_t)stream);
      delete ctx;
      throw;
    }
    *out = ctx;
    return IGAMG_OK;
  });
}

int igamg_num_dofs(const igamg_ctx *ctx, int64_t *n) {
  return guarded([&] {
    if (!ctx || !n) igamg::fail(IGAMG_EINVAL, "null argument");
    *n = ctx->c.lv.back().N;
    return IGAMG_OK;
  });
}

int igamg_num_levels(const igamg_ctx *ctx, int *levels) {
  return guarded([&] {
    if (!ctx || !levels) igamg::fail(IGAMG_EINVAL, "null argument");
    *levels = (int)ctx->c.lv.size();
    return IGAMG_OK;
  });
}

int igamg_apply(igamg_ctx *ctx, const double *x, double *y, int nrhs, void *stream) {
  return guarded([&] {
    if (!ctx || !x || !y || nrhs < 1) igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    igamg::LevelData &L = c.lv.back();
    const long long nt = L.Ntorn;
    for (int j0 = 0; j0 < nrhs; j0 += c.nb) {
      const int nb = std::min(c.nb, nrhs - j0);
      igamg::k_fill(c.x, 0.0, nt * nb, c.stream);
      igamg::k_scatter_compact(x + (size_t)j0 * L.N, L.N, c.d_fin_cp, c.d_fin_cidx, c.x, nt, nb,
                               c.stream);
      igamg::apply64(c, c.x, nullptr, nullptr, c.qq, 1.0, nb);
      igamg::k_gather_compact(c.qq, L.N, c.d_fin_cp, c.d_fin_cidx, 0, y + (size_t)j0 * L.N, nt, nb,
                              c.stream);
    }
    HIPCHK(hipGetLastError());
    return IGAMG_OK;
  });
}

int igamg_vcycle(igamg_ctx *ctx, const double *f, double *u, int nrhs, void *stream) {
  return guarded([&] {
    if (!ctx || !f || !u || nrhs < 1) igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    const long long N = c.lv.back().N;
    for (int j0 = 0; j0 < nrhs; j0 += c.nb) {
      const int nb = std::min(c.nb, nrhs - j0);
      igamg::vcycle_compact(c, f + (size_t)j0 * N, u + (size_t)j0 * N, nb);
    }
    HIPCHK(hipGetLastError());
    return IGAMG_OK;
  });
}

int igamg_solve(igamg_ctx *ctx, const double *rhs, double *u, int nrhs, double tol, int maxit,
                int use_initial_guess, igamg_solve_info *info, void *stream) {
  return guarded([&] {
    if (!ctx || !rhs || !u || nrhs < 1 || maxit < 0 || !(tol >= 0))
      igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    const long long N = c.lv.back().N;
    int status = IGAMG_OK;
    for (int j0 = 0; j0 < nrhs; j0 += c.nb) {
      const int nb = std::min(c.nb, nrhs - j0);
      int s = igamg::solve_batch(c, rhs + (size_t)j0 * N, u + (size_t)j0 * N, nb, tol, maxit,
                                 use_initial_guess, info ? info + j0 : nullptr);
      if (s != IGAMG_OK) status = s;
    }
    HIPCHK(hipGetLastError());
    return status;
  });
}

int igamg_load_manufactured(igamg_ctx *ctx, int which, double *f, void *stream) {
  return guarded([&] {
    if (!ctx || !f || which != IGAMG_MANUFACTURED_SINE)
      igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    igamg::LevelData &L = c.lv.back();
    igamg::k_load_manufactured(c, L, c.qq);
    // every copy holds its patch's integral: the assembled value is their sum
    igamg::k_gather_compact(c.qq, L.N, c.d_fin_cp, c.d_fin_cidx, 1, f, L.Ntorn, 1, c.stream);
    HIPCHK(hipGetLastError());
    return IGAMG_OK;
  });
}

int igamg_l2_error(igamg_ctx *ctx, const double *u, int which, double *err_host, void *stream) {
  return guarded([&] {
    if (!ctx || !u || !err_host || which != IGAMG_MANUFACTURED_SINE)
      igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    L2Tables t(c);
    igamg::DeviceScratch s_tB, s_tab, s_eloff, s_part, s_out;
    L2Buffers b{s_tB.alloc<double>(t.tB.size()), s_tab.alloc<int>(t.tab.size()),
                s_eloff.alloc<long long>(t.el_off.size()),
                s_part.alloc<double>((size_t)igamg::l2_error_partials(t.nel)),
                s_out.alloc<double>(1)};
    *err_host = l2_error_run(c, t, b, u);  // synchronizes: scratch freed at scope exit
    return IGAMG_OK;
  });
}

int igamg_l2_error_noalloc(igamg_ctx *ctx, const double *u, int which, double *err_host,
                           void *stream) {
  return guarded([&] {
    if (!ctx || !u || !err_host || which != IGAMG_MANUFACTURED_SINE)
      igamg::fail(IGAMG_EINVAL, "invalid argument");
    igamg::Context &c = ctx->c;
    c.stream = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != c.device)
      igamg::fail(IGAMG_EINVAL, "the context's device is not the current device");
    // looked up once per device by igamg_setup (or here on the first call)
    char *base = (char *)igamg::noalloc_scratch(dev);
    if (!base) base = (char *)igamg::noalloc_scratch_init();
    L2Tables t(c);
    // carve the device scratch: each array on a 256-byte boundary
    size_t at = 0;
    auto carve = [&](size_t bytes) {
      const size_t o = at;
      at += (bytes + 255) / 256 * 256;
      return base + o;
    };
    L2Buffers b;
    b.out = (double *)carve(sizeof(double));
    b.el_off = (long long *)carve(t.el_off.size() * sizeof(long long));
    b.tab = (int *)carve(t.tab.size() * sizeof(int));
    b.tB = (double *)carve(t.tB.size() * sizeof(double));
    b.part = (double *)carve((size_t)igamg::l2_error_partials(t.nel) * sizeof(double));
    if (at > igamg::NOALLOC_SCRATCH_BYTES)
      igamg::fail(IGAMG_EUNSUPPORTED,
                  "problem needs " + std::to_string(at) + " bytes of device scratch; the "
                  "allocation-free L2 error holds at most " +
                      std::to_string(igamg::NOALLOC_SCRATCH_BYTES) + " bytes");
    *err_host = l2_error_run(c, t, b, u);
    return IGAMG_OK;
  });
}

int igamg_memory(const igamg_ctx *ctx, size_t *bytes) {
  return guarded([&] {
    if (!ctx || !bytes) igamg::fail(IGAMG_EINVAL, "null argument");
    *bytes = ctx->c.arena.bytes;
    return IGAMG_OK;
  });
}

int igamg_kernel_stats(igamg_ctx *ctx, int cap, char (*names)[32], double *ms, int64_t *launches,
                       int *count, int reset) {
  return guarded([&] {
    if (!ctx || !count) igamg::fail(IGAMG_EINVAL, "null argument");
    igamg::Context &c = ctx->c;
    flush_timers(c);
    int n = 0;
    for (auto &kv : c.timers) {
      if (n < cap) {
        if (names) {
          std::strncpy(names[n], kv.first.c_str(), 31);
          names[n][31] = 0;
        }
        if (ms) ms[n] = kv.second.ms;
        if (launches) launches[n] = kv.second.launches;
      }
      ++n;
      if (reset) {
        kv.second.ms = 0;
        kv.second.launches = 0;
      }
    }
    *count = n < cap ? n : cap;
    return IGAMG_OK;
  });
}

int igamg_kernel_model(igamg_ctx *ctx, const char *family, int level, int nrhs, double *bytes,
                       double *flops) {
  return guarded([&] {
    if (!ctx || !family || !bytes || !flops) igamg::fail(IGAMG_EINVAL, "null argument");
    igamg::Context &c = ctx->c;
    if (level < 0) level = (int)c.lv.size() - 1;
    if (level >= (int)c.lv.size()) igamg::fail(IGAMG_EINVAL, "level out of range");
    if (nrhs < 1) igamg::fail(IGAMG_EINVAL, "nrhs must be positive");
    igamg::kernel_model(c, family, level, nrhs, bytes, flops);
    return IGAMG_OK;
  });
}

int igamg_set_timing(igamg_ctx *ctx, const char *filter) {
  return guarded([&] {
    if (!ctx) igamg::fail(IGAMG_EINVAL, "null argument");
    igamg::Context &c = ctx->c;
    c.opt.timing = filter ? 1 : 0;
    c.timing_filter = filter ? filter : "";
    return IGAMG_OK;
  });
}

int igamg_destroy(igamg_ctx *ctx) {
  return guarded([&] {
    if (!ctx) return IGAMG_OK;
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
    return IGAMG_OK;
  });
}

const char *igamg_strerror(int code) {
  switch (code) {
    case IGAMG_OK: return "success";
    case IGAMG_EINVAL: return "invalid argument";
    case IGAMG_EUNSUPPORTED: return "unsupported input";
    case IGAMG_ENOMEM: return "out of device memory";
    case IGAMG_EHIP: return "HIP runtime error";
    case IGAMG_ENOCONV: return "tolerance not reached";
    default: return "unknown status";
  }
}

const char *igamg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
