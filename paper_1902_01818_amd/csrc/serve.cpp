// Serving runtime: continuous batching of heterogeneous solve requests on one
// GPU.  Requests are admitted in arrival order whenever a worker slot is free
// and a contiguous block of the device memory pool can hold the request's
// footprint (igamg_footprint); each admitted request builds its hierarchy
// inside its block (no driver allocation while others run), solves on the
// worker's own stream, and returns its block when done.  Requests of
// different sizes, degrees and patch counts therefore run side by side on
// the device, and a request arriving while others run starts as soon as a
// slot and memory free up.  (Declarations and contracts: include/igamg.h.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "context.h"

namespace igamg {
namespace {

// First-fit sub-allocator over one device buffer (offsets, 256-byte units).
class Pool {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
  }
  bool take(size_t n, size_t *off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    return false;
  }
  void give(size_t off, size_t n) {
    n = round(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t cap() const { return cap_; }

 private:
  static size_t round(size_t n) { return (n + 255) / 256 * 256; }
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Request {
  int64_t id = 0;
  int dim = 2, K = 0, degree = 1;
  double sigma = 5.0, tol = 1e-8;
  int maxit = 200;
  igamg_options opt{};
  std::vector<double> corners;
  std::vector<int32_t> elems;
  std::vector<double> rhs, u;
  size_t footprint = 0;
  igamg_request_info info{};
  bool done = false;
};

}  // namespace
}  // namespace igamg

struct igamg_server {
  igamg_server_config cfg{};
  char *base = nullptr;
  igamg::Pool pool;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<igamg::Request *> queue;
  std::map<int64_t, std::unique_ptr<igamg::Request>> reqs;
  std::vector<std::thread> workers;
  int64_t next_id = 1;
  int running = 0;
  int64_t completed = 0;
  bool stop = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker_loop(int slot);
};

void igamg_server::worker_loop(int slot) {
  (void)slot;
  if (hipSetDevice(cfg.device) != hipSuccess) return;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
  void *pinned = nullptr;
  const size_t pinned_bytes = 4096;
  if (hipHostMalloc(&pinned, pinned_bytes, hipHostMallocDefault) != hipSuccess) pinned = nullptr;
  for (;;) {
    igamg::Request *r = nullptr;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(m);
      // admission in arrival order: the head request waits for a block
      cv_work.wait(lk, [&] {
        if (stop && queue.empty()) return true;
        if (queue.empty()) return false;
        igamg::Request *h = queue.front();
        if (h->footprint > pool.cap()) return true;  // can never fit: rejected below
        return pool.take(h->footprint, &off);
      });
      if (queue.empty()) break;
      r = queue.front();
      queue.pop_front();
      if (r->footprint > pool.cap()) {
        r->info.status = IGAMG_ENOMEM;
        r->info.t_admit = r->info.t_ready = r->info.t_done = now();
        r->done = true;
        ++completed;
        cv_done.notify_all();
        cv_work.notify_all();
        continue;
      }
      ++running;
      r->info.t_admit = now();
    }
    cv_work.notify_all();  // the next head may fit as well
    int status = IGAMG_OK;
    std::unique_ptr<igamg::Context> cp;
    try {
      cp = std::make_unique<igamg::Context>();
      igamg::Context &c = *cp;
      igamg::Lent lent;
      lent.device = base + off;
      lent.device_bytes = r->footprint;
      lent.pinned = pinned;
      lent.pinned_bytes = pinned ? pinned_bytes : 0;
      igamg_patches P{r->dim, r->K, r->corners.data(), r->elems.data()};
      igamg::build_context(c, &P, r->degree, r->sigma, &r->opt, s, &lent);
      igamg::LevelData &L = c.lv.back();
      double *d_rhs = c.arena.alloc<double>(L.N);
      double *d_u = c.arena.alloc<double>(L.N);
      HIPCHK(hipMemcpyAsync(d_rhs, r->rhs.data(), L.N * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      r->info.t_ready = now();
      igamg_solve_info si{};
      status = igamg::solve_batch(c, d_rhs, d_u, 1, r->tol, r->maxit, 0, &si);
      HIPCHK(hipGetLastError());  // a launch that failed inside the solve
      r->u.resize(L.N);
      HIPCHK(hipMemcpyAsync(r->u.data(), d_u, L.N * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      r->info.iterations = si.iterations;
      r->info.rel_residual = si.rel_residual;
      r->info.true_rel_residual = si.true_rel_residual;
      r->info.n_dofs = L.N;
      r->info.fallback_allocations = c.arena.fallbacks;
    } catch (const igamg::Error &e) {
      status = e.code;
    } catch (...) {
      status = IGAMG_EINVAL;
    }
    // the request's kernels finish before its context, and the arrays it
    // allocated outside its block, are released
    (void)hipStreamSynchronize(s);
    cp.reset();
    {
      std::lock_guard<std::mutex> lk(m);
      pool.give(off, r->footprint);
      --running;
      ++completed;
      r->info.status = status;
      r->info.t_done = now();
      r->done = true;
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
  if (pinned) (void)hipHostFree(pinned);
  (void)hipStreamDestroy(s);
}

namespace igamg {
void set_last_error(const std::string &msg);  // capi.cpp: igamg_last_error's message
}

namespace {
template <typename F>
int guarded_srv(F &&f) {
  try {
    return f();
  } catch (const igamg::Error &e) {
    igamg::set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    igamg::set_last_error("host allocation failed");
    return IGAMG_ENOMEM;
  } catch (...) {
    igamg::set_last_error("unknown error");
    return IGAMG_EINVAL;
  }
}
}  // namespace

extern "C" {

int igamg_problem_size(const igamg_patches *patches, int degree, const igamg_options *o,
                       int64_t *n_dofs, int *levels) {
  return guarded_srv([&] {
    if (!n_dofs) igamg::fail(IGAMG_EINVAL, "null argument");
    long long n = 0;
    int lv = 0;
    igamg::problem_size(patches, degree, o, &n, &lv);
    *n_dofs = n;
    if (levels) *levels = lv;
    return IGAMG_OK;
  });
}

int igamg_server_create(const igamg_server_config *cfg, igamg_server **out) {
  return guarded_srv([&] {
    if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->memory_budget < (1u << 20))
      igamg::fail(IGAMG_EINVAL, "invalid server configuration");
    *out = nullptr;
    auto srv = std::make_unique<igamg_server>();
    srv->cfg = *cfg;
    HIPCHK(hipSetDevice(cfg->device));
    void *p = nullptr;
    if (hipMalloc(&p, cfg->memory_budget) != hipSuccess)
      igamg::fail(IGAMG_ENOMEM, "memory budget cannot be allocated");
    srv->base = (char *)p;
    srv->pool.init(cfg->memory_budget);
    for (int i = 0; i < cfg->slots; ++i)
      srv->workers.emplace_back([s = srv.get(), i] { s->worker_loop(i); });
    *out = srv.release();
    return IGAMG_OK;
  });
}

int igamg_server_submit(igamg_server *srv, const igamg_patches *patches, int degree,
                        double penalty_sigma, const igamg_options *o, const double *rhs,
                        int64_t n_dofs, double tol, int maxit, int64_t *request_id) {
  return guarded_srv([&] {
    if (!srv || !patches || !o || !rhs || !request_id || maxit < 0 || !(tol >= 0))
      igamg::fail(IGAMG_EINVAL, "invalid argument");
    const double t_submit = srv->now();
    // float32 requests are switched off in the serving runtime: their first
    // run aborted the process for a reason not yet identified
    if (o->precision != IGAMG_FP64)
      igamg::fail(IGAMG_EUNSUPPORTED, "the serving runtime takes float64 requests only");
    if (patches->degrees)
      igamg::fail(IGAMG_EUNSUPPORTED, "the serving runtime takes one degree per request");
    long long n = 0;
    int lv = 0;
    igamg::problem_size(patches, degree, o, &n, &lv);
    if (n != n_dofs) igamg::fail(IGAMG_EINVAL, "right-hand side length does not match the problem");
    igamg_options oo = *o;
    oo.max_rhs = 1;
    oo.timing = 0;
    oo.graphs = 1;  // the preconditioner cycle of every request replays a captured graph
    size_t fp = igamg::estimate_footprint(patches, degree, &oo);
    fp += 2 * (size_t)n * sizeof(double) + (1u << 20);  // right-hand side, solution, slack
    auto r = std::make_unique<igamg::Request>();
    r->dim = patches->dim;
    r->K = patches->n_patches;
    r->degree = degree;
    r->sigma = penalty_sigma;
    r->tol = tol;
    r->maxit = maxit;
    r->opt = oo;
    const int nc = 1 << patches->dim;
    r->corners.assign(patches->corners, patches->corners + (size_t)r->K * nc * r->dim);
    r->elems.assign(patches->elems, patches->elems + (size_t)r->K * r->dim);
    r->rhs.assign(rhs, rhs + n);
    r->footprint = fp;
    r->info.footprint = fp;
    r->info.n_dofs = n;
    r->info.t_submit = t_submit;
    {
      std::lock_guard<std::mutex> lk(srv->m);
      if (srv->stop) igamg::fail(IGAMG_EINVAL, "server is shutting down");
      r->id = srv->next_id++;
      *request_id = r->id;
      srv->queue.push_back(r.get());
      srv->reqs[r->id] = std::move(r);
    }
    srv->cv_work.notify_all();
    return IGAMG_OK;
  });
}

int igamg_server_wait(igamg_server *srv, int64_t request_id, double *u, igamg_request_info *info) {
  return guarded_srv([&] {
    if (!srv) igamg::fail(IGAMG_EINVAL, "null server");
    std::unique_ptr<igamg::Request> r;
    {
      std::unique_lock<std::mutex> lk(srv->m);
      auto it = srv->reqs.find(request_id);
      if (it == srv->reqs.end()) igamg::fail(IGAMG_EINVAL, "unknown request id");
      igamg::Request *rp = it->second.get();
      srv->cv_done.wait(lk, [&] { return rp->done; });
      r = std::move(it->second);
      srv->reqs.erase(it);
    }
    if (u && !r->u.empty()) std::memcpy(u, r->u.data(), r->u.size() * sizeof(double));
    if (info) *info = r->info;
    return r->info.status;
  });
}

int igamg_server_status(igamg_server *srv, int *queued, int *running, int64_t *completed,
                        size_t *reserved_bytes, size_t *peak_reserved_bytes) {
  return guarded_srv([&] {
    if (!srv) igamg::fail(IGAMG_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(srv->m);
    if (queued) *queued = (int)srv->queue.size();
    if (running) *running = srv->running;
    if (completed) *completed = srv->completed;
    if (reserved_bytes) *reserved_bytes = srv->pool.used();
    if (peak_reserved_bytes) *peak_reserved_bytes = srv->pool.peak();
    return IGAMG_OK;
  });
}

int igamg_server_destroy(igamg_server *srv) {
  return guarded_srv([&] {
    if (!srv) return IGAMG_OK;
    {
      std::lock_guard<std::mutex> lk(srv->m);
      srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    if (srv->base) (void)hipFree(srv->base);
    delete srv;
    return IGAMG_OK;
  });
}

}  // extern "C"
