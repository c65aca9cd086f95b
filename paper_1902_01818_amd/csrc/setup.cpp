// Setup of the multigrid hierarchy: topology of the patch layout, grid
// levels, unknown numbering, interface terms of the SIPG form, smoother data
// and the coarse factorization.  Host work is plain C++; the volume stencils
// of the Gauss-Seidel smoother are assembled on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <unordered_map>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>

#include "context.h"
#include "geom.h"
#include "hostmath.h"
#include "kernels.h"

namespace igamg {

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

int vol_tile_2d(int p);
int stencil_tile_2d(int p);

namespace {
// Host wall time of setup phases, printed to stderr when IGAMG_SETUP_TIMING is
// set (diagnostics of the setup cost that serving latency includes).
struct PhaseClock {
  bool on = std::getenv("IGAMG_SETUP_TIMING") != nullptr;
  std::map<std::string, double> acc;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char *name, hipStream_t s = nullptr, bool sync = false) {
    if (!on) return;
    if (sync) (void)hipStreamSynchronize(s);
    auto n = std::chrono::steady_clock::now();
    acc[name] += std::chrono::duration<double>(n - t).count();
    t = n;
  }
  void report(long long N) {
    if (!on) return;
    std::fprintf(stderr, "[igamg setup] N=%lld", N);
    for (auto &kv : acc) std::fprintf(stderr, " %s=%.1fms", kv.first.c_str(), kv.second * 1e3);
    std::fprintf(stderr, "\n");
  }
};
}  // namespace

// Host threads for setup loops: IGAMG_HOST_THREADS, else the hardware count,
// at most 16.
static int host_threads() {
  static const int n = [] {
    const char *e = std::getenv("IGAMG_HOST_THREADS");
    int v = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(16, v));
  }();
  return n;
}

// fn(i) for i in [0, n) on up to host_threads() threads (dynamic
// assignment); the first exception thrown by fn is rethrown after all
// threads have joined.
template <class F>
static void parallel_for(int n, F fn) {
  const int nt = std::min(n, host_threads());
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex em;
  auto work = [&] {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) return;
      try {
        fn(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(em);
        if (!err) err = std::current_exception();
        next.store(n);
        return;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto &t : th) t.join();
  if (err) std::rethrow_exception(err);
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
void Context::launch_begin(const char *fam, hipEvent_t *b, hipEvent_t *e) {
  TimerFamily &t = timers[fam];
  if (t.pool.empty()) {
    hipEvent_t x, y;
    HIPCHK(hipEventCreate(&x));
    HIPCHK(hipEventCreate(&y));
    t.pool.push_back({x, y});
  }
  *b = t.pool.back().first;
  *e = t.pool.back().second;
  t.pool.pop_back();
  HIPCHK(hipEventRecord(*b, stream));
}

void Context::launch_end(const char *fam, hipEvent_t b, hipEvent_t e, int launches) {
  TimerFamily &t = timers[fam];
  HIPCHK(hipEventRecord(e, stream));
  t.pending.push_back({b, e});
  t.launches += launches;
  if (t.pending.size() > 256) {  // bound the number of outstanding events
    HIPCHK(hipEventSynchronize(e));
    for (auto &pe : t.pending) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pe.first, pe.second));
      t.ms += ms;
      t.pool.push_back(pe);
    }
    t.pending.clear();
  }
}

Context::~Context() {
  for (auto &kv : timers) {
    for (auto &pe : kv.second.pending) {
      (void)hipEventDestroy(pe.first);
      (void)hipEventDestroy(pe.second);
    }
    for (auto &pe : kv.second.pool) {
      (void)hipEventDestroy(pe.first);
      (void)hipEventDestroy(pe.second);
    }
  }
  for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (ev_scal) (void)hipEventDestroy(ev_scal);
  if (own_pinned && h_scal) (void)hipHostFree(h_scal);
  if (own_pinned && h_active) (void)hipHostFree(h_active);
  arena.release();
}

// ---------------------------------------------------------------------------
// topology (Section 2, eq. omega:1 and Assumption 1)
// ---------------------------------------------------------------------------
static std::vector<int> side_corners(int d, int dir, int s) {
  std::vector<int> out;
  std::vector<int> tang;
  for (int g = 0; g < d; ++g)
    if (g != dir) tang.push_back(g);
  for (int tb = 0; tb < (1 << (d - 1)); ++tb) {
    int b = s << dir;
    for (size_t j = 0; j < tang.size(); ++j) b |= ((tb >> j) & 1) << tang[j];
    out.push_back(b);
  }
  return out;
}

static void build_topology(Context &c) {
  const int d = c.d, K = c.K, nc = 1 << d;
  std::map<std::array<long long, 3>, int> keys;
  c.vid.assign(K, std::vector<int>(nc));
  for (int k = 0; k < K; ++k)
    for (int b = 0; b < nc; ++b) {
      std::array<long long, 3> key{0, 0, 0};
      for (int a = 0; a < d; ++a) key[a] = std::llround(c.corners[k][b * 3 + a] * 1e9);
      auto it = keys.find(key);
      if (it == keys.end()) it = keys.emplace(key, (int)keys.size()).first;
      c.vid[k][b] = it->second;
    }
  c.boundary.assign(K, std::array<unsigned char, 6>{1, 1, 1, 1, 1, 1});
  for (int k = 0; k < K; ++k)
    for (int dir = d; dir < 3; ++dir) c.boundary[k][2 * dir] = c.boundary[k][2 * dir + 1] = 0;
  for (int k = 0; k < K; ++k)
    for (int l = k + 1; l < K; ++l)
      for (int dk = 0; dk < d; ++dk)
        for (int sk = 0; sk < 2; ++sk) {
          std::vector<int> ck = side_corners(d, dk, sk);
          std::vector<int> vk;
          for (int b : ck) vk.push_back(c.vid[k][b]);
          for (int dl = 0; dl < d; ++dl)
            for (int sl = 0; sl < 2; ++sl) {
              std::vector<int> cl = side_corners(d, dl, sl);
              std::vector<int> vl;
              for (int b : cl) vl.push_back(c.vid[l][b]);
              std::vector<int> a = vk, bb = vl;
              std::sort(a.begin(), a.end());
              std::sort(bb.begin(), bb.end());
              if (a != bb) continue;
              if (vk != vl) fail(IGAMG_EUNSUPPORTED, "interface with flipped orientation");
              c.ifaces.push_back({k, dk, sk, l, dl, sl, 0.0});
              c.boundary[k][2 * dk + sk] = 0;
              c.boundary[l][2 * dl + sl] = 0;
            }
        }
  // patch colours for the Gauss-Seidel order: SIPG separates patches with a
  // common side; the conforming space separates patches with a common corner
  // (a glued unknown couples every patch around its vertex or edge)
  std::vector<std::vector<int>> nbr(K);
  if (c.opt.discretization == IGAMG_CONFORMING) {
    for (int k = 0; k < K; ++k)
      for (int l = k + 1; l < K; ++l) {
        bool common = false;
        for (int a : c.vid[k])
          for (int b : c.vid[l]) common |= a == b;
        if (common) {
          nbr[k].push_back(l);
          nbr[l].push_back(k);
        }
      }
  } else {
    for (auto &f : c.ifaces) {
      nbr[f.k].push_back(f.l);
      nbr[f.l].push_back(f.k);
    }
  }
  c.color.assign(K, 0);
  c.n_colors = 1;
  for (int k = 0; k < K; ++k) {
    std::vector<char> taken(K + 1, 0);
    for (int j : nbr[k])
      if (j < k) taken[c.color[j]] = 1;
    int col = 0;
    while (taken[col]) ++col;
    c.color[k] = col;
    c.n_colors = std::max(c.n_colors, col + 1);
  }
  // patch measures (Gauss, exact for multilinear maps) and orientation check
  GaussRule g4 = gauss_rule(4);
  c.measure.assign(K, 0.0);
  for (int k = 0; k < K; ++k) {
    double cs[8][3] = {};
    for (int b = 0; b < nc; ++b)
      for (int a = 0; a < d; ++a) cs[b][a] = c.corners[k][b * 3 + a];
    int gi[3] = {0, 0, 0};
    double m = 0.0;
    for (;;) {
      double xh[3], w = 1.0;
      for (int a = 0; a < d; ++a) {
        xh[a] = g4.x[gi[a]];
        w *= g4.w[gi[a]];
      }
      double det;
      if (d == 2) {
        double J[2][2];
        multilinear_jac<2>(cs, xh, J);
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      } else {
        double J[3][3], Ji[3][3];
        multilinear_jac<3>(cs, xh, J);
        det = inverse<3>(J, Ji);
      }
      if (!(det > 0)) fail(IGAMG_EINVAL, "patch map with non-positive Jacobian determinant");
      m += w * det;
      int a = 0;
      while (a < d && ++gi[a] == 4) gi[a++] = 0;
      if (a == d) break;
    }
    c.measure[k] = m;
  }
  // penalty sigma p^2 / h with the finest physical element size (eq. a:galerkin)
  for (auto &f : c.ifaces) {
    auto h = [&](int k) {
      int ne = 0;
      for (int a = 0; a < d; ++a) ne = std::max(ne, c.elems_fine[k][a]);
      return std::pow(c.measure[k], 1.0 / d) / ne;
    };
    const double pkl = std::max(c.pk[f.k], c.pk[f.l]);
    f.eta = c.sigma_pen * pkl * pkl / std::min(h(f.k), h(f.l));
  }
}

// ---------------------------------------------------------------------------
// levels
// ---------------------------------------------------------------------------
static std::vector<std::vector<std::array<int, 3>>> level_elements(const Context &c) {
  std::vector<std::vector<std::array<int, 3>>> out;
  std::vector<std::array<int, 3>> e = c.elems_fine;
  out.push_back(e);
  int cmin = c.opt.coarse_min > 0 ? c.opt.coarse_min : 2;
  for (;;) {
    bool ok = true;
    for (auto &a : e)
      for (int g = 0; g < c.d; ++g)
        if (a[g] % 2 != 0 || a[g] / 2 < cmin) ok = false;
    if (!ok) break;
    for (auto &a : e)
      for (int g = 0; g < c.d; ++g) a[g] /= 2;
    out.push_back(e);
  }
  std::reverse(out.begin(), out.end());
  return out;
}

static long long torn_index(const PatchDev &pt, const int *i) {
  return pt.off + (long long)i[0] + (long long)i[1] * pt.stride[1] + (long long)i[2] * pt.stride[2];
}

static void build_level_dofs(Context &c, LevelData &L, const std::vector<std::array<int, 3>> &el) {
  const int d = c.d, K = c.K;
  L.K = K;
  L.pd.assign(K, PatchDev{});
  // element tables per (element count, degree), Gauss rule of p+1 points
  std::map<std::pair<int, int>, int> tab_of_nel;
  long long off = 0;
  for (int k = 0; k < K; ++k) {
    PatchDev &pt = L.pd[k];
    const int p = c.pk[k];
    pt.p = p;
    for (int b = 0; b < (1 << d); ++b)
      for (int a = 0; a < d; ++a) pt.corners[b][a] = c.corners[k][b * 3 + a];
    for (int g = 0; g < 3; ++g) {
      pt.nel[g] = g < d ? el[k][g] : 1;
      pt.n[g] = g < d ? el[k][g] + p : 1;
    }
    pt.stride[0] = 1;
    pt.stride[1] = pt.n[0];
    pt.stride[2] = pt.n[0] * pt.n[1];
    pt.off = off;
    off += (long long)pt.n[0] * pt.n[1] * pt.n[2];
    pt.color = c.color[k];
    for (int g = 0; g < d; ++g) {
      int ne = pt.nel[g];
      auto it = tab_of_nel.find({ne, p});
      if (it == tab_of_nel.end()) {
        std::vector<double> B, D;
        element_tables(ne, p, gauss_rule(p + 1), B, D);
        int o = (int)L.tabB.size();
        L.tabB.insert(L.tabB.end(), B.begin(), B.end());
        L.tabD.insert(L.tabD.end(), D.begin(), D.end());
        it = tab_of_nel.emplace(std::make_pair(ne, p), o).first;
      }
      pt.tab[g] = it->second;
    }
  }
  L.Ntorn = off;
  // Dirichlet: non-vanishing trace on a boundary side
  L.mask.assign(L.Ntorn, 1);
  for (int k = 0; k < K; ++k) {
    const PatchDev &pt = L.pd[k];
    for (long long loc = 0; loc < (long long)pt.n[0] * pt.n[1] * pt.n[2]; ++loc) {
      int i[3] = {(int)(loc % pt.n[0]), (int)((loc / pt.n[0]) % pt.n[1]),
                  (int)(loc / ((long long)pt.n[0] * pt.n[1]))};
      for (int g = 0; g < d; ++g)
        for (int s = 0; s < 2; ++s)
          if (c.boundary[k][2 * g + s] && i[g] == (s ? pt.n[g] - 1 : 0)) L.mask[pt.off + loc] = 0;
    }
  }
  // conforming: glue patch-boundary unknowns by their Greville points
  std::vector<int> group(L.Ntorn, -1);
  int ngroups = 0;
  if (c.opt.discretization == IGAMG_CONFORMING) {
    std::map<std::array<long long, 3>, int> gkey;
    for (int k = 0; k < K; ++k) {
      const PatchDev &pt = L.pd[k];
      const int p = pt.p;
      std::vector<std::vector<double>> grev(d);
      for (int g = 0; g < d; ++g) {
        std::vector<double> t = open_knots(pt.nel[g], p);
        for (int i = 0; i < pt.n[g]; ++i) {
          double s = 0;
          for (int j = 1; j <= p; ++j) s += t[i + j];
          grev[g].push_back(s / p);
        }
      }
      for (long long loc = 0; loc < (long long)pt.n[0] * pt.n[1] * pt.n[2]; ++loc) {
        int i[3] = {(int)(loc % pt.n[0]), (int)((loc / pt.n[0]) % pt.n[1]),
                    (int)(loc / ((long long)pt.n[0] * pt.n[1]))};
        bool bd = false;
        for (int g = 0; g < d; ++g) bd |= (i[g] == 0 || i[g] == pt.n[g] - 1);
        if (!bd) continue;
        double xh[3] = {0, 0, 0}, X[3] = {0, 0, 0};
        for (int g = 0; g < d; ++g) xh[g] = grev[g][i[g]];
        if (d == 2)
          multilinear_map<2>(pt.corners, xh, X);
        else
          multilinear_map<3>(pt.corners, xh, X);
        std::array<long long, 3> key{0, 0, 0};
        for (int a = 0; a < d; ++a) key[a] = std::llround(X[a] * 1e9);
        auto it = gkey.find(key);
        if (it == gkey.end()) it = gkey.emplace(key, ngroups++).first;
        group[pt.off + loc] = it->second;
      }
    }
    std::vector<unsigned char> gd(ngroups, 1);
    for (long long t = 0; t < L.Ntorn; ++t)
      if (group[t] >= 0 && !L.mask[t]) gd[group[t]] = 0;
    for (long long t = 0; t < L.Ntorn; ++t)
      if (group[t] >= 0) L.mask[t] = gd[group[t]];
    // Assumption 2: both sides of an interface carry the same glued unknowns
    for (auto &f : c.ifaces) {
      auto side_groups = [&](int k, int dir, int s) {
        std::vector<int> gs;
        const PatchDev &pt = L.pd[k];
        for (long long loc = 0; loc < (long long)pt.n[0] * pt.n[1] * pt.n[2]; ++loc) {
          int i[3] = {(int)(loc % pt.n[0]), (int)((loc / pt.n[0]) % pt.n[1]),
                      (int)(loc / ((long long)pt.n[0] * pt.n[1]))};
          if (i[dir] == (s ? pt.n[dir] - 1 : 0)) gs.push_back(group[pt.off + loc]);
        }
        std::sort(gs.begin(), gs.end());
        return gs;
      };
      if (side_groups(f.k, f.dk, f.sk) != side_groups(f.l, f.dl, f.sl))
        fail(IGAMG_EINVAL, "conforming discretization needs fully matching interfaces");
    }
  }
  // compact numbering
  L.comp.assign(L.Ntorn, -1);
  L.rep.clear();
  std::vector<int> gcomp(ngroups, -1);
  for (long long t = 0; t < L.Ntorn; ++t) {
    if (!L.mask[t]) continue;
    int g = group[t];
    if (g >= 0 && gcomp[g] >= 0) {
      L.comp[t] = gcomp[g];
      continue;
    }
    int ci = (int)L.rep.size();
    L.comp[t] = ci;
    L.rep.push_back((int)t);
    if (g >= 0) gcomp[g] = ci;
  }
  L.N = (long long)L.rep.size();
  // copies of every compact unknown (CSR, increasing torn index: the
  // representative first)
  L.copy_ptr.assign(L.N + 1, 0);
  for (long long t = 0; t < L.Ntorn; ++t)
    if (L.comp[t] >= 0) ++L.copy_ptr[L.comp[t] + 1];
  for (long long ci = 0; ci < L.N; ++ci) L.copy_ptr[ci + 1] += L.copy_ptr[ci];
  L.copy_idx.assign(L.copy_ptr[L.N], 0);
  {
    std::vector<int> fillp(L.copy_ptr.begin(), L.copy_ptr.end() - 1);
    for (long long t = 0; t < L.Ntorn; ++t)
      if (L.comp[t] >= 0) L.copy_idx[fillp[L.comp[t]]++] = (int)t;
  }
}

// ---------------------------------------------------------------------------
// SIPG interface terms (Section 3, eq. model:discr2) by Gauss quadrature on
// the union of both sides' breakpoints
// ---------------------------------------------------------------------------
static void build_interfaces(Context &c, LevelData &L) {
  const int d = c.d;
  // one sparse accumulator per interface (interfaces in parallel); the
  // per-interface sums are added in interface order below, so the result
  // does not depend on the number of threads
  std::vector<std::vector<std::pair<unsigned long long, double>>> per(c.ifaces.size());
  parallel_for((int)c.ifaces.size(), [&](int fi) {
    const Context::Iface &f = c.ifaces[fi];
    std::unordered_map<unsigned long long, double> acc;
    acc.reserve(1 << 12);
    const PatchDev &pk = L.pd[f.k], &pl = L.pd[f.l];
    // q = p+1 Gauss points per merged segment, p the larger degree of the sides
    const int q = std::max(pk.p, pl.p) + 1;
    const GaussRule gq = gauss_rule(q);
    const int ps[2] = {pk.p, pl.p};
    int tk[2], tl[2], nt = 0;
    for (int g = 0; g < d; ++g)
      if (g != f.dk) tk[nt++] = g;
    nt = 0;
    for (int g = 0; g < d; ++g)
      if (g != f.dl) tl[nt++] = g;
    // merged breakpoints per tangential direction: m / lcm
    std::vector<std::vector<double>> pts(d - 1), wts(d - 1);
    for (int j = 0; j < d - 1; ++j) {
      long long na = pk.nel[tk[j]], nb = pl.nel[tl[j]];
      long long Lc = std::lcm(na, nb);
      std::vector<long long> ms;
      for (long long i = 0; i <= na; ++i) ms.push_back(i * (Lc / na));
      for (long long i = 0; i <= nb; ++i) ms.push_back(i * (Lc / nb));
      std::sort(ms.begin(), ms.end());
      ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
      for (size_t s = 0; s + 1 < ms.size(); ++s) {
        double a = (double)ms[s] / (double)Lc, b = (double)ms[s + 1] / (double)Lc;
        for (int g = 0; g < q; ++g) {
          pts[j].push_back(a + (b - a) * gq.x[g]);
          wts[j].push_back((b - a) * gq.w[g]);
        }
      }
    }
    std::vector<double> kn[2][3];
    for (int g = 0; g < d; ++g) {
      kn[0][g] = open_knots(pk.nel[g], ps[0]);
      kn[1][g] = open_knots(pl.nel[g], ps[1]);
    }
    size_t n0 = pts[0].size(), n1 = d == 3 ? pts[1].size() : 1;
    const int nside = 2;  // normal layers carrying value or derivative
    // active functions of a side: two normal layers x (p_side+1)^(d-1)
    // tangential ones; side 0's entries first, then side 1's
    int nacts[2];
    for (int side = 0; side < 2; ++side) {
      int ntan = 1;
      for (int j = 0; j < d - 1; ++j) ntan *= (ps[side] + 1);
      nacts[side] = nside * ntan;
    }
    const int aoff[2] = {0, nacts[0]};
    // the q (q^2 in 3D) points of a merged segment lie in one element of each
    // side: their contributions are summed in a dense local block that is
    // added to the sparse accumulator once per segment
    const int na2 = nacts[0] + nacts[1];
    std::vector<long long> idx(na2);
    std::vector<double> val(na2), dn(na2);
    std::vector<double> Mloc((size_t)na2 * na2);
    const size_t qs1 = d == 3 ? (size_t)q : 1;
    for (size_t s1 = 0; s1 < n1; s1 += qs1)
      for (size_t s0 = 0; s0 < n0; s0 += q) {
      std::fill(Mloc.begin(), Mloc.end(), 0.0);
      for (size_t i1 = s1; i1 < s1 + qs1; ++i1)
      for (size_t i0 = s0; i0 < s0 + q; ++i0) {
        double tpar[2] = {pts[0][i0], d == 3 ? pts[1][i1] : 0.0};
        double wt = wts[0][i0] * (d == 3 ? wts[1][i1] : 1.0);
        // physical normal and surface element from side k
        double J[3][3] = {}, Ji[3][3] = {}, nrm[3] = {0, 0, 0}, ds = 0.0;
        double xk[3] = {0, 0, 0}, xl[3] = {0, 0, 0};
        xk[f.dk] = f.sk;
        xl[f.dl] = f.sl;
        for (int j = 0; j < d - 1; ++j) {
          xk[tk[j]] = tpar[j];
          xl[tl[j]] = tpar[j];
        }
        double Jl[3][3] = {}, Jli[3][3] = {};
        if (d == 2) {
          double J2[2][2], Ji2[2][2], Jl2[2][2], Jli2[2][2];
          multilinear_jac<2>(pk.corners, xk, J2);
          inverse<2>(J2, Ji2);
          multilinear_jac<2>(pl.corners, xl, Jl2);
          inverse<2>(Jl2, Jli2);
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              J[a][b] = J2[a][b];
              Ji[a][b] = Ji2[a][b];
              Jl[a][b] = Jl2[a][b];
              Jli[a][b] = Jli2[a][b];
            }
          ds = std::hypot(J[0][tk[0]], J[1][tk[0]]);
        } else {
          double J3[3][3], Ji3[3][3], Jl3[3][3], Jli3[3][3];
          multilinear_jac<3>(pk.corners, xk, J3);
          inverse<3>(J3, Ji3);
          multilinear_jac<3>(pl.corners, xl, Jl3);
          inverse<3>(Jl3, Jli3);
          std::memcpy(J, J3, sizeof(J3));
          std::memcpy(Ji, Ji3, sizeof(Ji3));
          std::memcpy(Jl, Jl3, sizeof(Jl3));
          std::memcpy(Jli, Jli3, sizeof(Jli3));
          double a[3], b[3];
          for (int r = 0; r < 3; ++r) {
            a[r] = J[r][tk[0]];
            b[r] = J[r][tk[1]];
          }
          double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2],
                 cz = a[0] * b[1] - a[1] * b[0];
          ds = std::sqrt(cx * cx + cy * cy + cz * cz);
        }
        // outer normal of Omega_k: J^-T e_dk (sign of the side), normalized
        double sgn = f.sk ? 1.0 : -1.0, nn = 0.0;
        for (int a = 0; a < d; ++a) {
          nrm[a] = sgn * Ji[f.dk][a];
          nn += nrm[a] * nrm[a];
        }
        nn = std::sqrt(nn);
        for (int a = 0; a < d; ++a) nrm[a] /= nn;
        double w = wt * ds;
        // evaluate both sides
        for (int side = 0; side < 2; ++side) {
          const PatchDev &pt = side ? pl : pk;
          const int dir = side ? f.dl : f.dk, s = side ? f.sl : f.sk;
          const int *tg = side ? tl : tk;
          const double(*Jinv)[3] = side ? Jli : Ji;
          double cvec[3] = {0, 0, 0};  // J^-1 n
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) cvec[a] += Jinv[a][b] * nrm[b];
          const int p = ps[side], nact = nacts[side];
          double bv[3][MAXP + 1], bd[3][MAXP + 1];
          int first[3];
          for (int g = 0; g < d; ++g) {
            double x;
            int e;
            if (g == dir) {
              x = (double)s;
              e = s ? pt.nel[g] - 1 : 0;
            } else {
              int j = (g == tg[0]) ? 0 : 1;
              x = tpar[j];
              e = std::min(pt.nel[g] - 1, (int)std::floor(x * pt.nel[g]));
            }
            double out[2][MAXP + 1];
            bspline_span_ders(kn[side][g], p, p + e, x, 1, out);
            for (int a = 0; a <= p; ++a) {
              bv[g][a] = out[0][a];
              bd[g][a] = out[1][a];
            }
            first[g] = e;
          }
          // active functions: two normal layers next to the side x tangential (p+1)^(d-1)
          for (int a = 0; a < nact; ++a) {
            int lay = a % nside, rest = a / nside;
            int li[3];
            li[dir] = s ? p - lay : lay;  // local index inside the element
            for (int j = 0; j < d - 1; ++j) {
              li[tg[j]] = rest % (p + 1);
              rest /= (p + 1);
            }
            double value = 1.0, grad[3];
            for (int g = 0; g < d; ++g) value *= bv[g][li[g]];
            for (int g = 0; g < d; ++g) {
              grad[g] = bd[g][li[g]];
              for (int h = 0; h < d; ++h)
                if (h != g) grad[g] *= bv[h][li[h]];
            }
            double dnv = 0.0;
            for (int g = 0; g < d; ++g) dnv += grad[g] * cvec[g];
            int gi[3] = {0, 0, 0};
            for (int g = 0; g < d; ++g) gi[g] = first[g] + li[g];
            idx[aoff[side] + a] = torn_index(pt, gi);
            val[aoff[side] + a] = side ? -value : value;  // jump [u] = u_k - u_l
            dn[aoff[side] + a] = dnv;
          }
        }
        const double eta = f.eta;
        for (int A = 0; A < na2; ++A) {
          if (val[A] == 0.0 && dn[A] == 0.0) continue;
          double *row = &Mloc[(size_t)A * na2];
          for (int B = 0; B < na2; ++B)
            row[B] += w * (eta * val[A] * val[B] - 0.5 * dn[A] * val[B] - 0.5 * val[A] * dn[B]);
        }
      }
      for (int A = 0; A < na2; ++A)
        for (int B = 0; B < na2; ++B) {
          const double v = Mloc[(size_t)A * na2 + B];
          if (v == 0.0) continue;
          unsigned long long key = ((unsigned long long)idx[A] << 32) | (unsigned long long)idx[B];
          acc[key] += v;
        }
      }
    per[fi].assign(acc.begin(), acc.end());
    std::sort(per[fi].begin(), per[fi].end());
  });
  std::vector<std::pair<unsigned long long, double>> all;
  for (auto &v : per) all.insert(all.end(), v.begin(), v.end());
  std::stable_sort(all.begin(), all.end(),
                   [](const std::pair<unsigned long long, double> &a,
                      const std::pair<unsigned long long, double> &b) { return a.first < b.first; });
  std::vector<std::pair<unsigned long long, double>> ent;
  ent.reserve(all.size());
  for (auto &e : all) {
    if (!ent.empty() && ent.back().first == e.first)
      ent.back().second += e.second;
    else
      ent.push_back(e);
  }
  // CSR over torn rows (Dirichlet rows / columns dropped)
  L.if_ptr.assign(L.Ntorn + 1, 0);
  L.if_col.clear();
  L.if_val.clear();
  L.if_cross.clear();
  std::vector<long long> offs(L.K);
  for (int k = 0; k < L.K; ++k) offs[k] = L.pd[k].off;
  auto patch_of = [&](long long t) {
    return (int)(std::upper_bound(offs.begin(), offs.end(), t) - offs.begin()) - 1;
  };
  for (auto &e : ent) {
    long long r = (long long)(e.first >> 32), cc = (long long)(e.first & 0xffffffffULL);
    if (!L.mask[r] || !L.mask[cc]) continue;
    L.if_ptr[r + 1]++;
    L.if_col.push_back((int)cc);
    L.if_val.push_back(e.second);
    L.if_cross.push_back(patch_of(r) != patch_of(cc));
  }
  for (long long t = 0; t < L.Ntorn; ++t) L.if_ptr[t + 1] += L.if_ptr[t];
}

// A(t1, t2) of the torn operator: volume entry (same patch) + interface entry
static double torn_entry_iface(const LevelData &L, long long t1, long long t2) {
  int b = L.if_ptr.empty() ? 0 : L.if_ptr[t1], e = L.if_ptr.empty() ? 0 : L.if_ptr[t1 + 1];
  auto it = std::lower_bound(L.if_col.begin() + b, L.if_col.begin() + e, (int)t2);
  if (it != L.if_col.begin() + e && *it == (int)t2) return L.if_val[it - L.if_col.begin()];
  return 0.0;
}

// Dense P^T A P over a set of compact unknowns (conforming: summed over copies).
static std::vector<double> dense_block(const Context &c, const LevelData &L,
                                       const std::vector<int> &comps) {
  const int d = c.d, p = c.p;
  const int n = (int)comps.size();
  std::unordered_map<long long, int> loc;  // torn copy -> local index
  for (int a = 0; a < n; ++a)
    for (int t : L.copies(comps[a])) loc[t] = a;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int t1 : L.copies(comps[a])) {
      const int k = L.patch_of(t1);
      const PatchDev &pt = L.pd[k];
      long long lc = t1 - pt.off;
      int i[3] = {(int)(lc % pt.n[0]), (int)((lc / pt.n[0]) % pt.n[1]),
                  (int)(lc / ((long long)pt.n[0] * pt.n[1]))};
      int lo[3], hi[3];
      for (int g = 0; g < 3; ++g) {
        lo[g] = g < d ? std::max(0, i[g] - p) : 0;
        hi[g] = g < d ? std::min(pt.n[g] - 1, i[g] + p) : 0;
      }
      for (int j2 = lo[2]; j2 <= hi[2]; ++j2)
        for (int j1 = lo[1]; j1 <= hi[1]; ++j1)
          for (int j0 = lo[0]; j0 <= hi[0]; ++j0) {
            int j[3] = {j0, j1, j2};
            long long t2 = torn_index(pt, j);
            auto it = loc.find(t2);
            if (it == loc.end()) continue;
            double v = d == 2 ? vol_entry<2>(pt, L.tabB.data(), L.tabD.data(), c.gr, p, i, j)
                              : vol_entry<3>(pt, L.tabB.data(), L.tabD.data(), c.gr, p, i, j);
            A[(size_t)a * n + it->second] += v;
          }
      if (!L.if_ptr.empty())
        for (int e = L.if_ptr[t1]; e < L.if_ptr[t1 + 1]; ++e) {
          auto it = loc.find(L.if_col[e]);
          if (it != loc.end()) A[(size_t)a * n + it->second] += L.if_val[e];
        }
    }
  return A;
}

// Rows of the assembled float64 stencil (device) of the representatives of
// compact unknowns, copied to the host ([n][SP]).
static std::vector<double> stencil_rows_host(Context &c, const LevelData &L, const double *st64,
                                             int SP, const std::vector<int> &comps) {
  std::vector<int> rows(comps.size());
  for (size_t a = 0; a < comps.size(); ++a) rows[a] = L.rep[comps[a]];
  std::vector<double> out(rows.size() * SP);
  if (rows.empty()) return out;
  int *d_rows = nullptr;
  double *d_out = nullptr;
  const bool lent = c.arena.region != nullptr;  // inside a lent region: no driver calls
  if (lent) {
    d_rows = c.arena.alloc<int>(rows.size());
    d_out = c.arena.alloc<double>(out.size());
  } else {
    HIPCHK(hipMalloc((void **)&d_rows, rows.size() * sizeof(int)));
    HIPCHK(hipMalloc((void **)&d_out, out.size() * sizeof(double)));
  }
  HIPCHK(hipMemcpyAsync(d_rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice,
                        c.stream));
  k_gather_rows(st64, SP, d_rows, (int)rows.size(), d_out, c.stream);
  HIPCHK(hipMemcpyAsync(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  if (!lent) {
    (void)hipFree(d_rows);
    (void)hipFree(d_out);
  }
  return out;
}

// Rows of the assembled float64 stencil (device) at the given torn indices,
// copied to the host ([n][SP]).
static std::vector<double> torn_rows_host(Context &c, const double *st64, int SP,
                                          const std::vector<int> &rows) {
  std::vector<double> out(rows.size() * SP);
  if (rows.empty()) return out;
  int *d_rows = nullptr;
  double *d_out = nullptr;
  const bool lent = c.arena.region != nullptr;  // inside a lent region: no driver calls
  if (lent) {
    d_rows = c.arena.alloc<int>(rows.size());
    d_out = c.arena.alloc<double>(out.size());
  } else {
    HIPCHK(hipMalloc((void **)&d_rows, rows.size() * sizeof(int)));
    HIPCHK(hipMalloc((void **)&d_out, out.size() * sizeof(double)));
  }
  HIPCHK(hipMemcpyAsync(d_rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice,
                        c.stream));
  k_gather_rows(st64, SP, d_rows, (int)rows.size(), d_out, c.stream);
  HIPCHK(hipMemcpyAsync(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  if (!lent) {
    (void)hipFree(d_rows);
    (void)hipFree(d_out);
  }
  return out;
}

// Gauss-Seidel rows of the conforming space (Section 4 on the glued space of
// eq. igaspace0).  The matrix row of a glued unknown is the sum of the
// patch-local rows of its copies.  Its first copy (the owner, in patch k)
// carries the whole row: an entry of another copy's row (patch m) whose
// column has a copy in k inside the owner's (2p+1)^d stencil is added to
// that stencil slot; every other entry becomes a cross-patch coupling of the
// owner row, read at the column's copy in m.  The additions go to the device
// rows (unique (row, slot) pairs, summed on the host in a fixed order); the
// couplings are left in L.cf_* for the tile lists.  The couplings' columns
// belong to patches of other colours (the vertex-sharing colouring), so they
// are constant while the owner's colour is swept; a column of the owner's
// colour outside its stencil would break that and is rejected.
static void fold_conforming_rows(Context &c, LevelData &L, double *st64, int SP) {
  const int d = c.d, p = c.p, S1 = 2 * p + 1;
  int S = 1;
  for (int g = 0; g < d; ++g) S *= S1;
  std::vector<int> others;  // non-owner copies of glued unknowns, by compact index
  for (long long ci = 0; ci < L.N; ++ci)
    for (int t : L.copies(ci))
      if (t != L.rep[ci]) others.push_back(t);
  std::vector<double> rows = torn_rows_host(c, st64, SP, others);
  auto local = [&](long long t, int k, int *i) {
    long long a = t - L.pd[k].off;
    for (int g = 0; g < 3; ++g) {
      i[g] = g < d ? (int)(a % L.pd[k].n[g]) : 0;
      if (g < d) a /= L.pd[k].n[g];
    }
  };
  std::map<std::pair<int, int>, double> fold;              // (owner row, slot) -> sum
  std::map<int, std::vector<std::pair<int, double>>> cross;  // owner row -> (column, value)
  for (size_t q = 0; q < others.size(); ++q) {
    const int tm = others[q];
    const int ci = L.comp[tm];
    const int to = L.rep[ci];
    const int k = L.patch_of(to), m = L.patch_of(tm);
    int a[3], b[3];
    local(to, k, a);
    local(tm, m, b);
    const PatchDev &pm = L.pd[m];
    for (int sl = 0; sl < S; ++sl) {
      const double v = rows[q * SP + sl];
      if (v == 0.0) continue;
      int j[3] = {0, 0, 0};
      bool inside = true;
      for (int g = 0, r = sl; g < d; ++g, r /= S1) {
        j[g] = b[g] + r % S1 - p;
        inside &= j[g] >= 0 && j[g] < pm.n[g];
      }
      if (!inside) continue;
      const long long tj = pm.off + j[0] + (long long)j[1] * pm.stride[1] +
                           (long long)j[2] * pm.stride[2];
      const int cj = L.comp[tj];
      if (cj < 0) continue;  // Dirichlet column
      int slot = -1;
      for (int tk : L.copies(cj)) {
        if (L.patch_of(tk) != k) continue;
        int e[3];
        local(tk, k, e);
        int sk = 0;
        bool in = true;
        for (int g = 0, mul = 1; g < d; ++g, mul *= S1) {
          in &= std::abs(e[g] - a[g]) <= p;
          sk += (e[g] - a[g] + p) * mul;
        }
        if (in) slot = sk;
      }
      if (slot >= 0) {
        fold[{to, slot}] += v;
      } else {
        if (c.color[L.patch_of(L.rep[cj])] == c.color[k])
          fail(IGAMG_EUNSUPPORTED, "conforming coupling between unknowns of one patch colour "
                                   "outside the stencil");
        cross[to].push_back({(int)tj, v});
      }
    }
  }
  std::vector<int> frow, fslot;
  std::vector<double> fval;
  for (auto &kv : fold) {
    frow.push_back(kv.first.first);
    fslot.push_back(kv.first.second);
    fval.push_back(kv.second);
  }
  if (!frow.empty()) {
    int *dr = c.arena.upload(frow, c.stream), *ds = c.arena.upload(fslot, c.stream);
    double *dv = c.arena.upload(fval, c.stream);
    k_stencil_add(dr, ds, dv, (int)frow.size(), st64, SP, c.stream);
  }
  L.cf_ptr.assign(L.Ntorn + 1, 0);
  L.cf_col.clear();
  L.cf_val.clear();
  for (long long t = 0; t < L.Ntorn; ++t) {
    auto it = cross.find((int)t);
    if (it != cross.end())
      for (auto &cv : it->second) {
        L.cf_col.push_back(cv.first);
        L.cf_val.push_back(cv.second);
      }
    L.cf_ptr[t + 1] = (int)L.cf_col.size();
  }
}

// Dense P^T A P over compact unknowns of the SIPG space (one torn copy each)
// from the assembled stencil rows (volume + same-patch interface terms) and
// the cross-patch interface terms.
static std::vector<double> dense_block_rows(const Context &c, const LevelData &L,
                                            const std::vector<int> &comps, const double *rows,
                                            int SP) {
  const int n = (int)comps.size();
  std::unordered_map<long long, int> loc;
  loc.reserve(2 * n);
  for (int a = 0; a < n; ++a) loc[L.rep[comps[a]]] = a;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    const long long t1 = L.rep[comps[a]];
    const int k = L.patch_of(t1);
    const PatchDev &pt = L.pd[k];
    const int p = c.p, S1 = 2 * p + 1;  // rows in the layout of the largest degree
    long long lc = t1 - pt.off;
    int i[3] = {0, 0, 0};
    for (int g = 0; g < c.d; ++g) {
      i[g] = (int)(lc % pt.n[g]);
      lc /= pt.n[g];
    }
    int S = 1;
    for (int g = 0; g < c.d; ++g) S *= S1;
    for (int o = 0; o < S; ++o) {
      int j[3] = {0, 0, 0}, oo = o;
      bool in = true;
      for (int g = 0; g < c.d; ++g) {
        j[g] = i[g] + oo % S1 - p;
        oo /= S1;
        in = in && j[g] >= 0 && j[g] < pt.n[g];
      }
      if (!in) continue;
      auto it = loc.find(torn_index(pt, j));
      if (it != loc.end()) A[(size_t)a * n + it->second] += rows[(size_t)a * SP + o];
    }
    if (!L.if_ptr.empty())
      for (int e = L.if_ptr[t1]; e < L.if_ptr[t1 + 1]; ++e) {
        if (!L.if_cross[e]) continue;
        auto it = loc.find(L.if_col[e]);
        if (it != loc.end()) A[(size_t)a * n + it->second] += L.if_val[e];
      }
  }
  return A;
}

// ---------------------------------------------------------------------------
// smoother data
// ---------------------------------------------------------------------------
static std::vector<double> dense_block_rows(const Context &c, const LevelData &L,
                                            const std::vector<int> &comps, const double *rows,
                                            int SP);
static std::vector<double> stencil_rows_host(Context &c, const LevelData &L, const double *st64,
                                             int SP, const std::vector<int> &comps);

// st64: the level's assembled float64 stencil rows on the device (SIPG), or
// null (conforming: entries by quadrature on the host)
static void build_pieces(Context &c, LevelData &L, const double *st64, int SP) {
  const int d = c.d;
  std::map<std::vector<int>, int> key2piece;
  std::vector<std::vector<int>> members;
  for (long long ci = 0; ci < L.N; ++ci) {
    long long t = L.rep[ci];
    const int k = L.patch_of(t);
    const PatchDev &pt = L.pd[k];
    long long lc = t - pt.off;
    int i[3] = {(int)(lc % pt.n[0]), (int)((lc / pt.n[0]) % pt.n[1]),
                (int)(lc / ((long long)pt.n[0] * pt.n[1]))};
    int fixed[3] = {-1, -1, -1};
    bool interior = true;
    for (int g = 0; g < d; ++g) {
      if (i[g] == 0) fixed[g] = 0;
      if (i[g] == pt.n[g] - 1) fixed[g] = 1;
      if (fixed[g] >= 0) interior = false;
    }
    if (interior) continue;
    std::vector<int> key;
    for (int b = 0; b < (1 << d); ++b) {
      bool ok = true;
      for (int g = 0; g < d; ++g)
        if (fixed[g] >= 0 && ((b >> g) & 1) != fixed[g]) ok = false;
      if (ok) key.push_back(c.vid[k][b]);
    }
    std::sort(key.begin(), key.end());
    auto it = key2piece.find(key);
    if (it == key2piece.end()) {
      it = key2piece.emplace(key, (int)members.size()).first;
      members.push_back({});
    }
    members[it->second].push_back((int)ci);
  }
  std::vector<PieceDev> pcs;
  std::vector<int> idx, cp, cidx;
  std::vector<double> blocks;  // P_T^T A P_T of every piece, inverted on the GPU
  L.max_piece = 0;
  // the stencil rows of all piece unknowns in one gather (one device round trip)
  std::vector<double> rows;
  if (st64) {
    std::vector<int> all;
    for (auto &m : members) all.insert(all.end(), m.begin(), m.end());
    rows = stencil_rows_host(c, L, st64, SP, all);
  }
  // dense blocks of the pieces (pieces in parallel, kept in piece order)
  std::vector<size_t> row0(members.size() + 1, 0);
  for (size_t i = 0; i < members.size(); ++i) row0[i + 1] = row0[i] + members[i].size();
  std::vector<std::vector<double>> dense(members.size());
  parallel_for((int)members.size(), [&](int i) {
    dense[i] = st64 ? dense_block_rows(c, L, members[i], rows.data() + row0[i] * SP, SP)
                    : dense_block(c, L, members[i]);
  });
  for (size_t i = 0; i < members.size(); ++i) {
    const std::vector<int> &m = members[i];
    PieceDev pc{};
    pc.n = (int)m.size();
    pc.inv_off = (long long)blocks.size();
    pc.idx_off = (int)idx.size();
    pc.cp_off = (int)cp.size();
    for (int ci : m) {
      idx.push_back(L.rep[ci]);
      cp.push_back((int)cidx.size());
      for (int t : L.copies(ci)) cidx.push_back(t);
    }
    cp.push_back((int)cidx.size());
    std::vector<double> A = std::move(dense[i]);
    blocks.insert(blocks.end(), A.begin(), A.end());
    pcs.push_back(pc);
    L.max_piece = std::max(L.max_piece, pc.n);
    L.piece_sq += (double)pc.n * pc.n;
    L.piece_n += pc.n;
  }
  L.n_pieces = (int)pcs.size();
  // the piece kernel holds a piece's residual in LDS next to 16 x 64 partial
  // sums (float64 here: the float32 cycle needs half of it)
  if ((size_t)L.max_piece * sizeof(double) + 16 * 64 * sizeof(double) > 160 * 1024)
    fail(IGAMG_EUNSUPPORTED, "interface piece too large for the piece kernel's LDS");
  L.d_pieces = c.arena.upload(pcs, c.stream);
  L.d_piece_idx = c.arena.upload(idx, c.stream);
  L.d_piece_cp = c.arena.upload(cp, c.stream);
  L.d_piece_cidx = c.arena.upload(cidx, c.stream);
  // float64 inverses in place; float32 mode rounds them into their own array
  double *inv64 = c.arena.upload(blocks, c.stream);
  {
    std::vector<long long> offs;
    std::vector<int> ns;
    for (const PieceDev &pc : pcs) {
      offs.push_back(pc.inv_off);
      ns.push_back(pc.n);
    }
    long long *d_offs = c.arena.upload(offs, c.stream);
    int *d_ns = c.arena.upload(ns, c.stream);
    k_spd_inverse_batch(inv64, d_offs, d_ns, (int)pcs.size(), L.max_piece, c.d_bad, c.stream);
  }
  if (c.fp32()) {
    L.a32.piece_inv = c.arena.alloc<float>(blocks.size());
    k_convert<double, float>(inv64, nullptr, L.a32.piece_inv, (long long)blocks.size(), 1, c.stream);
  } else {
    L.a64.piece_inv = inv64;
  }
}

static std::vector<double> transpose(const std::vector<double> &A, int n) {
  std::vector<double> T((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[(size_t)j * n + i] = A[(size_t)i * n + j];
  return T;
}

// Patch interiors of the subspace corrected mass smoother (Section 5): with
// the 1D factors Q (Q^T M Q = I) and lam, L_T^-1 r = gamma^-1 (Qy x Qx)
// diag(1/(sigma + lam_y + lam_x)) (Qy x Qx)^T r, evaluated as
//   W = (Qy^T R Qx) ./ D   and   U += (tau/gamma) Qy W Qx^T
// on the interior block R of the patch tensor.
// Patch interiors of a 3D level as six batched product stages on the
// interior tensor R[z][y][x] (strides 1, nx, nx ny inside the patch tensor),
// intermediates alternating between two scratch tensors W1, W2:
//   1. W1_z = R_z Qx               (per z slice: Qx^T along x)
//   2. W2_z = Qy^T W1_z            (per z slice: Qy^T along y)
//   3. W1 = (Qz^T W2) ./ (sigma + lam_z[z] + lam_y[y] + lam_x[x])
//                                  (W2 as an mz x (my mx) matrix)
//   4. W2 = Qz W1
//   5. W1_z = Qy W2_z
//   6. U_z += scale W1_z Qx^T      (into the patch interior of u)
template <typename T>
static void build_scms3(Context &c, LevelData &L) {
  LevelArrays<T> &A = L.arr<T>();
  struct QT {
    T *Q, *QT;
    std::vector<double> lam;
  };
  // factors by (elements, degree) of a direction
  std::map<std::pair<int, int>, QT> qtab;
  for (int k = 0; k < L.K; ++k)
    for (int g = 0; g < 3; ++g) {
      const int ne = L.pd[k].nel[g], p = L.pd[k].p;
      if (qtab.count({ne, p})) continue;
      std::vector<double> Q, lam;
      scms_factors_1d(ne, p, Q, lam);
      int n = ne + p - 2;
      qtab[{ne, p}] = QT{c.arena.upload_as<T>(Q, c.stream),
                         c.arena.upload_as<T>(transpose(Q, n), c.stream), lam};
    }
  size_t scr = 0, nxy = 0;
  for (int k = 0; k < L.K; ++k) {
    const PatchDev &pt = L.pd[k];
    scr += (size_t)(pt.n[0] - 2) * (pt.n[1] - 2) * (pt.n[2] - 2);
    nxy += (size_t)(pt.n[0] - 2) * (pt.n[1] - 2);
  }
  L.wscratch_n = (long long)scr;
  A.wscratch = c.arena.alloc<T>(scr * c.nb);
  A.wscratch2 = c.arena.alloc<T>(scr * c.nb);
  // lam_y[j] + lam_x[i] of every patch, and lam_z per direction table
  std::vector<double> lxy;
  lxy.reserve(nxy);
  std::map<std::pair<int, int>, T *> lamz;
  for (auto &kv : qtab) lamz[kv.first] = c.arena.upload_as<T>(kv.second.lam, c.stream);
  std::vector<FdGemm<T>> g[6];
  const long long nt = L.Ntorn, ns = (long long)scr;
  size_t so = 0, lo = 0;
  std::vector<size_t> lxy_off;
  for (int k = 0; k < L.K; ++k) {
    const PatchDev &pt = L.pd[k];
    const int mx = pt.n[0] - 2, my = pt.n[1] - 2;
    const QT &qx = qtab[{pt.nel[0], pt.p}], &qy = qtab[{pt.nel[1], pt.p}];
    lxy_off.push_back(lo);
    for (int j = 0; j < my; ++j)
      for (int i = 0; i < mx; ++i) lxy.push_back(qy.lam[j] + qx.lam[i]);
    lo += (size_t)mx * my;
  }
  A.lam_xy = c.arena.upload_as<T>(lxy, c.stream);
  for (int k = 0; k < L.K; ++k) {
    PatchDev &pt = L.pd[k];
    const int nx = pt.n[0], ny = pt.n[1];
    const int mx = pt.n[0] - 2, my = pt.n[1] - 2, mz = pt.n[2] - 2;
    const long long sxy = (long long)mx * my, nxy_p = (long long)nx * ny;
    const QT &qx = qtab[{pt.nel[0], pt.p}], &qy = qtab[{pt.nel[1], pt.p}], &qz = qtab[{pt.nel[2], pt.p}];
    T *W1 = A.wscratch + so, *W2 = A.wscratch2 + so;
    so += (size_t)sxy * mz;
    T *rin = A.r + pt.off + nxy_p + nx + 1;
    T *uin = A.u + pt.off + nxy_p + nx + 1;
    double h = 1.0 / std::max(pt.nel[0], std::max(pt.nel[1], pt.nel[2]));
    pt.sigma = 1.0 / (c.opt.scaling_delta * h * h);
    double gamma = std::pow(c.measure[k], (c.d - 2.0) / c.d);
    pt.scms_scale = c.opt.damping_tau / gamma;
    const int tx = (mx + 63) / 64, txy = (int)((sxy + 63) / 64);
    for (int z = 0; z < mz; ++z) {
      const long long zr = z * nxy_p, zs = z * sxy;
      g[0].push_back(FdGemm<T>{rin + zr, qx.Q, W1 + zs, nx, mx, mx, nt, 0, ns, my, mx, mx, tx,
                               nullptr, nullptr, (T)0, (T)0, 0});
      g[1].push_back(FdGemm<T>{qy.QT, W1 + zs, W2 + zs, my, mx, mx, 0, ns, ns, my, mx, my, tx,
                               nullptr, nullptr, (T)0, (T)0, 0});
      g[4].push_back(FdGemm<T>{qy.Q, W2 + zs, W1 + zs, my, mx, mx, 0, ns, ns, my, mx, my, tx,
                               nullptr, nullptr, (T)0, (T)0, 0});
      g[5].push_back(FdGemm<T>{W1 + zs, qx.QT, uin + zr, mx, mx, nx, ns, 0, nt, my, mx, mx, tx,
                               nullptr, nullptr, (T)0, (T)pt.scms_scale, 2});
    }
    g[2].push_back(FdGemm<T>{qz.QT, W2, W1, mz, sxy, sxy, 0, ns, ns, mz, (int)sxy, mz, txy,
                             lamz[{pt.nel[2], pt.p}], A.lam_xy + lxy_off[k], (T)pt.sigma, (T)0, 1});
    g[3].push_back(FdGemm<T>{qz.Q, W1, W2, mz, sxy, sxy, 0, ns, ns, mz, (int)sxy, mz, txy,
                             nullptr, nullptr, (T)0, (T)0, 0});
  }
  for (int st = 0; st < 6; ++st) {
    L.fg_n[st] = (int)g[st].size();
    L.fg_t[st] = 0;
    for (const FdGemm<T> &it : g[st])
      L.fg_t[st] = std::max(L.fg_t[st], it.tn * ((it.M + 63) / 64));
    A.fg[st] = c.arena.upload(g[st], c.stream);
  }
  L.n_fd = L.fg_n[2];
  L.fd_work = 0;
  for (int k = 0; k < L.K; ++k)
    L.fd_work += (long long)(L.pd[k].n[0] - 2) * (L.pd[k].n[1] - 2) * (L.pd[k].n[2] - 2);
}

template <typename T>
static void build_scms(Context &c, LevelData &L) {
  if (c.d == 3) {
    build_scms3<T>(c, L);
    return;
  }
  LevelArrays<T> &A = L.arr<T>();
  struct QT {
    T *Q, *QT, *lam;
  };
  // 1D factors per (element count, degree)
  std::map<std::pair<int, int>, QT> qtab;
  for (int k = 0; k < L.K; ++k)
    for (int g = 0; g < c.d; ++g) {
      const int ne = L.pd[k].nel[g], p = L.pd[k].p;
      if (qtab.count({ne, p})) continue;
      std::vector<double> Q, lam;
      scms_factors_1d(ne, p, Q, lam);
      int n = ne + p - 2;
      qtab[{ne, p}] = QT{c.arena.upload_as<T>(Q, c.stream),
                         c.arena.upload_as<T>(transpose(Q, n), c.stream),
                         c.arena.upload_as<T>(lam, c.stream)};
    }
  size_t scr = 0;
  for (int k = 0; k < L.K; ++k) scr += (size_t)(L.pd[k].n[0] - 2) * (L.pd[k].n[1] - 2);
  L.wscratch_n = (long long)scr;
  A.wscratch = c.arena.alloc<T>(scr * c.nb);
  A.wscratch2 = c.arena.alloc<T>(scr * c.nb);
  std::vector<Fd2Item<T>> fa, fb;
  std::vector<FdGemm<T>> g1, g2, g3, g4;
  std::vector<FdWide<T>> w1, w2, w3, w4;
  L.fg_tiles = 0;
  L.fw_wide = L.fw_cat = 0;
  L.fd_work = 0;
  size_t so = 0;
  L.fd_rows = L.fd_K1 = L.fd_N = 0;
  const long long nt = L.Ntorn, ns = (long long)scr;
  for (int k = 0; k < L.K; ++k) {
    PatchDev &pt = L.pd[k];
    const int nx = pt.n[0], mx = pt.n[0] - 2, my = pt.n[1] - 2;
    const QT &qx = qtab[{pt.nel[0], pt.p}], &qy = qtab[{pt.nel[1], pt.p}];
    T *Wk = A.wscratch + so;
    so += (size_t)mx * my;
    T *rin = A.r + pt.off + nx + 1;
    T *uin = A.u + pt.off + nx + 1;
    double h = 1.0 / std::max(pt.nel[0], pt.nel[1]);
    pt.sigma = 1.0 / (c.opt.scaling_delta * h * h);
    double gamma = std::pow(c.measure[k], (c.d - 2.0) / c.d);
    pt.scms_scale = c.opt.damping_tau / gamma;
    // forward: W = (Qy^T R) Qx ./ (sigma + lam_y + lam_x)
    fa.push_back(Fd2Item<T>{qy.QT, rin, qx.Q, Wk, my, nx, mx, mx, nt, ns, my, my, mx, qy.lam,
                            qx.lam, (T)pt.sigma, (T)0});
    // backward: U += scale (Qy W) Qx^T
    fb.push_back(Fd2Item<T>{qy.Q, Wk, qx.QT, uin, my, mx, mx, nx, ns, nt, my, my, mx, nullptr,
                            nullptr, (T)0, (T)pt.scms_scale});
    // the same as four stages: Z = Qy^T R; W = Z Qx ./ D; Z = Qy W; U += scale Z Qx^T
    T *Zk = Wk, *W2 = A.wscratch2 + (so - (size_t)mx * my);
    const int tn = (mx + 63) / 64;
    g1.push_back(FdGemm<T>{qy.QT, rin, Zk, my, nx, mx, 0, nt, ns, my, mx, my, tn, nullptr, nullptr,
                           (T)0, (T)0, 0});
    g2.push_back(FdGemm<T>{Zk, qx.Q, W2, mx, mx, mx, ns, 0, ns, my, mx, mx, tn, qy.lam, qx.lam,
                           (T)pt.sigma, (T)0, 1});
    g3.push_back(FdGemm<T>{qy.Q, W2, Zk, my, mx, mx, 0, ns, ns, my, mx, my, tn, nullptr, nullptr,
                           (T)0, (T)0, 0});
    g4.push_back(FdGemm<T>{Zk, qx.QT, uin, mx, mx, nx, ns, 0, nt, my, mx, mx, tn, nullptr, nullptr,
                           (T)0, (T)pt.scms_scale, 2});
    // the same four stages over the whole batch (right-hand sides
    // concatenated along n for the left products, along the rows for the
    // right ones)
    w1.push_back(FdWide<T>{qy.QT, rin, Zk, my, nx, nt, mx, ns, my, mx, my, nullptr, nullptr,
                           (T)0, (T)0, 0});
    w2.push_back(FdWide<T>{qx.QT, Zk, W2, mx, mx, ns, mx, ns, mx, my, mx, qy.lam, qx.lam,
                           (T)pt.sigma, (T)0, 1});
    w3.push_back(FdWide<T>{qy.Q, W2, Zk, my, mx, ns, mx, ns, my, mx, my, nullptr, nullptr, (T)0,
                           (T)0, 0});
    w4.push_back(FdWide<T>{qx.Q, Zk, uin, mx, mx, ns, nx, nt, mx, my, mx, nullptr, nullptr, (T)0,
                           (T)pt.scms_scale, 2});
    L.fw_wide = std::max(L.fw_wide, std::max(mx, my));
    L.fw_cat = std::max(L.fw_cat, std::max(mx, my));
    L.fg_tiles = std::max(L.fg_tiles, tn * ((my + 63) / 64));
    L.fd_work += (long long)my * mx * ((my + 15) / 16);
    L.fd_rows = std::max(L.fd_rows, my);
    L.fd_K1 = std::max(L.fd_K1, my);
    L.fd_N = std::max(L.fd_N, mx);
  }
  if (L.fd_N > 320 || L.fd_K1 > 320) fail(IGAMG_EUNSUPPORTED, "patch too large for the SCMS kernel");
  L.n_fd = L.K;
  A.fd[0] = c.arena.upload(fa, c.stream);
  A.fd[1] = c.arena.upload(fb, c.stream);
  A.fg[0] = c.arena.upload(g1, c.stream);
  A.fg[1] = c.arena.upload(g2, c.stream);
  A.fg[2] = c.arena.upload(g3, c.stream);
  A.fg[3] = c.arena.upload(g4, c.stream);
  A.fw[0] = c.arena.upload(w1, c.stream);
  A.fw[1] = c.arena.upload(w2, c.stream);
  A.fw[2] = c.arena.upload(w3, c.stream);
  A.fw[3] = c.arena.upload(w4, c.stream);
}

// keep64: the float64 couplings are uploaded too (float32 cycle whose finest
// level also serves the float64 outer apply from the stored rows)
// Tiles of T^3 unknowns in classes (patch colour, tile parity) in key order.
// The cross-patch couplings are kept as a CSR over the coupled rows, rows
// grouped by patch colour: a face of a 3D tile couples to thousands of
// unknowns of the neighbouring patch, which one thread per row gathers in
// parallel (and in a fixed order) far faster than a per-tile list.
// Cross-patch couplings of torn row t (SIPG: the interface terms to other
// patches; conforming: the couplings left by fold_conforming_rows)
template <class F>
static void for_cross_of(const LevelData &L, long long t, F fn) {
  if (!L.cf_ptr.empty()) {
    for (int e = L.cf_ptr[t]; e < L.cf_ptr[t + 1]; ++e) fn(L.cf_col[e], L.cf_val[e]);
    return;
  }
  if (L.if_ptr.empty()) return;
  for (int e = L.if_ptr[t]; e < L.if_ptr[t + 1]; ++e)
    if (L.if_cross[e]) fn(L.if_col[e], L.if_val[e]);
}

// Conforming: the other copies of the glued unknown whose owner is torn row t
template <class F>
static void for_mirror_of(const LevelData &L, long long t, F fn) {
  if (L.cf_ptr.empty()) return;
  const int ci = L.comp[t];
  if (ci < 0 || L.rep[ci] != t) return;
  for (int tc : L.copies(ci))
    if (tc != t) fn(tc);
}

static void build_gs3(Context &c, LevelData &L, bool keep64) {
  const int T = c.opt.gs_tile;
  {
    std::vector<int> rows, ptr{0}, col;
    std::vector<double> val;
    L.x_cptr.assign(1, 0);
    for (int colr = 0; colr < c.n_colors; ++colr) {
      for (int k = 0; k < L.K; ++k) {
        if (c.color[k] != colr) continue;
        const PatchDev &pt = L.pd[k];
        const long long n = (long long)pt.n[0] * pt.n[1] * pt.n[2];
        for (long long t = pt.off; t < pt.off + n; ++t) {
          bool any = false;
          for_cross_of(L, t, [&](int cc, double v) {
            col.push_back(cc);
            val.push_back(v);
            any = true;
          });
          if (any) {
            rows.push_back((int)t);
            ptr.push_back((int)col.size());
          }
        }
      }
      L.x_cptr.push_back((int)rows.size());
    }
    L.x_n = (int)rows.size();
    L.d_x_rows = c.arena.upload(rows, c.stream);
    L.d_x_ptr = c.arena.upload(ptr, c.stream);
    L.d_x_col = c.arena.upload(col, c.stream);
    const size_t nv = (size_t)L.Ntorn * c.nb;
    if (c.fp32()) {
      L.a32.x_val = c.arena.upload_as<float>(val, c.stream);
      L.a32.xsum = c.arena.alloc<float>(nv);
      k_fill<float>(L.a32.xsum, 0.0f, (long long)nv, c.stream);
    }
    if (!c.fp32() || keep64) L.a64.x_val = c.arena.upload_as<double>(val, c.stream);
    if (!c.fp32()) {
      L.a64.xsum = c.arena.alloc<double>(nv);
      k_fill<double>(L.a64.xsum, 0.0, (long long)nv, c.stream);
    }
  }
  std::vector<GsTile3> all;
  std::vector<int> mli, mdst;
  for (int colr = 0; colr < c.n_colors; ++colr)
    for (int par = 0; par < 8; ++par) {
      std::vector<GsTile3> tiles;
      for (int k = 0; k < L.K; ++k) {
        if (c.color[k] != colr) continue;
        const PatchDev &pt = L.pd[k];
        int nb[3];
        for (int g = 0; g < 3; ++g) nb[g] = (pt.n[g] + T - 1) / T;
        for (int b2 = 0; b2 < nb[2]; ++b2)
          for (int b1 = 0; b1 < nb[1]; ++b1)
            for (int b0 = 0; b0 < nb[0]; ++b0) {
              if (((b0 & 1) | ((b1 & 1) << 1) | ((b2 & 1) << 2)) != par) continue;
              GsTile3 tl{pt.off, {pt.n[0], pt.n[1], pt.n[2]}, {b0 * T, b1 * T, b2 * T},
                         (int)mli.size(), 0};
              // conforming: mirror copies of the tile's owned glued unknowns
              for (int iz = b2 * T; iz < std::min(pt.n[2], (b2 + 1) * T); ++iz)
                for (int iy = b1 * T; iy < std::min(pt.n[1], (b1 + 1) * T); ++iy)
                  for (int ix = b0 * T; ix < std::min(pt.n[0], (b0 + 1) * T); ++ix) {
                    const long long t = pt.off + ((long long)iz * pt.n[1] + iy) * pt.n[0] + ix;
                    for_mirror_of(L, t, [&](int dst) {
                      mli.push_back(((iz - b2 * T) * T + iy - b1 * T) * T + ix - b0 * T);
                      mdst.push_back(dst);
                    });
                  }
              tl.mr_n = (int)mli.size() - tl.mr_off;
              tiles.push_back(tl);
            }
      }
      GsClass cl;
      cl.count = (int)tiles.size();
      cl.tiles3 = c.arena.upload(tiles, c.stream);
      L.gs.push_back(cl);
      all.insert(all.end(), tiles.begin(), tiles.end());
    }
  L.n_atiles = (int)all.size();
  L.d_atiles3 = c.arena.upload(all, c.stream);
  L.d_mr_li = c.arena.upload(mli, c.stream);
  L.d_mr_dst = c.arena.upload(mdst, c.stream);
}

// Cross-patch couplings of one Gauss-Seidel tile (entries (row, column,
// value), rows ascending) in the slot layout of GsTile: a row's couplings are
// cut into slots of K entries in consecutive lanes of one pass, so that every
// lane sums its slot in order and the row's first lane adds its slots' sums
// in lane order.  K minimizes passes x (K + slots per row).
static void pack_cross(const std::vector<int> &rl, const std::vector<int> &rc,
                       const std::vector<double> &rv, GsTile &tl, std::vector<int> &slots,
                       std::vector<int> &col, std::vector<double> &val) {
  tl.cx_off = (int)col.size();
  tl.cx_sl = (int)slots.size();
  tl.cx_k = tl.cx_np = tl.cx_r = 0;
  if (rl.empty()) return;
  std::vector<std::array<int, 3>> rows;  // row, first entry, count
  for (size_t i = 0; i < rl.size();) {
    size_t j = i;
    while (j < rl.size() && rl[j] == rl[i]) ++j;
    if (!rows.empty() && rows.back()[0] >= rl[i]) fail(IGAMG_EUNSUPPORTED, "cross couplings out of row order");
    rows.push_back({rl[i], (int)i, (int)(j - i)});
    i = j;
  }
  int maxc = 0;
  for (const auto &r : rows) maxc = std::max(maxc, r[2]);
  auto plan = [&](int K, int &np, int &mr) {
    np = 0;
    mr = 0;
    int used = 64;
    for (const auto &r : rows) {
      const int ns = (r[2] + K - 1) / K;
      mr = std::max(mr, ns);
      if (used + ns > 64) {
        ++np;
        used = 0;
      }
      used += ns;
    }
  };
  int K = maxc;
  long long best = -1;
  for (int k = (maxc + 63) / 64; k <= maxc; ++k) {
    int np, mr;
    plan(k, np, mr);
    const long long cost = (long long)np * (k + mr);
    if (best < 0 || cost < best) {
      best = cost;
      K = k;
    }
  }
  int np, mr;
  plan(K, np, mr);
  tl.cx_k = K;
  tl.cx_np = np;
  tl.cx_r = mr;
  const size_t s0 = slots.size(), e0 = col.size();
  slots.resize(s0 + (size_t)np * 64, -1);
  col.resize(e0 + (size_t)np * K * 64, -1);
  val.resize(col.size(), 0.0);
  int q = -1, used = 64;
  for (const auto &r : rows) {
    const int ns = (r[2] + K - 1) / K;
    if (used + ns > 64) {
      ++q;
      used = 0;
    }
    for (int sl = 0; sl < ns; ++sl) {
      const int lane = used + sl;
      slots[s0 + (size_t)q * 64 + lane] = r[0] | (sl << 16) | (ns << 24);
      for (int k = 0; k < K && sl * K + k < r[2]; ++k) {
        const size_t at = e0 + ((size_t)q * K + k) * 64 + lane;
        col[at] = rc[r[1] + sl * K + k];
        val[at] = rv[r[1] + sl * K + k];
      }
    }
    used += ns;
  }
}

static void build_gs(Context &c, LevelData &L, bool keep64) {
  const int d = c.d, T = c.opt.gs_tile;
  if (T != 2 * (c.p + 1)) fail(IGAMG_EUNSUPPORTED, "Gauss-Seidel tiles of width 2(p+1) only");
  if (d == 3) {
    build_gs3(c, L, keep64);
    return;
  }
  auto for_cross = [&](long long t, auto fn) { for_cross_of(L, t, fn); };
  auto for_mirror = [&](long long t, auto fn) { for_mirror_of(L, t, fn); };
  std::vector<int> li, col, mli, mdst;
  std::vector<double> val;
  std::vector<GsTile> all;
  for (int colr = 0; colr < c.n_colors; ++colr)
    for (int par = 0; par < (1 << d); ++par) {
      std::vector<GsTile> tiles;
      for (int k = 0; k < L.K; ++k) {
        if (c.color[k] != colr) continue;
        const PatchDev &pt = L.pd[k];
        int nb[3] = {1, 1, 1};
        for (int g = 0; g < d; ++g) nb[g] = (pt.n[g] + T - 1) / T;
        for (int b1 = 0; b1 < nb[1]; ++b1)
          for (int b0 = 0; b0 < nb[0]; ++b0) {
            int pr = (b0 & 1) | ((b1 & 1) << 1);
            if (pr != par) continue;
            GsTile tl{};
            tl.off = pt.off;
            tl.nx = pt.n[0];
            tl.ny = pt.n[1];
            tl.i0[0] = b0 * T;
            tl.i0[1] = b1 * T;
            tl.mr_off = (int)mli.size();
            // cross-patch couplings of the tile rows; conforming: the mirror
            // copies of the owned glued unknowns
            std::vector<int> rl, rc;
            std::vector<double> rv;
            for (int iy = b1 * T; iy < std::min(pt.n[1], (b1 + 1) * T); ++iy)
              for (int ix = b0 * T; ix < std::min(pt.n[0], (b0 + 1) * T); ++ix) {
                const long long t = pt.off + (long long)iy * pt.n[0] + ix;
                const int lt = (iy - b1 * T) * T + (ix - b0 * T);
                for_cross(t, [&](int cc, double v) {
                  rl.push_back(lt);
                  rc.push_back(cc);
                  rv.push_back(v);
                });
                for_mirror(t, [&](int dst) {
                  mli.push_back(lt);
                  mdst.push_back(dst);
                });
              }
            pack_cross(rl, rc, rv, tl, li, col, val);
            tl.mr_n = (int)mli.size() - tl.mr_off;
            tiles.push_back(tl);
          }
      }
      GsClass cl;
      cl.count = (int)tiles.size();
      cl.tiles = c.arena.upload(tiles, c.stream);
      L.gs.push_back(cl);
      all.insert(all.end(), tiles.begin(), tiles.end());
    }
  L.n_atiles = (int)all.size();
  L.d_atiles = c.arena.upload(all, c.stream);
  L.d_gcx_li = c.arena.upload(li, c.stream);
  L.d_gcx_col = c.arena.upload(col, c.stream);
  L.d_mr_li = c.arena.upload(mli, c.stream);
  L.d_mr_dst = c.arena.upload(mdst, c.stream);
  if (c.fp32()) L.a32.gcx_val = c.arena.upload_as<float>(val, c.stream);
  // float32 batches: row blocks of the lane-per-right-hand-side operator and
  // the cross-patch couplings as a CSR over the coupled rows (torn order)
  const int bx = sp_rhs_bx(c.p);
  if (c.fp32() && bx > 0 && L.st_apply && c.nb >= SP_RHS_MIN) {
    // strips of bx rows on one line; four consecutive lines of one strip
    // column per block (their stencil-line windows overlap in the caches)
    std::vector<GsTile> sp;
    std::vector<long long> plines;
    long long ptot = 0;
    for (int k = 0; k < L.K; ++k) {
      const PatchDev &pt = L.pd[k];
      const int pw = pt.n[0] + 2 * c.p;
      for (int y = 0; y < pt.n[1]; ++y) {
        plines.push_back(pt.off + (long long)y * pt.n[0]);
        plines.push_back(ptot + (long long)(y + c.p) * pw + c.p);
        plines.push_back(pt.n[0]);
      }
      for (int y0 = 0; y0 < pt.n[1]; y0 += 4)
        for (int x = 0; x < pt.n[0]; x += bx)
          for (int y = y0; y < std::min(pt.n[1], y0 + 4); ++y) {
            GsTile g{};
            g.off = pt.off;
            g.nx = pt.n[0];
            g.ny = pt.n[1];
            g.i0[0] = x;
            g.i0[1] = y;
            g.pad_off = ptot;
            sp.push_back(g);
          }
      ptot += (long long)(pt.n[0] + 2 * c.p) * (pt.n[1] + 2 * c.p);
    }
    L.pad_tot = ptot;
    L.n_plines = (int)(plines.size() / 3);
    L.d_plines = c.arena.upload(plines, c.stream);
    // groups of 64 right-hand sides; slack of one strip past the end
    const size_t nut = (size_t)((c.nb + 63) / 64) * (size_t)(ptot + bx) * 64;
    L.ut = c.arena.alloc<float>(nut);
    k_fill<float>(L.ut, 0.0f, (long long)nut, c.stream);
    L.n_sptiles = (int)sp.size();
    L.d_sptiles = c.arena.upload(sp, c.stream);
    std::vector<int> xr, xp{0}, xc;
    std::vector<double> xv;
    for (long long t = 0; t < L.Ntorn; ++t) {
      bool any = false;
      for_cross_of(L, t, [&](int cc, double v) {
        xc.push_back(cc);
        xv.push_back(v);
        any = true;
      });
      if (any) {
        xr.push_back((int)t);
        xp.push_back((int)xc.size());
      }
    }
    L.x_n = (int)xr.size();
    L.d_x_rows = c.arena.upload(xr, c.stream);
    L.d_x_ptr = c.arena.upload(xp, c.stream);
    L.d_x_col = c.arena.upload(xc, c.stream);
    L.a32.x_val = c.arena.upload_as<float>(xv, c.stream);
  }
  if (!c.fp32() || keep64) L.a64.gcx_val = c.arena.upload_as<double>(val, c.stream);
}

static void build_transfer(Context &c, LevelData &F, const LevelData &C) {
  const int d = c.d;
  struct Tab {
    int prow, rrow;
  };
  // 1D embeddings per (coarse element count, degree)
  std::map<std::pair<int, int>, Tab> tabs;
  std::vector<std::vector<double>> Ps;
  std::vector<std::pair<int, int>> ncs;
  int PW = 1, RW = 1;
  for (int k = 0; k < F.K; ++k)
    for (int g = 0; g < d; ++g) {
      const int ncel = C.pd[k].nel[g], p = C.pd[k].p;
      if (F.pd[k].nel[g] != 2 * ncel) fail(IGAMG_EINVAL, "levels are not dyadic");
      if (tabs.count({ncel, p})) continue;
      tabs[{ncel, p}] = Tab{0, 0};
      Ps.push_back(embedding_1d(ncel, p));
      ncs.push_back({ncel, p});
    }
  // widths
  for (size_t t = 0; t < Ps.size(); ++t) {
    const int p = ncs[t].second;
    int nc = ncs[t].first + p, nf = 2 * ncs[t].first + p;
    const std::vector<double> &P = Ps[t];
    for (int i = 0; i < nf; ++i) {
      int a = -1, b = -1;
      for (int j = 0; j < nc; ++j)
        if (P[(size_t)i * nc + j] != 0.0) {
          if (a < 0) a = j;
          b = j;
        }
      if (a >= 0) PW = std::max(PW, b - a + 1);
    }
    for (int j = 0; j < nc; ++j) {
      int a = -1, b = -1;
      for (int i = 0; i < nf; ++i)
        if (P[(size_t)i * nc + j] != 0.0) {
          if (a < 0) a = i;
          b = i;
        }
      if (a >= 0) RW = std::max(RW, b - a + 1);
    }
  }
  std::vector<int> Plo, Rlo;
  std::vector<double> Pv, Rv;
  size_t t = 0;
  for (auto &kv : tabs) {
    const int ncel = kv.first.first, p = kv.first.second;
    size_t ti = std::find(ncs.begin(), ncs.end(), kv.first) - ncs.begin();
    const std::vector<double> &P = Ps[ti];
    int nc = ncel + p, nf = 2 * ncel + p;
    kv.second.prow = (int)Plo.size();
    kv.second.rrow = (int)Rlo.size();
    for (int i = 0; i < nf; ++i) {
      int a = 0;
      while (a < nc && P[(size_t)i * nc + a] == 0.0) ++a;
      if (a == nc) a = 0;
      Plo.push_back(a);
      for (int w = 0; w < PW; ++w) Pv.push_back(a + w < nc ? P[(size_t)i * nc + a + w] : 0.0);
    }
    for (int j = 0; j < nc; ++j) {
      int a = 0;
      while (a < nf && P[(size_t)a * nc + j] == 0.0) ++a;
      if (a == nf) a = 0;
      Rlo.push_back(a);
      for (int w = 0; w < RW; ++w) Rv.push_back(a + w < nf ? P[(size_t)(a + w) * nc + j] : 0.0);
    }
    ++t;
  }
  for (int k = 0; k < F.K; ++k)
    for (int g = 0; g < d; ++g) {
      const Tab &tb = tabs[{C.pd[k].nel[g], C.pd[k].p}];
      F.pd[k].xp[g] = tb.prow;
      F.pd[k].xr[g] = tb.rrow;
    }
  if (PW > 12 || RW > 12) fail(IGAMG_EUNSUPPORTED, "transfer band wider than the kernels hold");
  // output tiles of 16 rows x tx columns; the input window of every tile
  // must fit the kernel's LDS window of wxm x wym values (false otherwise)
  auto tiles_of = [&](const LevelData &Li, const LevelData &Lo, const std::vector<int> &lo, int W,
                      bool coarse_side, int tx, int wxm, int wym, std::vector<XferTile> &out) {
    out.clear();
    for (int k = 0; k < Lo.K; ++k) {
      const PatchDev &pi = Li.pd[k], &po = Lo.pd[k];
      for (int y0 = 0; y0 < po.n[1]; y0 += 16)
        for (int x0 = 0; x0 < po.n[0]; x0 += tx) {
          XferTile t{};
          t.in_off = pi.off;
          t.out_off = po.off;
          t.in_nx = pi.n[0];
          t.out_nx = po.n[0];
          for (int g = 0; g < 2; ++g) {
            const int o0 = g == 0 ? x0 : y0;
            const int o1 = std::min(po.n[g], o0 + (g == 0 ? tx : 16)) - 1;
            const int base = (coarse_side ? F.pd[k].xr[g] : F.pd[k].xp[g]) + o0;
            int mn = lo[base], mx = lo[base];
            for (int o = 0; o <= o1 - o0; ++o) {
              mn = std::min(mn, lo[base + o]);
              mx = std::max(mx, lo[base + o]);
            }
            t.o0[g] = o0;
            t.no[g] = o1 - o0 + 1;
            t.base[g] = base;
            t.w0[g] = mn;
            t.wn[g] = std::min(mx + W, pi.n[g]) - mn;
            if (t.wn[g] > (g == 0 ? wxm : wym) || mn < 0) return false;
          }
          out.push_back(t);
        }
    }
    return true;
  };
  if (d == 2) {
    std::vector<XferTile> rt, pt;
    F.r_wide = tiles_of(F, C, Rlo, RW, true, XFER_R_TX, XFER_R_WX, XFER_R_WY, rt);
    if (!F.r_wide && !tiles_of(F, C, Rlo, RW, true, XFER_TX, XFER_WX, XFER_WX, rt))
      fail(IGAMG_EUNSUPPORTED, "transfer window exceeds the kernel's LDS tile");
    F.p_wide = tiles_of(C, F, Plo, PW, false, XFER_P_TX, XFER_P_WX, XFER_P_WY, pt);
    if (!F.p_wide && !tiles_of(C, F, Plo, PW, false, XFER_TX, XFER_WX, XFER_WX, pt))
      fail(IGAMG_EUNSUPPORTED, "transfer window exceeds the kernel's LDS tile");
    F.n_rtiles = (int)rt.size();
    F.n_ptiles = (int)pt.size();
    F.d_rtiles = c.arena.upload(rt, c.stream);
    F.d_ptiles = c.arena.upload(pt, c.stream);
  }
  F.PW = PW;
  F.RW = RW;
  F.d_P_lo = c.arena.upload(Plo, c.stream);
  F.d_R_lo = c.arena.upload(Rlo, c.stream);
  if (c.fp32()) {
    F.a32.P_val = c.arena.upload_as<float>(Pv, c.stream);
    F.a32.R_val = c.arena.upload_as<float>(Rv, c.stream);
  } else {
    F.a64.P_val = c.arena.upload_as<double>(Pv, c.stream);
    F.a64.R_val = c.arena.upload_as<double>(Rv, c.stream);
  }
}

static void build_maps(Context &c, const LevelData &L, int **d_cp, int **d_cidx) {
  std::vector<int> cp, cidx;
  for (long long ci = 0; ci < L.N; ++ci) {
    cp.push_back((int)cidx.size());
    for (int t : L.copies(ci)) cidx.push_back(t);
  }
  cp.push_back((int)cidx.size());
  *d_cp = c.arena.upload(cp, c.stream);
  *d_cidx = c.arena.upload(cidx, c.stream);
}

// ---------------------------------------------------------------------------
template <typename T>
static void alloc_work(Context &c, LevelData &L) {
  LevelArrays<T> &A = L.arr<T>();
  const size_t n = (size_t)L.Ntorn * c.nb;
  A.f = c.arena.alloc<T>(n);
  A.u = c.arena.alloc<T>(n);
  A.r = c.arena.alloc<T>(n);
  for (T *v : {A.f, A.u, A.r}) k_fill<T>(v, (T)0, (long long)n, c.stream);
}

template <typename T>
static T *upload_vals(Context &c, const std::vector<double> &v) {
  return c.arena.upload_as<T>(v, c.stream);
}

void init_problem(Context &c, const igamg_patches *P, int degree, double sigma,
                  const igamg_options *o) {
  if (!P || !o) fail(IGAMG_EINVAL, "null argument");
  if (P->dim != 2 && P->dim != 3) fail(IGAMG_EINVAL, "dim must be 2 or 3");
  if (P->n_patches < 1 || !P->corners || !P->elems) fail(IGAMG_EINVAL, "no patches");
  if (degree < 1 || degree > MAXP) fail(IGAMG_EINVAL, "degree out of range 1..8");
  c.d = P->dim;
  c.K = P->n_patches;
  c.pk.assign(c.K, degree);
  if (P->degrees)
    for (int k = 0; k < c.K; ++k) {
      if (P->degrees[k] < 1 || P->degrees[k] > MAXP) fail(IGAMG_EINVAL, "degree out of range 1..8");
      c.pk[k] = P->degrees[k];
    }
  c.p = *std::max_element(c.pk.begin(), c.pk.end());
  c.mixed = *std::min_element(c.pk.begin(), c.pk.end()) != c.p;
  degree = c.p;
  c.opt = *o;
  c.sigma_pen = sigma;
  if (c.opt.gs_tile <= 0) c.opt.gs_tile = 2 * (degree + 1);
  if (c.opt.gs_tile < degree) fail(IGAMG_EINVAL, "gs_tile must be >= degree");
  if (c.opt.mu < 1) c.opt.mu = 1;
  if (c.opt.nu < 1) c.opt.nu = 1;
  if (c.opt.max_rhs < 0 || c.opt.max_rhs > 4096) fail(IGAMG_EINVAL, "max_rhs out of range 0..4096");
  if (c.opt.graphs != 0 && c.opt.graphs != 1) fail(IGAMG_EINVAL, "graphs must be 0 or 1");
  c.nb = c.opt.max_rhs > 0 ? c.opt.max_rhs : 1;
  if (c.opt.discretization == IGAMG_SIPG && !(sigma > 0)) fail(IGAMG_EINVAL, "penalty must be positive");
  const bool use_gs = c.opt.smoother != IGAMG_SMOOTHER_SCMS;
  if (use_gs && c.opt.gs_tile != 2 * (degree + 1))
    fail(IGAMG_EUNSUPPORTED, "Gauss-Seidel tiles of width 2(p+1) only");
  if (c.opt.precision != IGAMG_FP64 && c.opt.precision != IGAMG_FP32 &&
      c.opt.precision != IGAMG_BF16_SCMS)
    fail(IGAMG_EINVAL, "unknown precision");
  if (c.opt.outer < IGAMG_OUTER_PCG || c.opt.outer > IGAMG_OUTER_IR)
    fail(IGAMG_EINVAL, "unknown outer iteration");
  if (c.opt.operator_apply < IGAMG_APPLY_AUTO || c.opt.operator_apply > IGAMG_APPLY_ROWS)
    fail(IGAMG_EINVAL, "unknown operator_apply");
  if (c.opt.operator_apply == IGAMG_APPLY_ROWS &&
      (c.opt.discretization != IGAMG_SIPG || !use_gs))
    fail(IGAMG_EUNSUPPORTED, "stored operator rows exist for SIPG with a Gauss-Seidel smoother only");
  if (c.d == 3 && degree > 4) fail(IGAMG_EUNSUPPORTED, "3D problems: degree 1..4");
  if (c.mixed && c.opt.discretization != IGAMG_SIPG)
    fail(IGAMG_EUNSUPPORTED, "patches of different degrees: SIPG only");
  c.gr = gauss_rule(degree + 1);
  const int nc = 1 << c.d;
  c.corners.assign(c.K, {});
  c.elems_fine.assign(c.K, {1, 1, 1});
  for (int k = 0; k < c.K; ++k) {
    for (int b = 0; b < nc; ++b)
      for (int a = 0; a < c.d; ++a) c.corners[k][b * 3 + a] = P->corners[((size_t)k * nc + b) * c.d + a];
    for (int a = 0; a < c.d; ++a) {
      int e = P->elems[(size_t)k * c.d + a];
      if (e < 1) fail(IGAMG_EINVAL, "element counts must be positive");
      c.elems_fine[k][a] = e;
    }
  }
  build_topology(c);
}

void problem_size(const igamg_patches *P, int degree, const igamg_options *o, long long *n,
                  int *levels) {
  Context c;
  init_problem(c, P, degree, 5.0, o);
  auto lev_el = level_elements(c);
  LevelData L;
  build_level_dofs(c, L, lev_el.back());
  *n = L.N;
  *levels = (int)lev_el.size();
}

void build_context(Context &c, const igamg_patches *P, int degree, double sigma,
                   const igamg_options *o, hipStream_t s, const Lent *lent) {
  PhaseClock pc;
  init_problem(c, P, degree, sigma, o);
  pc.lap("topology");
  c.stream = s;
  HIPCHK(hipGetDevice(&c.device));
  HIPCHK(hipEventCreateWithFlags(&c.ev_scal, hipEventDisableTiming));
  if (lent && lent->device) {
    c.arena.region = (char *)lent->device;
    c.arena.region_cap = lent->device_bytes;
  }
  const bool use_gs = c.opt.smoother != IGAMG_SMOOTHER_SCMS;
  const bool use_scms = c.opt.smoother != IGAMG_SMOOTHER_GS;
  const bool f32 = c.fp32();
  c.d_bad = c.arena.alloc<int>(1);
  k_fill<int>(c.d_bad, 0, 1, c.stream);
  {
    std::vector<GaussRule> rules(MAXQ + 1);
    for (int n = 1; n <= MAXQ; ++n) rules[n] = gauss_rule(n);
    c.d_rules = c.arena.upload(rules, c.stream);
  }
  auto lev_el = level_elements(c);
  const int NL = (int)lev_el.size();
  c.lv.resize(NL);
  const int S1 = 2 * c.p + 1;
  int S = 1;
  for (int g = 0; g < c.d; ++g) S *= S1;
  const int SP = (S + 15) / 16 * 16;  // stencil rows padded to 16-lane groups
  int center = 0;
  for (int g = 0, m = 1; g < c.d; ++g, m *= S1) center += c.p * m;
  for (int l = 0; l < NL; ++l) {
    LevelData &L = c.lv[l];
    L.l = l;
    const bool finest = l == NL - 1;
    // residuals from the stored rows (SIPG Gauss-Seidel levels); a float32
    // cycle keeps the finest level's float64 rows for the outer apply
    const bool rows = c.opt.operator_apply != IGAMG_APPLY_SUMFACT &&
                      c.opt.discretization == IGAMG_SIPG && use_gs && l >= 1;
    const bool keep64 = rows && f32 && finest;
    L.st_apply = rows;
    if (finest) c.apply64_rows = rows;
    pc.lap("misc", c.stream, true);
    build_level_dofs(c, L, lev_el[l]);
    pc.lap("dofs");
    if (c.opt.discretization == IGAMG_SIPG) build_interfaces(c, L);
    pc.lap("interfaces");
    L.d_tabB = c.arena.upload(L.tabB, c.stream);
    L.d_tabD = c.arena.upload(L.tabD, c.stream);
    L.d_mask = c.arena.upload(L.mask, c.stream);
    std::vector<double> w(L.Ntorn, 0.0);
    for (long long ci = 0; ci < L.N; ++ci) w[L.rep[ci]] = 1.0;
    std::vector<int> ip = L.if_ptr.empty() ? std::vector<int>(L.Ntorn + 1, 0) : L.if_ptr;
    L.d_if_ptr = c.arena.upload(ip, c.stream);
    L.d_if_col = c.arena.upload(L.if_col, c.stream);
    // cycle arithmetic on every level; the finest level also keeps the
    // float64 operator and weights of the outer iteration
    if (f32) {
      L.a32.weight = upload_vals<float>(c, w);
      L.a32.if_val = upload_vals<float>(c, L.if_val);
    }
    if (!f32 || finest) {
      L.a64.weight = upload_vals<double>(c, w);
      L.a64.if_val = upload_vals<double>(c, L.if_val);
    }
    // same-side interface terms are added to the Gauss-Seidel stencil rows;
    // cross-patch terms are kept per tile (build_gs)
    std::vector<int> srow, sslot;
    std::vector<double> sval;
    for (long long t = 0; t < L.Ntorn; ++t) {
      if (L.if_ptr.empty()) continue;
      for (int e = L.if_ptr[t]; e < L.if_ptr[t + 1]; ++e) {
        if (L.if_cross[e]) continue;
        const int k = L.patch_of(t);
        const PatchDev &pt = L.pd[k];
        long long a = t - pt.off, b = L.if_col[e] - pt.off;
        // slot in a row of the level's layout ((2p+1)^d entries, p the
        // largest degree)
        int slot = 0, m = 1;
        for (int g = 0; g < c.d; ++g) {
          int ia = (int)(a % pt.n[g]), ib = (int)(b % pt.n[g]);
          a /= pt.n[g];
          b /= pt.n[g];
          if (std::abs(ib - ia) > pt.p) fail(IGAMG_EINVAL, "interface coupling outside the stencil");
          slot += (ib - ia + c.p) * m;
          m *= 2 * c.p + 1;
        }
        srow.push_back((int)t);
        sslot.push_back(slot);
        sval.push_back(L.if_val[e]);
      }
    }
    {
      std::vector<unsigned char> has(L.Ntorn, 0);
      std::vector<int> rows;
      for (long long t = 0; t < L.Ntorn; ++t)
        if (!L.if_ptr.empty() && L.if_ptr[t + 1] > L.if_ptr[t]) {
          has[t] = 1;
          rows.push_back((int)t);
        }
      L.n_if_rows = (int)rows.size();
      L.d_has_if = c.arena.upload(has, c.stream);
      L.d_if_rows = c.arena.upload(rows, c.stream);
    }
    // volume tiles, grouped by patch degree and colour class (one launch
    // each).  A tile of TE elements writes TE + p unknowns per direction;
    // tiles of one class lie m = floor((TE + p - 1) / TE) + 1 tiles apart per
    // direction (TE + p - 1 < m TE), so their output windows are disjoint
    std::vector<VolTile> vt;
    L.vgroups.clear();
    for (int pdeg = 1; pdeg <= MAXP; ++pdeg) {
      const int TE = c.d == 2 ? vol_tile_2d(pdeg) : VOL3D_TILE;
      const int m = (TE + pdeg - 1) / TE + 1;
      int ncls = 1;
      for (int g = 0; g < c.d; ++g) ncls *= m;
      for (int cls = 0; cls < ncls; ++cls) {
        const int first = (int)vt.size();
        for (int k = 0; k < c.K; ++k) {
          if (L.pd[k].p != pdeg) continue;
          for (int e2 = 0; e2 < (c.d == 3 ? L.pd[k].nel[2] : 1); e2 += TE)
            for (int e1 = 0; e1 < L.pd[k].nel[1]; e1 += TE)
              for (int e0 = 0; e0 < L.pd[k].nel[0]; e0 += TE) {
                const int key = (e0 / TE) % m + m * ((e1 / TE) % m + m * ((e2 / TE) % m));
                if (key == cls) vt.push_back(VolTile{k, {e0, e1, e2}});
              }
        }
        if ((int)vt.size() > first) L.vgroups.push_back({pdeg, first, (int)vt.size() - first});
      }
    }
    L.n_vtiles = (int)vt.size();
    L.d_vtiles = c.arena.upload(vt, c.stream);
    if (c.d == 2) {
      std::vector<OpTile2> ot;
      for (const VolTile &v : vt) {
        const PatchDev &pt = L.pd[v.patch];
        OpTile2 o{};
        for (int b = 0; b < 4; ++b)
          for (int a = 0; a < 2; ++a) o.corners[b][a] = pt.corners[b][a];
        o.off = pt.off;
        o.nx = pt.n[0];
        o.nel[0] = pt.nel[0];
        o.nel[1] = pt.nel[1];
        o.tab[0] = pt.tab[0];
        o.tab[1] = pt.tab[1];
        o.e0[0] = v.e0[0];
        o.e0[1] = v.e0[1];
        ot.push_back(o);
      }
      L.d_optiles = c.arena.upload(ot, c.stream);
    }
    if (c.d == 2 && ((use_gs && l >= 1) || c.opt.discretization == IGAMG_SIPG)) {
      std::vector<VolTile> stl;
      L.sgroups.clear();
      for (int pdeg = 1; pdeg <= MAXP; ++pdeg) {
        const int first = (int)stl.size();
        const int RT = stencil_tile_2d(pdeg);
        for (int k = 0; k < c.K; ++k) {
          if (L.pd[k].p != pdeg) continue;
          for (int y = 0; y < L.pd[k].n[1]; y += RT)
            for (int x = 0; x < L.pd[k].n[0]; x += RT) stl.push_back(VolTile{k, {x, y, 0}});
        }
        if ((int)stl.size() > first) L.sgroups.push_back({pdeg, first, (int)stl.size() - first});
      }
      L.n_stiles = (int)stl.size();
      L.d_stiles = c.arena.upload(stl, c.stream);
    }
    // glue groups
    std::vector<int> gp{0}, gi;
    for (long long ci = 0; ci < L.N; ++ci)
      if (L.copies(ci).size() > 1) {
        for (int t : L.copies(ci)) gi.push_back(t);
        gp.push_back((int)gi.size());
      }
    L.n_glue = (int)gp.size() - 1;
    L.d_glue_ptr = c.arena.upload(gp, c.stream);
    L.d_glue_idx = c.arena.upload(gi, c.stream);
    // work vectors ([nb][Ntorn]); the finest float64 iterate is the output of
    // the preconditioner in float64 cycles
    if (f32)
      alloc_work<float>(c, L);
    else
      alloc_work<double>(c, L);
    if (l >= 1) {
      pc.lap("misc", c.stream, true);
      build_transfer(c, L, c.lv[l - 1]);
      pc.lap("transfer");
      if (use_scms) {
        if (f32)
          build_scms<float>(c, L);
        else
          build_scms<double>(c, L);
        pc.lap("scms");
      }
    }
    L.d_pd = c.arena.upload(L.pd, c.stream);
    // float64 stencil rows (volume + same-patch interface terms): the
    // Gauss-Seidel rows, and in the SIPG space the source of the dense
    // blocks of the interface pieces and of the coarse matrix
    const bool sipg = c.opt.discretization == IGAMG_SIPG;
    const bool gs_rows = l >= 1 && use_gs;
    const bool need_st = gs_rows || (sipg && (l == 0 || use_scms));
    double *st64 = nullptr, *id64 = nullptr;
    std::vector<void *> tmp;
    // 2D Gauss-Seidel rows are padded past the level's end: the rows of a
    // ragged tile that lie outside their patch then read padding instead of
    // being clamped (they are never applied)
    long long gs_pad = 0;
    if (gs_rows && c.d == 2) {
      int maxnx = 0;
      for (const PatchDev &pt : L.pd) maxnx = std::max(maxnx, pt.n[0]);
      gs_pad = (long long)c.opt.gs_tile * (maxnx + 1);
    }
    if (need_st) {
      if (gs_rows && (!f32 || keep64)) {
        st64 = L.a64.stencil = c.arena.alloc<double>((size_t)(L.Ntorn + gs_pad) * SP);
        if (gs_pad) k_fill<double>(st64 + (size_t)L.Ntorn * SP, 0.0, gs_pad * SP, c.stream);
        id64 = L.a64.invdiag = c.arena.alloc<double>(L.Ntorn);
      } else if (c.arena.region) {
        // lent region: the float64 staging stays inside it (counted in the footprint)
        st64 = c.arena.alloc<double>((size_t)L.Ntorn * SP);
        if (gs_rows) id64 = c.arena.alloc<double>(L.Ntorn);
      } else {
        HIPCHK(hipMalloc((void **)&st64, (size_t)L.Ntorn * SP * sizeof(double)));
        tmp.push_back(st64);
        if (gs_rows) {
          HIPCHK(hipMalloc((void **)&id64, (size_t)L.Ntorn * sizeof(double)));
          tmp.push_back(id64);
        }
      }
      pc.lap("misc", c.stream, true);
      k_stencil_assemble(c, L, st64);
      int *dr = c.arena.upload(srow, c.stream), *ds = c.arena.upload(sslot, c.stream);
      double *dv = c.arena.upload(sval, c.stream);
      k_stencil_add(dr, ds, dv, (int)srow.size(), st64, SP, c.stream);
      const unsigned char *gmask = L.d_mask;
      if (gs_rows && !sipg) {
        fold_conforming_rows(c, L, st64, SP);
        // a sweep updates owner rows only: 1/a_ii = 0 on the other copies
        std::vector<unsigned char> own(L.Ntorn, 0);
        for (long long ci = 0; ci < L.N; ++ci) own[L.rep[ci]] = 1;
        gmask = c.arena.upload(own, c.stream);
      }
      if (gs_rows) k_invdiag(st64, SP, center, gmask, id64, L.Ntorn, c.stream);
      pc.lap("stencil", c.stream, true);
    }
    // Gauss-Seidel tiles with their cross-patch couplings (conforming: those
    // left by folding the copies' rows into the owner rows above)
    if (gs_rows) {
      build_gs(c, L, keep64);
      pc.lap("gs_tiles");
    }
    if (l >= 1 && use_scms) {
      build_pieces(c, L, sipg ? st64 : nullptr, SP);
      pc.lap("pieces", c.stream, true);
    }
    if (l == 0) {
      // coarse level: dense inverse of A_0, float64 always
      std::vector<int> all(L.N);
      std::iota(all.begin(), all.end(), 0);
      c.N0 = (int)L.N;
      if (c.N0 > 16384)
        fail(IGAMG_EUNSUPPORTED, "coarsest level too large for the direct solve");
      std::vector<double> A0 = sipg ? dense_block_rows(c, L, all, stencil_rows_host(c, L, st64, SP, all).data(), SP)
                                    : dense_block(c, L, all);
      pc.lap("coarse_matrix");
      c.d_A0inv = c.arena.upload(A0, c.stream);
      k_spd_inverse(c.d_A0inv, c.N0, c.d_bad, c.stream);
      // enough (row block, column split) blocks to stream the inverse from HBM
      const int rb = (c.N0 + 63) / 64;
      c.coarse_splits = std::max(1, std::min(16, (512 + rb - 1) / rb));
      c.d_coarse_part = c.arena.alloc<double>((size_t)c.nb * c.coarse_splits * c.N0);
      pc.lap("coarse_inverse", c.stream, true);
      build_maps(c, L, &c.d_c0_cp, &c.d_c0_cidx);
    }
    if (gs_rows && f32) {
      L.a32.stencil = c.arena.alloc<float>((size_t)(L.Ntorn + gs_pad) * SP);
      if (gs_pad) k_fill<float>(L.a32.stencil + (size_t)L.Ntorn * SP, 0.0f, gs_pad * SP, c.stream);
      L.a32.invdiag = c.arena.alloc<float>(L.Ntorn);
      k_convert<double, float>(st64, nullptr, L.a32.stencil, (long long)L.Ntorn * SP, 1, c.stream);
      k_convert<double, float>(id64, nullptr, L.a32.invdiag, L.Ntorn, 1, c.stream);
    }
    if (!tmp.empty()) {
      HIPCHK(hipStreamSynchronize(c.stream));
      for (void *q : tmp) HIPCHK(hipFree(q));
    }
  }
  LevelData &LF = c.lv.back();
  build_maps(c, LF, &c.d_fin_cp, &c.d_fin_cidx);
  // outer iteration vectors, float64, [nb][Ntorn]
  const size_t nt = (size_t)LF.Ntorn * c.nb;
  c.x = c.arena.alloc<double>(nt);
  c.rr = c.arena.alloc<double>(nt);
  c.z = f32 ? c.arena.alloc<double>(nt) : LF.a64.u;  // float64 cycles write z in place
  c.pp = c.arena.alloc<double>(nt);
  c.qq = c.arena.alloc<double>(nt);
  c.ff = c.arena.alloc<double>(nt);
  for (double *v : {c.x, c.rr, c.z, c.pp, c.qq, c.ff}) k_fill(v, 0.0, (long long)nt, c.stream);
  if (c.opt.outer == IGAMG_OUTER_FCG) {
    c.rold = c.arena.alloc<double>(nt);
    k_fill(c.rold, 0.0, (long long)nt, c.stream);
  }
  if (c.opt.outer == IGAMG_OUTER_IR && f32) {
    for (float **v : {&c.d32, &c.r32, &c.p32, &c.q32}) {
      *v = c.arena.alloc<float>(nt);
      k_fill(*v, 0.0f, (long long)nt, c.stream);
    }
  } else if (c.opt.outer == IGAMG_OUTER_IR) {
    c.dd = c.arena.alloc<double>(nt);
    c.rin = c.arena.alloc<double>(nt);
    k_fill(c.dd, 0.0, (long long)nt, c.stream);
    k_fill(c.rin, 0.0, (long long)nt, c.stream);
  }
  c.d_red = c.arena.alloc<double>((size_t)2 * RED_BLOCKS * c.nb);
  c.d_scal = c.arena.alloc<double>((size_t)S_COUNT * c.nb);
  k_fill(c.d_scal, 0.0, (long long)S_COUNT * c.nb, c.stream);
  c.d_active = c.arena.alloc<int>(c.nb);
  const size_t pinned_need = (size_t)S_COUNT * c.nb * sizeof(double) + (size_t)c.nb * sizeof(int);
  if (lent && lent->pinned && lent->pinned_bytes >= pinned_need) {
    c.own_pinned = false;
    c.h_scal = (double *)lent->pinned;
    c.h_active = (int *)(c.h_scal + (size_t)S_COUNT * c.nb);
  } else {
    HIPCHK(hipHostMalloc((void **)&c.h_active, (size_t)c.nb * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c.h_scal, (size_t)S_COUNT * c.nb * sizeof(double),
                         hipHostMallocDefault));
  }
  for (int j = 0; j < c.nb; ++j) c.h_active[j] = 1;
  HIPCHK(hipMemcpyAsync(c.d_active, c.h_active, c.nb * sizeof(int), hipMemcpyHostToDevice,
                        c.stream));
  {
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c.d_bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (bad) fail(IGAMG_EINVAL, "matrix of a smoother piece or the coarse level is not SPD");
  }
  HIPCHK(hipGetLastError());
  c.arena.staging.clear();
  pc.lap("misc");
  pc.report(c.lv.back().N);
}

// ---------------------------------------------------------------------------
// roofline model: algorithmic work of one launch (not counting redundant
// loads of tile halos or recomputation)
// ---------------------------------------------------------------------------
void kernel_model(const Context &c, const std::string &fam, int level, int nrhs, double *bytes,
                  double *flops) {
  const LevelData &L = c.lv[level];
  const double nt = (double)L.Ntorn;
  const double wb = c.fp32() ? 4.0 : 8.0;  // bytes of a value in the cycle arithmetic
  const double nb = nrhs < 1 ? 1.0 : (double)nrhs;
  const int q = c.p + 1, P1 = c.p + 1;
  int S = 1;
  for (int g = 0; g < c.d; ++g) S *= (2 * c.p + 1);
  const double nnz = L.if_col.size();
  *bytes = 0;
  *flops = 0;
  if (fam == "vol_apply" && c.d == 3) {
    // per element: the three contractions and their transposes over the
    // tile's Gauss points, the metric (~150 flops) and its product
    double el = 0;
    for (int k = 0; k < c.K; ++k) el += (double)L.pd[k].nel[0] * L.pd[k].nel[1] * L.pd[k].nel[2];
    const double q4 = (double)q * q * q * q, q3 = (double)q * q * q;
    *flops = nb * el * (32.0 * q4 + 170.0 * q3);
    *bytes = 3.0 * wb * nt * nb;
  } else if (fam == "vol_apply") {
    for (int k = 0; k < c.K; ++k) {
      const PatchDev &pt = L.pd[k];
      double Qx = (double)pt.nel[0] * q, Qy = (double)pt.nel[1] * q;
      *flops += 4.0 * pt.n[1] * Qx * P1;        // x-contraction (values and derivatives)
      *flops += 4.0 * Qy * Qx * P1;             // y-contraction
      *flops += 60.0 * Qx * Qy;                 // metric from the corners, 2x2 product
      *flops += 4.0 * pt.n[1] * Qx * P1;        // transposed y-contraction
      *flops += 4.0 * pt.n[1] * pt.n[0] * Qx / pt.nel[0] * P1;  // transposed x-contraction
    }
    *flops *= nb;
    *bytes = 3.0 * wb * nt * nb;                // read u, read and write r
  } else if (fam == "gauss_seidel") {
    // one colour-class launch, algorithmic bytes only: the (2p+1)^d stencil
    // of every unknown read once for the batch, f and u read and u written
    // per right-hand side (compact unknowns: no padding, masks, Dirichlet
    // rows or cross-patch coupling lists); a sweep is split evenly over its
    // class launches
    int launches = 0;
    for (const GsClass &cl : L.gs) launches += cl.count > 0;
    if (launches == 0) launches = 1;
    const double n = (double)L.N;
    *bytes = (n * wb * S + nb * n * 3.0 * wb) / launches;
    *flops = nb * 2.0 * S * n / launches;
  } else if (fam == "stencil_apply" || fam == "outer_apply" || fam == "stencil_rows") {
    // algorithmic bytes: the (2p+1)^d stencil of every unknown once for the
    // batch; u and f read and r written per right-hand side (outer_apply:
    // the float64 finest-level operator of a mixed-precision solve;
    // stencil_rows: the row kernel of a float32 batch, whose transposed
    // input and cross-patch couplings are launched beside it)
    const double b = fam == "outer_apply" ? 8.0 : wb;
    const double n = (double)L.N;
    *bytes = n * b * S + nb * n * 3.0 * b;
    *flops = nb * 2.0 * S * n;
  } else if (fam == "scms") {
    // one application to the patch interiors: four products per patch;
    // bytes: r read, u read and written per right-hand side, the factors once
    // (3D: six mode products, each m^3 times the contracted extent)
    for (int k = 0; k < c.K; ++k) {
      double mx = L.pd[k].n[0] - 2, my = L.pd[k].n[1] - 2;
      if (c.d == 3) {
        double mz = L.pd[k].n[2] - 2, m3 = mx * my * mz;
        *flops += nb * 4.0 * m3 * (mx + my + mz);
        *bytes += nb * 3.0 * wb * m3 + wb * 2.0 * (mx * mx + my * my + mz * mz);
        continue;
      }
      *flops += nb * 2.0 * (my * my * mx + my * mx * mx + my * my * mx + my * mx * mx);
      *bytes += nb * 3.0 * wb * mx * my + wb * 2.0 * (mx * mx + my * my);
    }
  } else if (fam == "pieces") {
    // stored inverses once, the pieces' residuals read and corrections added
    *bytes = wb * L.piece_sq + L.piece_n * 8.0 + nb * 3.0 * wb * L.piece_n;
    *flops = nb * 2.0 * L.piece_sq;
  } else if (fam == "restrict" || fam == "prolong") {
    // level = the fine side; restriction reads r_f and writes r_c (and clears
    // the coarse iterate), prolongation reads e_c and updates u_f
    if (level < 1) fail(IGAMG_EINVAL, "transfers start on level 1");
    const double nc = (double)c.lv[level - 1].Ntorn;
    *bytes = nb * wb * (fam == "restrict" ? nt + 2.0 * nc : nc + 2.0 * nt);
    *flops = nb * 2.0 * nt * (L.PW + L.RW);
  } else if (fam == "coarse") {
    const double n0 = (double)c.N0;
    *bytes = n0 * n0 * 8.0 + nb * 2.0 * 8.0 * n0;
    *flops = nb * 2.0 * n0 * n0;
  } else if (fam == "iface_apply") {
    *bytes = nt * 2.0 + nnz * (4.0 + wb) + nb * (nt * 2.0 * wb + nnz * wb);
    *flops = nb * 2.0 * nnz;
  } else {
    fail(IGAMG_EINVAL, "no model for this kernel family");
  }
}

size_t estimate_footprint(const igamg_patches *P, int degree, const igamg_options *o) {
  if (!P || !o || P->dim < 2 || P->dim > 3 || P->n_patches < 1 || degree < 1 || !P->elems)
    fail(IGAMG_EINVAL, "invalid problem");
  const int d = P->dim, p = degree;
  const int nb = o->max_rhs > 0 ? o->max_rhs : 1;
  const double wb = o->precision != IGAMG_FP64 ? 4.0 : 8.0;
  long long fine = 0;
  for (int k = 0; k < P->n_patches; ++k) {
    long long n = 1;
    for (int a = 0; a < d; ++a) n *= (P->elems[(size_t)k * d + a] + p);
    fine += n;
  }
  // levels shrink by 2^d; geometric sum bounded by 2^d/(2^d-1)
  const double all_levels = fine * (double)(1 << d) / ((1 << d) - 1);
  int S = 1;
  for (int a = 0; a < d; ++a) S *= (2 * p + 1);
  const int SP = (S + 15) / 16 * 16;
  const bool gs = o->smoother != IGAMG_SMOOTHER_SCMS;
  const bool scms = o->smoother != IGAMG_SMOOTHER_GS;
  // per unknown and level: f, u, r per right-hand side, two SCMS intermediates,
  // stencil row and 1/a_ii, weight, masks and index maps
  double per = wb * (3.0 * nb + (scms ? 2.0 * nb : 0) + (gs ? SP + 1 : 0) + 1) + 16.0;
  double bytes = all_levels * per;
  // dense inverses: interface pieces (both sides' boundary layers of every
  // interface, summed over levels) and the coarse level
  for (int k = 0; k < P->n_patches; ++k) {
    double side = 1.0;
    for (int a = 1; a < d; ++a) side *= (P->elems[(size_t)k * d + a] + p);
    bytes += 2.0 * d * (2.0 * side) * (2.0 * side) * 8.0 * ((1 << d) / ((1 << d) - 1.0)) / 2.0 *
             (wb == 4.0 ? 1.5 : 1.0);
    // stencil rows of the piece unknowns gathered at setup (kept inside a lent region)
    bytes += 2.0 * d * side * (SP * 8.0 + 4.0) * ((1 << d) / ((1 << d) - 1.0));
  }
  {
    // coarsest element counts by the halving rule of the hierarchy
    const int cmin = o->coarse_min > 0 ? o->coarse_min : 2;
    std::vector<int> e(P->elems, P->elems + (size_t)P->n_patches * d);
    for (;;) {
      bool ok = true;
      for (int v : e) ok = ok && v % 2 == 0 && v / 2 >= cmin;
      if (!ok) break;
      for (int &v : e) v /= 2;
    }
    double n0 = 0.0;
    for (int k = 0; k < P->n_patches; ++k) {
      double m = 1.0;
      for (int a = 0; a < d; ++a) m *= (e[(size_t)k * d + a] + p);
      n0 += m;
    }
    bytes += n0 * n0 * 8.0 + n0 * (SP * 8.0 + 4.0);
  }
  // outer float64 vectors [nb][Ntorn]: x, r, z, p, q, f (+ r_old)
  bytes += fine * 8.0 * nb *
           (7 + (o->outer == IGAMG_OUTER_FCG ? 1 : 0) + (o->outer == IGAMG_OUTER_IR ? 2 : 0));
  // float32 setup assembles the stencils in float64 first: freed afterwards
  // with driver allocations, kept inside a lent region (every level)
  if (gs && wb == 4.0) bytes += all_levels * 8.0 * (SP + 1);
  // padding rows past the end of the 2D Gauss-Seidel rows (one tile height
  // of the widest patch per level; levels halve, so twice the finest bound)
  if (gs && d == 2) {
    int maxn = 0;
    for (int k = 0; k < P->n_patches; ++k) maxn = std::max(maxn, P->elems[(size_t)k * d] + p);
    bytes += 2.0 * (2.0 * (p + 1)) * (maxn + 1) * SP * (wb + (wb == 4.0 ? 8.0 : 0.0));
  }
  // margin for the terms estimated from counts (interface lists, tiles); at
  // 8 % a 2000-request serving stream had 11 requests allocate past their block
  return (size_t)(bytes * 1.15) + (32u << 20);
}

}  // namespace igamg
