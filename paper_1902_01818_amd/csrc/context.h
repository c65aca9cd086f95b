// The solver context: hierarchy, device data and work vectors.
#pragma once
#include <array>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

namespace igamg {

// Device allocation of a context.  By default every array is a hipMalloc of
// its own.  A caller-provided region (the serving runtime's per-request block)
// is bump-allocated instead, so that a request allocates nothing from the
// driver while other requests run; arrays beyond the region fall back to
// hipMalloc and are counted.
struct Arena {
  std::vector<void *> ptrs;      // hipMalloc'd (freed by release)
  size_t bytes = 0;              // bytes handed out
  char *region = nullptr;        // optional external region
  size_t region_cap = 0, region_used = 0;
  int fallbacks = 0;             // allocations that did not fit the region
  void *raw(size_t nbytes) {
    if (nbytes == 0) nbytes = 1;
    const size_t a = (nbytes + 255) / 256 * 256;
    bytes += a;
    if (region && region_used + a <= region_cap) {
      void *p = region + region_used;
      region_used += a;
      return p;
    }
    if (region) ++fallbacks;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, a);
    if (e != hipSuccess) fail(IGAMG_ENOMEM, "hipMalloc failed");
    ptrs.push_back(p);
    return p;
  }
  template <typename T>
  T *alloc(size_t n) {
    return (T *)raw(n * sizeof(T));
  }
  template <typename T>
  T *upload(const std::vector<T> &v, hipStream_t s) {
    T *p = alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  // upload a float64 host array as T (host copy kept alive until the stream syncs)
  template <typename T>
  T *upload_as(const std::vector<double> &v, hipStream_t s) {
    staging.emplace_back();
    std::vector<char> &buf = staging.back();
    buf.resize(v.size() * sizeof(T));
    T *h = (T *)buf.data();
    for (size_t i = 0; i < v.size(); ++i) h[i] = (T)v[i];
    T *p = alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, h, v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  std::vector<std::vector<char>> staging;
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
    region_used = 0;
  }
};

// Device scratch owned for one scope (freed also when an error unwinds it).
struct DeviceScratch {
  void *p = nullptr;
  DeviceScratch() = default;
  DeviceScratch(const DeviceScratch &) = delete;
  DeviceScratch &operator=(const DeviceScratch &) = delete;
  template <typename T>
  T *alloc(size_t n) {
    HIPCHK(hipMalloc(&p, n * sizeof(T) > 0 ? n * sizeof(T) : 1));
    return (T *)p;
  }
  ~DeviceScratch() {
    if (p) (void)hipFree(p);
  }
};

// Resources a caller may lend to a context (serving runtime): a device region
// for all arrays and pinned host memory for the scalar read-back.
struct Lent {
  void *device = nullptr;
  size_t device_bytes = 0;
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
};

struct GsClass {
  GsTile *tiles = nullptr;    // 2D tiles
  GsTile3 *tiles3 = nullptr;  // 3D tiles
  int count = 0;
};

// Arrays of one level in one arithmetic precision.  Work vectors hold a batch
// of right-hand sides, one after the other with stride Ntorn.
template <typename T>
struct LevelArrays {
  T *f = nullptr, *u = nullptr, *r = nullptr;  // cycle right-hand side, iterate, residual
  T *stencil = nullptr, *invdiag = nullptr;    // Gauss-Seidel rows (volume + same-side interface)
  T *if_val = nullptr;                         // interface CSR values
  T *gcx_val = nullptr;                        // cross-patch couplings per Gauss-Seidel tile
  T *piece_inv = nullptr;                      // inverses of the interface pieces
  T *P_val = nullptr, *R_val = nullptr;        // banded 1D embeddings (from the coarser level)
  T *weight = nullptr;                         // 1 on the representative copy of a free unknown
  T *wscratch = nullptr;                       // fast-diagonalization intermediate
  T *wscratch2 = nullptr;                      // second intermediate of the staged form
  Fd2Item<T> *fd[2] = {nullptr, nullptr};      // patch interiors: forward, backward
  FdGemm<T> *fg[6] = {};                      // the same as product stages (2D: 4, 3D: 6)
  FdWide<T> *fw[4] = {};                       // 2D stages over a whole batch (wide tiles)
  T *lam_xy = nullptr;                         // 3D: lam_y[j] + lam_x[i] per patch (y-major)
  T *x_val = nullptr;                          // 3D: cross-patch couplings (CSR of coupled rows)
  T *xsum = nullptr;                           // 3D: sum of a colour's cross couplings per row
};

struct LevelData {
  int l = 0;
  int K = 0;
  std::vector<PatchDev> pd;                 // host copy
  PatchDev *d_pd = nullptr;
  long long Ntorn = 0;
  long long N = 0;                          // compact unknowns
  std::vector<unsigned char> mask;          // 1 = free, 0 = Dirichlet
  std::vector<int> comp;                    // torn -> compact (-1 Dirichlet)
  std::vector<int> rep;                     // compact -> representative torn
  std::vector<int> copy_ptr, copy_idx;      // compact -> all torn copies (CSR; conforming
                                            // glue gives several, SIPG exactly one)
  struct Span {
    const int *b, *e;
    const int *begin() const { return b; }
    const int *end() const { return e; }
    size_t size() const { return (size_t)(e - b); }
  };
  // patch holding torn index t (patches are stored in offset order)
  int patch_of(long long t) const {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (pd[mid].off <= t)
        lo = mid;
      else
        hi = mid - 1;
    }
    return lo;
  }
  Span copies(long long ci) const {
    return Span{copy_idx.data() + copy_ptr[ci], copy_idx.data() + copy_ptr[ci + 1]};
  }
  // element tables of this level (distinct element counts share entries)
  std::vector<double> tabB, tabD;
  double *d_tabB = nullptr, *d_tabD = nullptr;
  // interface CSR over torn rows: all interface terms, cross-patch part flagged
  std::vector<int> if_ptr, if_col;
  std::vector<double> if_val;
  std::vector<unsigned char> if_cross;
  int *d_if_ptr = nullptr, *d_if_col = nullptr;
  // rows carrying interface terms (lane-parallel part of the residual kernel)
  unsigned char *d_has_if = nullptr;
  int *d_if_rows = nullptr;
  int n_if_rows = 0;
  // cross-patch couplings per Gauss-Seidel tile: (row inside tile, column)
  int *d_gcx_li = nullptr, *d_gcx_col = nullptr;
  // conforming Gauss-Seidel levels: the cross-patch couplings of every owner
  // row (first copy of a compact unknown) as a CSR over torn rows (host), and
  // the mirror writes of the tiles (row inside tile, torn copy to overwrite)
  std::vector<int> cf_ptr, cf_col;
  std::vector<double> cf_val;
  int *d_mr_li = nullptr, *d_mr_dst = nullptr;
  unsigned char *d_mask = nullptr;
  // glue groups (conforming): CSR of torn copies of every shared unknown
  int n_glue = 0;
  int *d_glue_ptr = nullptr, *d_glue_idx = nullptr;
  // tiles
  VolTile *d_vtiles = nullptr;
  OpTile2 *d_optiles = nullptr;  // the same tiles with their patch fields (operator kernel)
  int n_vtiles = 0;
  VolTile *d_stiles = nullptr;  // row tiles of the stencil assembly (first row in e0)
  int n_stiles = 0;
  // tiles grouped by patch degree (degree, first tile, count): the volume
  // operator (d_vtiles / d_optiles) and the stencil assembly (d_stiles)
  std::vector<std::array<int, 3>> vgroups, sgroups;
  std::vector<GsClass> gs;  // classes in key order
  GsTile *d_atiles = nullptr;  // every Gauss-Seidel tile of the level (stored-row operator)
  GsTile3 *d_atiles3 = nullptr;  // the same for 3D patches
  // 2D: row blocks (sp_rhs_bx(p) x 8) of the lane-per-right-hand-side operator
  GsTile *d_sptiles = nullptr;
  int n_sptiles = 0;
  // its transposed right-hand sides: per group of 64, every patch with a halo
  // of p zero rows and columns ([group][pad_tot + slack][64]; the halo is
  // zeroed at setup and never written)
  float *ut = nullptr;
  long long *d_plines = nullptr;  // per patch line: torn offset, padded offset, length
  int n_plines = 0;
  long long pad_tot = 0;
  // cross-patch couplings as a CSR over the coupled rows (3D: rows grouped by
  // patch colour, x_cptr[c] .. x_cptr[c+1]; 2D: in torn order, for the
  // lane-per-right-hand-side operator)
  int *d_x_rows = nullptr, *d_x_ptr = nullptr, *d_x_col = nullptr;
  int x_n = 0;
  std::vector<int> x_cptr;
  int n_atiles = 0;
  // the cycle's residuals on this level use the stored rows (k_stencil_apply)
  bool st_apply = false;
  // SCMS interiors
  int n_fd = 0;
  int fd_rows = 0, fd_K1 = 0, fd_N = 0;
  int fg_tiles = 0;       // 64 x 64 output tiles of the largest stage item
  int fw_wide = 0, fw_cat = 0;  // 2D batch stages: largest wide and per-right-hand-side extents
  int fg_n[6] = {}, fg_t[6] = {};  // 3D: items and largest tile count of each stage
  long long fd_work = 0;  // sum over patches of my * mx * ceil(my / 16) (fused-form re-reads)
  long long wscratch_n = 0;
  // interface pieces
  PieceDev *d_pieces = nullptr;
  int n_pieces = 0, max_piece = 0;
  double piece_sq = 0, piece_n = 0;  // sums of n_T^2 and n_T over the pieces (kernel model)
  int *d_piece_idx = nullptr, *d_piece_cp = nullptr, *d_piece_cidx = nullptr;
  // transfer tables between this level and the next coarser one
  int *d_P_lo = nullptr, *d_R_lo = nullptr;
  int PW = 0, RW = 0;
  XferTile *d_rtiles = nullptr, *d_ptiles = nullptr;  // coarse-side / fine-side output tiles
  int n_rtiles = 0, n_ptiles = 0;
  // 2D output tiles 16 rows high: 32 coarse (restriction) / 64 fine
  // (prolongation) columns wide, or 16 where a window exceeds those kernels'
  bool r_wide = false, p_wide = false;
  LevelArrays<double> a64;
  LevelArrays<float> a32;
  template <typename T>
  LevelArrays<T> &arr();
};
template <>
inline LevelArrays<double> &LevelData::arr<double>() { return a64; }
template <>
inline LevelArrays<float> &LevelData::arr<float>() { return a32; }

struct TimerFamily {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double ms = 0.0;
  int64_t launches = 0;
};

struct Context {
  int d = 2, p = 2, K = 0;  // p: the largest degree of the patches
  std::vector<int> pk;      // degree per patch (the non-matching spaces of Section 5)
  bool mixed = false;       // patches of different degrees
  GaussRule *d_rules = nullptr;  // Gauss rules by number of points (device, [MAXQ + 1])
  igamg_options opt{};
  double sigma_pen = 5.0;
  GaussRule gr{};
  int nb = 1;  // right-hand sides the work vectors hold (batch capacity)
  std::vector<std::array<double, 24>> corners;   // [K][8*3]
  std::vector<std::array<int, 3>> elems_fine;
  // topology
  std::vector<std::vector<int>> vid;              // [K][2^d] vertex ids
  struct Iface {
    int k, dk, sk, l, dl, sl;
    double eta;
  };
  std::vector<Iface> ifaces;
  std::vector<std::array<unsigned char, 6>> boundary;  // [K][2*dir+s]
  std::vector<int> color;
  int n_colors = 1;
  std::vector<double> measure;
  std::vector<LevelData> lv;                      // level 0 = coarsest
  int *d_bad = nullptr;  // set by setup kernels when a dense block is not SPD
  // coarse solve (float64 always)
  int N0 = 0;
  int coarse_splits = 1;            // column splits of the dense solve
  double *d_coarse_part = nullptr;  // partial row sums [nb][splits][N0]
  double *d_A0inv = nullptr;
  int *d_c0_cp = nullptr, *d_c0_cidx = nullptr;  // compact -> copies CSR
  // finest-level maps (ABI)
  int *d_fin_cp = nullptr, *d_fin_cidx = nullptr;
  bool apply64_rows = false;  // the float64 finest-level apply reads the stored rows
  // outer iteration vectors (float64, torn layout, finest level, [nb][Ntorn])
  double *x = nullptr, *rr = nullptr, *z = nullptr, *pp = nullptr, *qq = nullptr, *ff = nullptr;
  double *rold = nullptr;        // previous residual (flexible CG)
  double *dd = nullptr, *rin = nullptr;  // inner correction and residual (refinement)
  // float32 cycles: the refinement's inner iteration in float32 vectors
  // (correction, residual, direction, operator times direction; its
  // preconditioned residual is the finest float32 iterate)
  float *d32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
  double *d_red = nullptr;       // reduction partials [nb][RED_BLOCKS]
  hipEvent_t ev_scal = nullptr;  // marks the scalars' copy to the host mirror
  double *d_scal = nullptr;      // device scalars [nb][S_COUNT]
  double *h_scal = nullptr;      // pinned host mirror
  int *d_active = nullptr;       // per right-hand side: 1 = still iterating
  int *h_active = nullptr;       // pinned host mirror (written only after a stream sync)
  bool own_pinned = true;        // h_scal / h_active allocated by the context
  hipStream_t stream = nullptr;
  // preconditioner cycles replayed from HIP graphs (option graphs): one per
  // (residual vector, batch size); uses counts first runs, captured at the
  // second on a private stream (the caller's may be the null stream)
  struct CycleGraph {
    const void *r = nullptr;  // residual the cycle reads (float64 or float32)
    int nb = 0;
    int uses = 0;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<CycleGraph> graphs;
  hipStream_t cap_stream = nullptr;
  int device = 0;  // HIP device the context was built on
  Arena arena;
  std::map<std::string, TimerFamily> timers;
  std::string timing_filter;  // time only families whose key starts with this

  // float32 cycle (IGAMG_FP32, or IGAMG_BF16_SCMS whose patch-interior
  // contractions take bfloat16 operands)
  bool fp32() const { return opt.precision != IGAMG_FP64; }
  bool bf16_scms() const { return opt.precision == IGAMG_BF16_SCMS; }
  void launch_begin(const char *fam, hipEvent_t *b, hipEvent_t *e);
  void launch_end(const char *fam, hipEvent_t b, hipEvent_t e, int launches = 1);
  ~Context();
};

// Validate the input and build the topology (host only, no GPU work).
void init_problem(Context &c, const igamg_patches *P, int degree, double sigma,
                  const igamg_options *o);
// Finest-level unknowns and level count of a problem (host only).
void problem_size(const igamg_patches *P, int degree, const igamg_options *o, long long *n,
                  int *levels);
void build_context(Context &c, const igamg_patches *P, int degree, double sigma,
                   const igamg_options *o, hipStream_t s, const Lent *lent = nullptr);
size_t estimate_footprint(const igamg_patches *P, int degree, const igamg_options *o);
// algorithmic bytes / flops of one launch of a kernel family on a level for a
// batch of nrhs right-hand sides
void kernel_model(const Context &c, const std::string &family, int level, int nrhs,
                  double *bytes, double *flops);

// cycle / outer iteration (cycle.cpp); vectors in torn layout, nrhs <= c.nb
void apply64(Context &c, const double *u, const double *f, const double *fw, double *r,
             double alpha, int nrhs);
void vcycle_compact(Context &c, const double *f, double *u, int nrhs);
int solve_batch(Context &c, const double *rhs, double *u, int nrhs, double tol, int maxit,
                int use_x0, igamg_solve_info *info);

}  // namespace igamg
