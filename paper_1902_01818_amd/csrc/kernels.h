// Kernel launchers (kernels.hip).  All launches are asynchronous on the
// context stream (or `s`).  Work vectors of the cycle carry a batch of nrhs
// right-hand sides with stride Ntorn; operator data is shared by the batch.
#pragma once
#include "context.h"

namespace igamg {

constexpr int RED_BLOCKS = 256;  // partial sums per right-hand side of a reduction
constexpr int VOL3D_TILE = 2;    // elements per direction of a 3D volume-operator tile

// elementwise (batched: n values per right-hand side, nrhs of them)
template <typename T>
void k_fill(T *x, T v, long long n, hipStream_t s);
// y = w .* x converted to To (w = null: plain conversion), per right-hand side;
// zero (optional) is cleared alongside; with `active`, right-hand sides j with
// active[j] == 0 are skipped
template <typename Ti, typename To>
void k_convert(const Ti *x, const To *w, To *y, long long n, int nrhs, hipStream_t s,
               To *zero = nullptr, const int *active = nullptr);

// setup
void k_stencil_assemble(Context &c, LevelData &L, double *out);
void k_stencil_add(const int *rows, const int *slots, const double *vals, int n, double *stencil,
                   int S, hipStream_t s);
void k_invdiag(const double *stencil, int S, int center, const unsigned char *mask, double *invd,
               long long n, hipStream_t s);
// squared L2 error of torn coefficients ut against prod sin(pi x), summed in a
// fixed order into out[0] (part: l2_error_partials(nel) scratch values)
void k_l2_error(Context &c, LevelData &L, const double *ut, const long long *el_off,
                const int *tab, const double *tB, const GaussRule &gq, double *part,
                long long nel, double *out);
long long l2_error_partials(long long nel);
// strip width (rows of one line) of the lane-per-right-hand-side stored-row
// operator for degree p, 0 = not available
int sp_rhs_bx(int p);
// float32 batches of at least this many right-hand sides take that operator
constexpr int SP_RHS_MIN = 32;
// Device scratch of the allocation-free entry points: NOALLOC_SCRATCH_BYTES
// per GPU.  noalloc_scratch_init() looks up its address on the current device
// (once per device) and returns it; noalloc_scratch(device) returns the
// address found for that device, or null before the lookup.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
void *noalloc_scratch_init();
void *noalloc_scratch(int device);
void k_load_manufactured(Context &c, LevelData &L, double *out);
// in-place inverse of a dense SPD n x n matrix (blocked Gauss-Jordan);
// bad[0] is set to 1 when a pivot is not positive (not SPD)
void k_spd_inverse(double *A, int n, int *bad, hipStream_t s);
// the same for nmat matrices at base + offs[z] of orders ns[z] <= nmax (device
// arrays), one launch per kernel and block step for the whole batch
void k_spd_inverse_batch(double *base, const long long *offs, const int *ns, int nmat, int nmax,
                         int *bad, hipStream_t s);
// out[r][:] = st[rows[r]][:] (rows of SP values)
void k_gather_rows(const double *st, int SP, const int *rows, int nrows, double *out,
                   hipStream_t s);

// operator: r = mask (beta fw.*f + alpha A u); volume part by sum factorization
template <typename T>
void k_iface_apply(Context &c, LevelData &L, const T *u, const T *f, const T *fw, T beta, T alpha,
                   T *r, int nrhs);
template <typename T>
void k_vol_apply(Context &c, LevelData &L, const T *u, T *r, T alpha, int nrhs);
template <typename T>
void k_glue_sum(LevelData &L, T *y, int nrhs, hipStream_t s);
// the same operator from the stored rows of levels that keep them (SIPG
// Gauss-Seidel levels): r = mask (beta fw.*f + alpha A u), no glue needed
template <typename T>
void k_stencil_apply(Context &c, LevelData &L, const LevelArrays<T> &A, const T *u, const T *f,
                     const T *fw, T beta, T alpha, T *r, int nrhs);

// smoothers (on L.arr<T>().f / .u / .r)
template <typename T>
void k_gs_sweep(Context &c, LevelData &L, bool backward, int nrhs);
// patch interiors; returns true when the interface pieces ran in the same
// launches (then k_pieces is not called for this step)
template <typename T>
bool k_scms_interior(Context &c, LevelData &L, int nrhs);
template <typename T>
void k_pieces(Context &c, LevelData &L, int nrhs);

// transfer between level F (fine) and C (coarse); restriction also zeroes
// uc_zero (the coarse initial guess) when given
template <typename T>
void k_restrict(Context &c, LevelData &F, LevelData &C, const T *rf, T *rc, T *uc_zero, int nrhs);
template <typename T>
void k_prolong_add(Context &c, LevelData &F, LevelData &C, const T *ec, T *uf, int nrhs);
template <typename T>
void k_coarse_solve(Context &c, const T *f0, T *u0, int nrhs);

// compact <-> torn (float64, batched: compact stride N, torn stride Ntorn)
void k_scatter_compact(const double *xc, long long N, const int *cp, const int *cidx, double *xt,
                       long long Ntorn, int nrhs, hipStream_t s);
void k_gather_compact(const double *xt, long long N, const int *cp, const int *cidx, int sum,
                      double *xc, long long Ntorn, int nrhs, hipStream_t s);

// deterministic reductions and outer updates; scalars per right-hand side in
// c.d_scal[j * S_COUNT + slot]; c.d_active masks converged right-hand sides
enum Scalar { S_RZ = 0, S_PQ, S_RR, S_RZNEW, S_FF, S_ALPHA, S_BETA, S_TMP, S_ZRO, S_COUNT };
// mode 0: scal[slot] = sum; 1: alpha = rz / sum; 2: beta = sum / rz, rz = sum
void k_dot(Context &c, const double *a, const double *b, long long n, int slot, int mode, int nrhs);
void k_dot(Context &c, const float *a, const float *b, long long n, int slot, int mode, int nrhs);
// flexible CG: beta = ((z, r) - (z, r_old)) / rz, rz = (z, r)
void k_dot_fcg(Context &c, long long n, int nrhs);
// x += alpha p, r -= alpha q, ||r||^2 into S_RR; zeroes z; optionally keeps r_old
void k_pcg_update_xr(Context &c, long long n, int nrhs, bool keep_rold);
void k_pcg_update_p(Context &c, long long n, int nrhs);
// the same on float32 vectors given explicitly (the inner iteration of the
// refinement): x += alpha p, r -= alpha q, ||r||^2 into S_RR, z_zero = 0;
// p = z + beta p
void k_pcg_update_xr(Context &c, float *x, float *r, const float *p, const float *q,
                     float *z_zero, long long n, int nrhs);
void k_pcg_update_p(Context &c, float *p, const float *z, long long n, int nrhs);
// y += x for the active right-hand sides
void k_add_active(Context &c, double *y, const double *x, long long n, int nrhs);
void k_add_active(Context &c, double *y, const float *x, long long n, int nrhs);

}  // namespace igamg
