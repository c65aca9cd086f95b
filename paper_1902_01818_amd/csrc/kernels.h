// Kernel launchers (kernels.hip).  All launches are asynchronous on `s`.
#pragma once
#include "context.h"

namespace igamg {

void k_fill(double *x, double v, long long n, hipStream_t s);
void k_copy_weighted(const double *x, const double *w, double *y, long long n, hipStream_t s);

// setup
void k_stencil_assemble(Context &c, LevelData &L);
void k_stencil_add(const int *rows, const int *slots, const double *vals, int n, double *stencil,
                   int S, hipStream_t s);
void k_invdiag(const double *stencil, int S, int center, const unsigned char *mask, double *invd,
               long long n, hipStream_t s);
void k_load_manufactured(Context &c, LevelData &L, double *out);

// operator: r = mask*(beta f + alpha A u); volume part by sum factorization
void k_iface_apply(Context &c, LevelData &L, const double *u, const double *f, const double *fw,
                   double beta, double alpha, double *r);
void k_vol_apply(Context &c, LevelData &L, const double *u, double *r, double alpha);
void k_glue_sum(LevelData &L, double *y, hipStream_t s);

// smoothers
void k_gs_sweep(Context &c, LevelData &L, bool backward);
void k_scms_interior(Context &c, LevelData &L);
void k_pieces(Context &c, LevelData &L, const double *r, double *u);

// transfer between level l (fine) and l-1 (coarse)
// rc = P^T (w rf); if uc_zero != null it is set to zero (coarse initial guess)
void k_restrict(Context &c, LevelData &F, LevelData &C, const double *rf, double *rc,
                double *uc_zero);
void k_prolong_add(Context &c, LevelData &F, LevelData &C, const double *ec, double *uf);
void k_coarse_solve(Context &c, const double *f0, double *u0);

// compact <-> torn
void k_scatter_compact(const double *xc, long long N, const int *cp, const int *cidx, double *xt,
                       hipStream_t s);
void k_gather_compact(const double *xt, long long N, const int *cp, const int *cidx, int sum,
                      double *xc, hipStream_t s);

// deterministic reductions and PCG updates (device scalars in c.d_scal)
enum Scalar { S_RZ = 0, S_PQ, S_RR, S_RZNEW, S_FF, S_ALPHA, S_BETA, S_TMP, S_COUNT };
void k_dot(Context &c, const double *a, const double *b, long long n, int slot, int mode);
// x += alpha p, r -= alpha q, ||r||^2 (weighted); also zeroes the cycle iterate z
void k_pcg_update_xr(Context &c, long long n);
void k_pcg_update_p(Context &c, long long n);
void k_axpy(double a, const double *x, double *y, long long n, hipStream_t s);

}  // namespace igamg
