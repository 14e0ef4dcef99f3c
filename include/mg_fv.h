/*
 * mg_fv.h -- C ABI of the cell-centred finite-volume multigrid solver in libmg.so: the
 * paper's own benchmark solver (Angersbach, Kuckuk, Koestler, arXiv 2403.08063, Sect. 5 and
 * Sect. 6) on a uniform grid.
 *
 * Problem (Sect. 5, Eq. 1-2): -Laplace(u) = f on [0,1]^3 with Dirichlet data g, discretised
 * with the cell-centred finite-volume method; V(nu1, nu2) multigrid with a damped Jacobi
 * smoother (omega = 0.8 in the paper, V(3,3)), damped Jacobi also as the coarsest-grid solver
 * (a fixed number of iterations: 256 in Sect. 6), stopped when the L2 residual norm falls
 * below a threshold or after a maximum number of cycles (1e-16 and 35 in Sect. 5).
 *
 * Conventions (shared with mg.h: statuses, device pointers, caller's stream):
 *  - a level of N cells per side is an array of (N+2)^3 doubles, C order [z][y][x]; cell i
 *    in 1..N per axis has its centre at (i - 1/2)/N; the ghost layer (index 0 and N+1)
 *    holds the Dirichlet value at the centre of the adjacent boundary face, and a ghost
 *    neighbour enters the 7-point operator as 2 g - u_i (the flux (u_i - g)/(h/2));
 *  - (A u)_i = (1/h^2) sum over the six face neighbours of (u_i - v_nb); level l has
 *    N >> l cells per side and h = 2^l / N;
 *  - damped Jacobi: u <- u + omega (h^2/6) (f - A u), out of place inside the library;
 *  - restriction: mean of the 8 child cells; prolongation: trilinear interpolation of the
 *    coarse cell centres with the homogeneous ghost extension -e (zero on the faces);
 *  - every array pointer is a device pointer owned by the caller; f is read only; the
 *    ghost layer of u is read, never written; the library calls no hipMalloc: the
 *    workspace (mgfv_workspace_bytes) is the caller's, 256-byte aligned;
 *  - all work goes on the stream given to mgfv_setup; mgfv_solve synchronises once per
 *    cycle to read the residual norm; the other calls do not synchronise;
 *  - errors: MG_EINVAL (bad size or argument), MG_ENOMEM (workspace too small), MG_EHIP
 *    (a HIP error, its text in mgfv_last_error), MG_ENOCONV (cycle limit reached before
 *    the tolerance; u holds the last iterate), MG_ENAN (non-finite residual norm).
 */
#ifndef MG_FV_H
#define MG_FV_H

#include <stddef.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgfv_ctx mgfv_ctx;

typedef struct {
  int N;             /* cells per side on the finest level: a power of two, 4 <= N <= 2048 */
  int levels;        /* levels, N >> (levels-1) >= 2 cells on the coarsest (the paper: 4) */
  int nu1, nu2;      /* Jacobi sweeps before / after the coarse-grid correction (3, 3) */
  int coarse_iters;  /* Jacobi iterations on the coarsest level, from 0 (256) */
  double omega;      /* Jacobi damping, 0 < omega < 2 (0.8) */
  int max_cycles;    /* mgfv_solve: cycle limit (35) */
} mgfv_grid;

/* Bytes of device workspace for this grid (host-only, no HIP call); 0 if the description is
 * invalid. */
size_t mgfv_workspace_bytes(const mgfv_grid* grid);

/* Validates the grid, lays out the workspace and enqueues its clearing on `stream` (a
 * hipStream_t; NULL = the default stream).  *out receives a context owned by the caller,
 * released with mgfv_destroy. */
mg_status mgfv_setup(const mgfv_grid* grid, void* workspace, size_t bytes, void* stream,
                     mgfv_ctx** out);

void mgfv_destroy(mgfv_ctx* ctx);

/* Message of the last error on ctx (a static text when ctx is NULL). */
const char* mgfv_last_error(const mgfv_ctx* ctx);

/* `sweeps` damped Jacobi sweeps on level `level` (Sect. 5's smoother): f and u are arrays of
 * that level; u is updated in place (the ghost layer is its Dirichlet data). */
mg_status mgfv_jacobi(mgfv_ctx* ctx, int level, const double* f, double* u, int sweeps);

/* r = f - A u on the cells of level `level`, 0 on r's ghost layer. */
mg_status mgfv_residual(mgfv_ctx* ctx, int level, const double* f, const double* u, double* r);

/* fc = restriction of f - A u of level `level` to level `level`+1 (mean of the 8 children);
 * fc's ghost layer is set to 0. */
mg_status mgfv_restrict_residual(mgfv_ctx* ctx, int level, const double* f, const double* u,
                                 double* fc);

/* u += P ec: trilinear prolongation of the level-(`level`+1) correction ec (its ghost layer
 * is not read: the homogeneous extension is used) onto the cells of level `level`. */
mg_status mgfv_prolong_correct(mgfv_ctx* ctx, int level, const double* ec, double* u);

/* The coarsest-grid solver: coarse_iters Jacobi iterations on the coarsest level's arrays,
 * starting from the u given (the V-cycle passes 0). */
mg_status mgfv_coarse_solve(mgfv_ctx* ctx, const double* f, double* u);

/* *out = sum over the finest cells of (f - A u)^2 (the square of the L2 residual norm);
 * synchronises the stream. */
mg_status mgfv_residual_norm2(mgfv_ctx* ctx, const double* f, const double* u, double* out);

/* One V(nu1, nu2)-cycle on the finest level, in place on u. */
mg_status mgfv_vcycle(mgfv_ctx* ctx, const double* f, double* u);

/* V-cycles until the L2 residual norm is <= tol or max_cycles cycles ran (Sect. 5).
 * *cycles and *resnorm (both optional) receive the count and the final norm. */
mg_status mgfv_solve(mgfv_ctx* ctx, const double* f, double* u, double tol, int* cycles,
                     double* resnorm);

#ifdef __cplusplus
}
#endif

#endif /* MG_FV_H */
