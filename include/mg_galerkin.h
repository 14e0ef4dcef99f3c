/*
 * mg_galerkin.h -- C ABI of Galerkin coarsening for the variable-coefficient operator in
 * libmg.so: V(nu1, nu2)-cycles for -div(k grad u) = f on a vertex-centred n^3 grid whose
 * coarse operators are the Galerkin products A_{l+1} = R A_l P (P: trilinear interpolation of
 * coarse corrections, R = P^T / 8: full weighting) instead of rediscretisations.  The paper
 * leaves variable coefficients as future work (Angersbach, Kuckuk, Koestler, arXiv
 * 2403.08063, Sect. 7); the fine operator is the one of mg.h: face coefficients
 * k_f = (k_i + k_nb)/2, (A u)_i = (1/h^2) sum_nb k_f (u_i - u_nb), h = 1/(n-1).
 *
 * Levels: n_l = (n-1)/2^l + 1 down to n_{L-1} = 3 (one interior node, solved exactly).  Level 0
 * keeps the 7-point operator and red-black Gauss-Seidel (red = even index sum, first); every
 * coarser level stores its 27-point stencil and is smoothed by Gauss-Seidel in eight colours
 * (colour 4 (z%2) + 2 (y%2) + x%2, in that order: nodes of one colour never couple).  Coarse
 * problems have zero Dirichlet data and start from 0.
 *
 * Stencil layout (mggal_stencil): 27 arrays of n_l^3 doubles, C order [z][y][x]; array
 * o = 9 (dz+1) + 3 (dy+1) + (dx+1) holds the coupling of node i to node i + (dx, dy, dz) at
 * interior nodes (0 where the neighbour is a boundary node, and on boundary nodes).  Setup
 * builds them on the GPU by probing: for each of the 27 residue classes c of coarse nodes mod
 * 3 per axis, P applied to the comb of class c, then A_l and R, gives at every coarse node the
 * coupling to its one neighbour of class c.
 *
 * Conventions as in mg.h: device pointers owned by the caller, C order, n^3 values including
 * the boundary (u's boundary is the Dirichlet data); a caller-provided workspace
 * (mggal_workspace_bytes, 256-byte aligned), no allocation by the library; all work on the
 * stream given to mggal_setup; mggal_solve synchronises once per cycle to read the norm.
 */
#ifndef MG_GALERKIN_H
#define MG_GALERKIN_H

#include <stddef.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mggal_ctx mggal_ctx;

typedef struct {
  int n;           /* nodes per side: 2^m + 1, 5 <= n <= 1025 */
  int levels;      /* must reach n_{levels-1} = 3 */
  int nu1, nu2;    /* sweeps per level (2, 2) */
  int max_cycles;  /* mggal_solve: cycle limit */
  int coarse_f32;  /* 1: the cycle's 27-point kernels read an FP32 copy of the coarse stencils
                      (built in FP64; half the coefficient traffic; the coarse levels only
                      compute corrections, the fine level and the stopping test stay FP64) */
} mggal_grid;

/* Bytes of device workspace (host-only); 0 if the description is invalid. */
size_t mggal_workspace_bytes(const mggal_grid* grid);

/* Validates, copies k (n^3 node values > 0, device) into the workspace and builds the
 * Galerkin hierarchy on `stream` (synchronises once at the end). */
mg_status mggal_setup(const mggal_grid* grid, const double* k, void* workspace, size_t bytes,
                      void* stream, mggal_ctx** out);

void mggal_destroy(mggal_ctx* ctx);

const char* mggal_last_error(const mggal_ctx* ctx);

/* Copies the 27-point stencil of level `level` (1 <= level < levels) into out (27 n_l^3
 * doubles, device), in the layout above. */
mg_status mggal_stencil(mggal_ctx* ctx, int level, double* out);

/* One V(nu1, nu2)-cycle, in place on u. */
mg_status mggal_vcycle(mggal_ctx* ctx, const double* f, double* u);

/* V-cycles until ||f - A u||_2 / ||f - A u_B||_2 <= tol over interior nodes (u_B: u with its
 * interior set to 0) or max_cycles ran; *cycles and *relres (optional) receive the count and
 * the last relative residual.  MG_ENOCONV if the tolerance was not reached, MG_ENAN if the
 * norm is not finite. */
mg_status mggal_solve(mggal_ctx* ctx, const double* f, double* u, double tol, int* cycles,
                      double* relres);

#ifdef __cplusplus
}
#endif

#endif /* MG_GALERKIN_H */
