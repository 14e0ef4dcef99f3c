/*
 * mg_blocks.h -- C ABI of the 2:1 refined block layout in libmg.so: the ghost-layer exchange
 * between blocks of different refinement levels (Angersbach, Kuckuk, Koestler, arXiv
 * 2403.08063, Sect. 3: same-level copies, fine-to-coarse (F2C) linear interpolation,
 * coarse-to-fine (C2F) extrapolation of constant, linear or quadratic order) on the layout
 * of Sect. 5, with a damped-Jacobi solver of the composite cell-centred system (Eq. 1-2).
 *
 * Layout: [0,1]^3 split into 4^3 level-2 blocks of width 1/4, the central 2^3 of them
 * refined into 8 level-3 blocks of width 1/8 each: 56 + 64 = 120 blocks (the counts of
 * Sect. 5).  Every block holds B^3 cells (B even, 4 <= B <= 256; its own h = width / B),
 * stored as (B+2)^3 doubles with a one-cell ghost layer, C order [z][y][x]; the blocks are
 * concatenated: first the level-2 blocks in (z, y, x) order of their block index, then the
 * level-3 blocks in (z, y, x) order of their level-3 block index.
 *
 * Ghost layer of a face:
 *  - on the domain boundary: the Dirichlet value at the ghost cell's own centre (half a cell
 *    outside the domain), written by the caller and never by the library; the operator
 *    reads it like any other neighbour (the reading under which Table 1's errors, Sect. 5,
 *    are reproduced);
 *  - towards a block of the same level: a copy of the neighbour's adjacent inner cell;
 *  - of a level-2 block towards refined blocks (F2C): the mean of the 8 level-3 inner cells
 *    the coarse ghost cell covers (weights 0.125);
 *  - of a level-3 block towards a level-2 block (C2F): from the coarse block's inner cells
 *    only, by Lagrange bases along each axis (order+1 of them): along the normal the coarse
 *    cell at the interface and the next ones away from it, extrapolated to the fine ghost
 *    centre a quarter coarse cell towards the face; along each tangential axis the cell and
 *    its neighbours, evaluated at -1/4 or +1/4 coarse cell, with a base that would fall into
 *    the coarse block's ghost region replaced by the inner cell at -2 o (Sect. 3's
 *    remapping; order 1 takes the cell and its downwind neighbour -o for both fine cells, or
 *    the upwind one at the block's lower edge; order 0 copies the coarse cell).  With the
 *    boundary treatment above these schemes reproduce Table 1's printed errors (Sect. 5).
 * The operator of every block is the 7-point finite-volume one, (A u)_i = h^-2 sum over
 * the six neighbours of (u_i - u_nb) with that block's h, every ghost neighbour read as
 * stored; damped Jacobi: u <- u + omega (h^2/6) (f - A u).
 *
 * Multigrid (Sect. 5: V(3,3)-cycles, damped Jacobi with omega = 0.8 as smoother and as
 * coarsest-level solver, coarser levels until a block holds 4^3 cells): level l keeps the
 * 120-block layout with B/2^l cells per block and its own h per block, rediscretised and
 * exchanged by the same rules.  The paper leaves the transfers open; here
 *  - restriction: the mean of the 8 child residuals of a coarse cell (children in z, y, x
 *    order), within the block;
 *  - prolongation: a fine cell lies a quarter coarse cell from its parent P along every axis,
 *    towards +1 where its 0-based index is odd and -1 where even; its correction is
 *    (e_P + e_x + e_y + e_z) / 4 with e_a the parent's face neighbour on that side along axis a
 *    (the barycentric weights of the fine centre in the tetrahedron of those four centres:
 *    exact for linear functions, and reading only face ghosts, which the exchange fills);
 *    a neighbour across the domain boundary counts as -e_P (zero correction on the face);
 *  - coarse problems: the correction with zero Dirichlet data on the boundary face (on levels
 *    l >= 1 a domain-boundary ghost enters the operator as 2 g - u_i with its stored g = 0,
 *    where the finest level reads the Dirichlet value at the ghost centre as stored; with the
 *    zero at the coarse ghost centres the V(3,3) factor would grow with the block size) and
 *    initial guess 0.
 * Coarse-level arrays live in the workspace; the finest level's are the caller's.
 *
 * Conventions as in mg.h: device pointers owned by the caller; a caller-provided workspace
 * (mgblk_workspace_bytes, 256-byte aligned), no allocation by the library; all work on the
 * stream given to mgblk_setup; mgblk_residual_norm2 and mgblk_solve synchronise to read norms.
 */
#ifndef MG_BLOCKS_H
#define MG_BLOCKS_H

#include <stddef.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgblk_ctx mgblk_ctx;

typedef struct {
  int B;             /* cells per block and axis: even, 4 <= B <= 256 */
  int order;         /* C2F extrapolation order: 0, 1 or 2 (the paper's quadratic scheme) */
  double omega;      /* Jacobi damping, 0 < omega < 2 (0.8) */
  int levels;        /* multigrid levels B, B/2, ...: 0 = halve while the half is even and
                        >= 4 (down to 4^3 cells per block for B = 4 * 2^k); otherwise every
                        level but the last must have a size divisible by 4 */
  int nu1, nu2;      /* pre- and post-smoothing sweeps per level (3, 3) */
  int coarse_iters;  /* Jacobi iterations on the coarsest level (256) */
  int max_cycles;    /* mgblk_mg_solve: cycle limit (35) */
} mgblk_grid;

/* Number of blocks of the layout (120). */
int mgblk_block_count(void);

/* Bytes of device workspace (host-only); 0 if the description is invalid. */
size_t mgblk_workspace_bytes(const mgblk_grid* grid);

/* Validates, lays out the workspace and uploads the layout's face table on `stream`. */
mg_status mgblk_setup(const mgblk_grid* grid, void* workspace, size_t bytes, void* stream,
                      mgblk_ctx** out);

void mgblk_destroy(mgblk_ctx* ctx);

const char* mgblk_last_error(const mgblk_ctx* ctx);

/* Fills every ghost cell not on the domain boundary of the concatenated block arrays u from
 * the neighbouring blocks' inner cells (Sect. 3's exchange). */
mg_status mgblk_fill(mgblk_ctx* ctx, double* u);

/* `sweeps` damped Jacobi sweeps of the composite system, each preceded by a ghost fill; u in
 * place (its domain-boundary ghosts are the Dirichlet data).  Same as mgblk_smooth(ctx, 0, ...). */
mg_status mgblk_jacobi(mgblk_ctx* ctx, const double* f, double* u, int sweeps);

/* Number of multigrid levels of the context (level l has B >> l cells per block); 0 for NULL. */
int mgblk_levels(const mgblk_ctx* ctx);

/* `sweeps` damped Jacobi sweeps on arrays of level `level` (block size B >> level), each
 * preceded by a ghost fill; u in place, its domain-boundary ghosts being the Dirichlet data
 * (level 0; levels >= 1 use the correction levels' operator, see above). */
mg_status mgblk_smooth(mgblk_ctx* ctx, int level, const double* f, double* u, int sweeps);

/* Fills u's interface ghosts (level `level`), then fc (level `level`+1) = the mean of the 8
 * child residuals f - A u (the operator of level `level`) of every coarse inner cell.  fc's
 * ghost cells are not written. */
mg_status mgblk_restrict_residual(mgblk_ctx* ctx, int level, const double* f, double* u,
                                  double* fc);

/* Fills the interface ghosts of the level-(`level`+1) correction ec (in place; its domain-
 * boundary ghosts are not read), then u (level `level`) += P ec on the inner cells. */
mg_status mgblk_prolong_correct(mgblk_ctx* ctx, int level, double* ec, double* u);

/* One V(nu1, nu2)-cycle on the finest level, in place on u. */
mg_status mgblk_vcycle(mgblk_ctx* ctx, const double* f, double* u);

/* Fills u's ghosts, then *out = sum over all inner cells of (f - A u)^2. */
mg_status mgblk_residual_norm2(mgblk_ctx* ctx, const double* f, double* u, double* out);

/* Jacobi sweeps until the L2 residual norm is <= tol (checked every check_every sweeps) or
 * max_sweeps ran; *sweeps and *resnorm (optional) receive the count and the last norm.
 * MG_ENOCONV if the tolerance was not reached. */
mg_status mgblk_solve(mgblk_ctx* ctx, const double* f, double* u, double tol, int max_sweeps,
                      int check_every, int* sweeps, double* resnorm);

/* V-cycles until the L2 residual norm (over all inner cells, unweighted) is <= tol or
 * max_cycles cycles ran (Sect. 5: 1e-16 or 35); synchronises once per cycle to read the norm.
 * *cycles and *resnorm (optional) receive the count and the last norm.  MG_ENOCONV if the
 * tolerance was not reached (u holds the last iterate). */
mg_status mgblk_mg_solve(mgblk_ctx* ctx, const double* f, double* u, double tol, int* cycles,
                         double* resnorm);

#ifdef __cplusplus
}
#endif

#endif /* MG_BLOCKS_H */
