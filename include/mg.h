/*
 * mg.h -- C interface of libmg.so, a geometric-multigrid solver for gfx950 (MI355X).
 *
 * Problem (paper: Angersbach, Kuckuk, Koestler, "Towards Code Generation for Octree-Based
 * Multigrid Solvers", Sect. 5, Eq. 1-2): -Laplace(u) = f on the unit square or cube with
 * Dirichlet boundary values, discretised by vertex-centred finite differences
 * (5-point in 2D, 7-point in 3D); optionally -div(k grad u) = f with a positive nodal
 * coefficient k (variable coefficients: Sect. 7), face coefficient (k_i + k_j)/2.
 * Solver: multigrid V(nu1,nu2)-cycles (Sect. 1, Sect. 5) with red-black Gauss-Seidel
 * smoothing, full-weighting restriction, (bi/tri)linear prolongation, coarse operators
 * re-discretised with each level's mesh width (Sect. 4.2) and an exact FP64 solve on the
 * coarsest level; stopping on the residual norm (Sect. 5) used as a relative test.
 *
 * Conventions for every function below:
 *  - Arrays are DEVICE pointers owned by the caller, one value per node of an n^d grid
 *    INCLUDING the boundary nodes, contiguous C order [z][y][x] (x fastest; 2D: [y][x]).
 *    Node (.., i) sits at x_i = i * h, h = 1/(n-1).  Interior nodes have every index in
 *    1..n-2.
 *  - The library never allocates device memory.  mg_setup receives a caller-allocated
 *    device workspace of at least mg_workspace_bytes() bytes, which must stay allocated
 *    and unused by anyone else until mg_destroy.
 *  - All work is enqueued on the stream given to mg_setup (a hipStream_t passed as void*,
 *    NULL = the null stream).  mg_solve and mg_solve_adjoint synchronise that stream once
 *    per cycle to read the residual norm; all other calls return without synchronising.
 *  - One context serves one stream; calls on one context must not overlap.
 *  - No call throws.  Every call returns an mg_status; on failure mg_last_error() gives a
 *    message.  Arguments are validated before any work is enqueued.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

typedef enum {
  MG_OK = 0,
  MG_EINVAL = 1,   /* invalid argument (grid description, pointer, tolerance, level) */
  MG_ENOMEM = 2,   /* workspace smaller than mg_workspace_bytes() */
  MG_EHIP = 3,     /* HIP runtime error; the message carries hipGetErrorString */
  MG_ENOCONV = 4,  /* max_cycles reached above tolerance; u holds the last iterate */
  MG_ENAN = 5,     /* a residual norm was not finite */
  MG_ESTATE = 6    /* call not valid in this state (e.g. coefficients never set) */
} mg_status;

typedef enum {
  MG_F64 = 0,      /* FP64 V-cycles */
  MG_F32_IR = 1    /* FP32 V-cycles as the inner solver of FP64 iterative refinement:
                      fine-grid residual, solution update, norms and the coarsest solve
                      in FP64 */
} mg_precision;

typedef struct {
  int dim;         /* 2 or 3 */
  int n;           /* nodes per side including boundary; (n-1) divisible by 2^(levels-1) */
  int levels;      /* >= 2; level l has n_l = (n-1)/2^l + 1 nodes per side, n_(levels-1) >= 3
                      and at most 1024 interior nodes on the coarsest level */
  int nu1, nu2;    /* pre- and post-smoothing sweeps (>= 0, sum >= 1); 2 and 2 for V(2,2) */
  int max_cycles;  /* >= 1: cap on V-cycles (or refinement steps) per solve */
  int precision;   /* mg_precision */
  int variable;    /* 0: -Laplace(u) = f;  1: -div(k grad u) = f, k set by
                      mg_set_coefficients before the first cycle */
} mg_grid;

/* Checks a grid description without touching the GPU.  MG_OK or MG_EINVAL. */
mg_status mg_validate(const mg_grid* grid);

/* Workspace bytes needed for this grid (0 if the grid is invalid).  Host only. */
size_t mg_workspace_bytes(const mg_grid* grid);

/* Creates a context.  workspace: device memory of `bytes` >= mg_workspace_bytes(grid),
 * owned by the caller.  stream: hipStream_t or NULL.  Enqueues the initialisation of the
 * workspace (zeroed coarse arrays and, for constant coefficients, the factorisation of the
 * coarsest operator) on the stream.  *out is NULL on failure. */
mg_status mg_setup(const mg_grid* grid, void* workspace, size_t bytes, void* stream,
                   mg_ctx** out);

/* Variable-coefficient contexts only.  k: device array of n^d values, all > 0 (not
 * checked).  Copied into the workspace; coarse-level coefficients are formed on the GPU
 * (interior coarse node: exp of the full-weighted log k; boundary coarse node: the
 * coinciding fine value) and the coarsest operator is re-factorised.  k may be freed or
 * changed after the call returns and the stream has passed it. */
mg_status mg_set_coefficients(mg_ctx* ctx, const double* k);

/* One V(nu1,nu2)-cycle on A u = f (MG_F64), or one refinement step (MG_F32_IR:
 * r = f - A u, one FP32 V-cycle for A e = r from e = 0, u += e).  f: n^d values, boundary
 * entries ignored.  u: in/out, interior = current iterate, boundary = Dirichlet data
 * (never written).  Synchronises once in MG_F32_IR mode (to scale the residual). */
mg_status mg_vcycle(mg_ctx* ctx, const double* f, double* u);

/* Solves A u = f: cycles until ||b - A u||_2 <= tol * ||b||_2 over interior nodes, where
 * b is the full right-hand side (f plus the Dirichlet terms; b = f for zero boundary
 * data; if ||b|| = 0 the test is absolute), checked before the first and after every
 * cycle.  u: in/out initial guess, boundary entries = Dirichlet data.  cycles, relres:
 * host pointers (nullable) receiving the number of cycles run and the final relative
 * residual.  tol > 0.  Returns MG_OK, MG_ENOCONV or MG_ENAN. */
mg_status mg_solve(mg_ctx* ctx, const double* f, double* u, double tol, int* cycles,
                   double* relres);

/* Solves the adjoint system A^T lambda = g with zero boundary values.  A is symmetric,
 * so this runs the solver of mg_solve on the same hierarchy (and precision).
 * g: n^d values (boundary entries ignored), e.g. dL/du = u - u_obs.  lambda: in/out
 * initial guess; its boundary entries are set to 0. */
mg_status mg_solve_adjoint(mg_ctx* ctx, const double* g, double* lambda, double tol,
                           int* cycles, double* relres);

/* Gradient of a loss L(u) through the solution of A(k) u = f, by implicit
 * differentiation: dL/df = lambda and dL/dk = -lambda^T (dA/dk) u, i.e. for every node j
 *   dk[j] = -1/(2 h^2) * sum over axis neighbours m of j inside the grid of
 *           (lambda_j - lambda_m) * (u_j - u_m),          lambda taken as 0 on the boundary,
 *   df[j] = lambda_j on interior nodes, 0 on boundary nodes.
 * u: the solution, lambda: the adjoint solution (mg_solve_adjoint), both n^d.  dk, df:
 * n^d outputs, either may be NULL.  One fused pass over the grid. */
mg_status mg_grad(mg_ctx* ctx, const double* u, const double* lambda, double* dk, double* df);

/* ---- single steps of the cycle, on the arrays of one level (parity tests, timing) ----
 * level: 0..levels-1; arrays have n_level^d values; T = double unless the name ends in
 * _f32 (float; then the level operator uses the FP32 copy of the coefficients, available
 * in MG_F32_IR contexts only).  The coefficients of variable contexts are those of the
 * hierarchy built by mg_set_coefficients. */

/* sweeps red-black Gauss-Seidel sweeps (red: (x+y+z) even, first) on A_l u = f, in place.
 * Uses the same kernels as the cycle (temporally blocked on large 3D levels). */
mg_status mg_smooth(mg_ctx* ctx, int level, const double* f, double* u, int sweeps);
mg_status mg_smooth_f32(mg_ctx* ctx, int level, const float* f, float* u, int sweeps);

/* r = f - A_l u on interior nodes, 0 on boundary nodes. */
mg_status mg_residual(mg_ctx* ctx, int level, const double* f, const double* u, double* r);

/* Fused residual and full-weighting restriction: fc (n_(l+1)^d values) receives
 * FW(f - A_l u) on coarse interior nodes and 0 on coarse boundary nodes.  level < levels-1. */
mg_status mg_restrict_residual(mg_ctx* ctx, int level, const double* f, const double* u,
                               double* fc);
mg_status mg_restrict_residual_f32(mg_ctx* ctx, int level, const float* f, const float* u,
                                   float* fc);

/* u (level l) += P ec (level l+1) on interior nodes of level l.  level < levels-1. */
mg_status mg_prolong_correct(mg_ctx* ctx, int level, const double* ec, double* u);
mg_status mg_prolong_correct_f32(mg_ctx* ctx, int level, const float* ec, float* u);

/* Exact solve on the coarsest level: interior of u = A_(levels-1)^-1 f (zero Dirichlet
 * data; boundary of u untouched).  f, u: n_(levels-1)^d values. */
mg_status mg_coarsest_solve(mg_ctx* ctx, const double* f, double* u);

/* *norm2 (host pointer) = sum over interior nodes of (f - A_0 u)^2, reduced on the GPU in a
 * fixed order (bitwise reproducible).  Synchronises the stream. */
mg_status mg_residual_norm2(mg_ctx* ctx, const double* f, const double* u, double* norm2);

/* Kernel-fusion flags (diagnostics and tests), a bitwise OR of:
 *  MG_FUSE_BLOCKED  temporally blocked out-of-place smoother and single-pass streaming
 *                   residual / restriction / norm / refinement kernels on large 3D levels
 *                   (otherwise the per-colour smoother and one launch per step);
 *  MG_FUSE_PROLONG  the coarse-grid correction u += P e applied inside the first
 *                   post-smoothing pass (blocked levels: FP32 passes and the FP64
 *                   constant-coefficient pass) or, on levels served
 *                   by the per-colour kernels, inside the first colour-0 half-sweep, instead
 *                   of a separate pass;
 *  MG_FUSE_ZERO     a zero initial guess read as 0 by the first pre-smoothing pass (or the
 *                   first colour-0 half-sweep, which also writes the other colour's zeros)
 *                   instead of being written first;
 *  MG_FUSE_TAIL     all levels with at most 4096 interior nodes in one launch;
 *  MG_FUSE_RESTRICT on such large 3D levels, the residual and its full-weighting restriction
 *                   computed inside the pre-smoothing pass (constant coefficient, FP32
 *                   and FP64) instead of a separate pass;
 *  MG_FUSE_REFINE   in an MG_F32_IR solve with a large 3D finest level, a constant
 *                   coefficient and nu2 = 2 (with MG_FUSE_PROLONG), the refinement step
 *                   (u += s e, the FP64 residual, its norm and the next FP32 right-hand side)
 *                   performed inside the FP32 cycle's last post-smoothing pass instead of a
 *                   separate pass, so the correction is never stored.
 * Default MG_FUSE_ALL.  Clearing MG_FUSE_PROLONG, MG_FUSE_ZERO, MG_FUSE_TAIL or
 * MG_FUSE_RESTRICT leaves every result bitwise unchanged; without MG_FUSE_BLOCKED smoothing results are unchanged but
 * residual sums are accumulated in another order; MG_FUSE_REFINE leaves the iterate bitwise
 * unchanged and sums the residual norm in another order.  EINVAL for bits outside
 * MG_FUSE_ALL. */
enum {
  MG_FUSE_BLOCKED = 1,
  MG_FUSE_PROLONG = 2,
  MG_FUSE_ZERO = 4,
  MG_FUSE_TAIL = 8,
  MG_FUSE_RESTRICT = 16,
  MG_FUSE_REFINE = 32,
  MG_FUSE_ALL = 63
};
mg_status mg_set_fusion(mg_ctx* ctx, int flags);

/* ---- allocation-free solve ----
 * For callers that cannot allocate device memory or set up a context at the time of the
 * solve (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): mg_solve on a context built for this one call, whose workspace is a static
 * device array of MG_NOALLOC_MAX_BYTES inside the library instead of a caller-allocated
 * one.  The call makes no device or host allocation of any kind (no hipMalloc, hipFree,
 * pinned memory or heap); FP32-refined solves read their norms synchronously.
 *   grid:   as for mg_setup; mg_workspace_bytes(grid) must not exceed MG_NOALLOC_MAX_BYTES
 *           (else MG_ENOMEM, before any HIP call).  32 MiB holds e.g. a 129^3 FP64 or a
 *           65^3 FP32-refined variable-coefficient grid.
 *   k:      variable-coefficient grids: device array of n^d values > 0; NULL otherwise.
 *   f, u, tol, cycles, relres: as for mg_solve (u in/out, boundary = Dirichlet data).
 *   stream: hipStream_t (or NULL) of the current HIP device, which must hold k, f and u.
 * Results are those of mg_setup + mg_set_coefficients + mg_solve with the same arguments
 * (the same kernels in the same order).  The static array exists once per GPU, from the
 * first call on that GPU until the process ends, and keeps the last call's contents; each
 * call re-initialises the part it uses.  Calls that overlap on one GPU (other threads,
 * other streams) race on it.  The stream is synchronised once per cycle, as by mg_solve.
 * Errors are reported by mg_last_error(NULL). */
#define MG_NOALLOC_MAX_BYTES ((size_t)32 << 20)
mg_status mg_solve_noalloc(const mg_grid* grid, const double* k, const double* f, double* u,
                           double tol, void* stream, int* cycles, double* relres);

/* Message for the last failing call on ctx, or for the last failing mg_setup /
 * mg_validate / mg_solve_noalloc call of this thread when ctx is NULL.  Never NULL. */
const char* mg_last_error(const mg_ctx* ctx);

/* Releases the context (not the workspace).  Does not synchronise. */
void mg_destroy(mg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
