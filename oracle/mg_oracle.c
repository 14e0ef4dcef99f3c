/*
 * mg_oracle.c -- plain, slow, obviously-correct CPU oracle for the geometric-multigrid
 * V-cycle path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library.  The GPU library neither links nor calls it, and it
 * includes no header of the GPU library; the two share no code.
 *
 * Paper: R. Angersbach, S. Kuckuk, H. Koestler, "Towards Code Generation for Octree-Based
 * Multigrid Solvers" (arXiv 2403.08063).  What is computed, and where it comes from:
 *   - the model problem -Laplace(u) = f on [0,1]^d with Dirichlet data in the boundary
 *     nodes (Sect. 5, Eq. 1 and 2), generalised to -div(k grad u) = f (variable
 *     coefficients: Sect. 7);
 *   - a geometric multigrid V(nu1,nu2)-cycle (Sect. 1; V(3,3) in Sect. 5), with operators
 *     re-discretised on every level from that level's mesh width (Sect. 4.2, 4.3);
 *   - a residual-norm stopping test (Sect. 5), used as a relative test;
 *   - FP32 inner V-cycles inside FP64 iterative refinement;
 *   - the gradient of L = 0.5 ||u - u_obs||^2 with respect to k and f, from the adjoint
 *     of the discrete system.
 * The paper gives no smoother other than damped Jacobi and no transfer operators.  The
 * readings taken here, each restated at the function that uses it:
 *   vertex-centred finite differences with n = 2^m + 1 nodes per side; red-black
 *   Gauss-Seidel (omega = 1, red = (x+y+z) even first, in pre- and post-smoothing);
 *   full-weighting restriction; (bi/tri)linear prolongation; re-discretised (not
 *   Galerkin) coarse operators; arithmetic-mean face coefficients; coarse k as exp of the
 *   full-weighted log k (injection on the boundary); an exact dense Cholesky solve on the
 *   coarsest level; relative residual ||b - A u||_2 / ||b||_2 over interior nodes.
 *
 * Parity pins for every function are in the test-suite (closed-form discrete solutions,
 * dense direct solves, exactness on polynomials, transfer-operator identities,
 * smoother fixed points, convergence-factor bands and brute-force finite differences).
 *
 * Parallelism: OpenMP over z inside one colour or one output array only, so results are
 * identical at any thread count.  Norms are summed per plane and then serially.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define IDX(n, z, y, x) ((((size_t)(z)) * (size_t)(n) + (size_t)(y)) * (size_t)(n) + (size_t)(x))
#define MAXL 16

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_ENOCONV = 4, OR_ENAN = 5 };

static size_t node_count(int dim, int n)
{
  return dim == 3 ? (size_t)n * n * n : (size_t)n * n;
}

/* Index offsets of the 2d axis neighbours, in the fixed order -x, +x, -y, +y, -z, +z. */
static void neighbour_offsets(int n, ptrdiff_t off[6])
{
  const ptrdiff_t sy = n, sz = (ptrdiff_t)n * n;
  off[0] = -1; off[1] = 1; off[2] = -sy; off[3] = sy; off[4] = -sz; off[5] = sz;
}

/* Linear interpolation along one axis: fine index i maps to coarse index i/2 with weight
 * 1 if i is even, else to (i-1)/2 and (i+1)/2 with weight 1/2 each. */
static int linear_weights(int i, int c[2], double w[2])
{
  if ((i & 1) == 0) { c[0] = i / 2; w[0] = 1.0; return 1; }
  c[0] = (i - 1) / 2; c[1] = (i + 1) / 2; w[0] = w[1] = 0.5;
  return 2;
}

#define REAL double
#define FN(name) name##_f64
#include "level_ops.inc"
#undef REAL
#undef FN
#define REAL float
#define FN(name) name##_f32
#include "level_ops.inc"
#undef REAL
#undef FN

/* Sum of squares of v over interior nodes; per-plane partial sums added serially. */
static double interior_norm2(int dim, int n, const double* v)
{
  const int z0 = dim == 3 ? 1 : 0, z1 = dim == 3 ? n - 2 : 0;
  double* part = (double*)calloc((size_t)n, sizeof(double));
  if (!part) return NAN;
#pragma omp parallel for schedule(static)
  for (int z = z0; z <= z1; ++z) {
    double s = 0;
    for (int y = 1; y <= n - 2; ++y)
      for (int x = 1; x <= n - 2; ++x) {
        const double a = v[IDX(n, z, y, x)];
        s += a * a;
      }
    part[z] = s;
  }
  double s = 0;
  for (int z = z0; z <= z1; ++z) s += part[z];
  free(part);
  return s;
}

/* ------------------------------------------------------------------ coefficients */

/* Coarse coefficient from fine coefficient: at interior coarse nodes the exponential of
 * the full-weighted logarithm (a geometric mean with full-weighting weights), at coarse
 * boundary nodes the fine value at the coinciding node (injection). */
void or_coarsen_k(int dim, int nf, const double* k, double* kc)
{
  const int nc = (nf - 1) / 2 + 1;
  static const double w[3] = {0.25, 0.5, 0.25};
  const int Zn = dim == 3 ? nc : 1;
#pragma omp parallel for schedule(static)
  for (int Z = 0; Z < Zn; ++Z)
    for (int Y = 0; Y < nc; ++Y)
      for (int X = 0; X < nc; ++X) {
        const int interior = X >= 1 && X <= nc - 2 && Y >= 1 && Y <= nc - 2 &&
                             (dim == 2 || (Z >= 1 && Z <= nc - 2));
        const int fz = dim == 3 ? 2 * Z : 0;
        if (!interior) {
          kc[IDX(nc, Z, Y, X)] = k[IDX(nf, fz, 2 * Y, 2 * X)];
          continue;
        }
        double s = 0;
        for (int oz = (dim == 3 ? -1 : 0); oz <= (dim == 3 ? 1 : 0); ++oz)
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox)
              s += w[ox + 1] * w[oy + 1] * (dim == 3 ? w[oz + 1] : 1.0) *
                   log(k[IDX(nf, fz + oz, 2 * Y + oy, 2 * X + ox)]);
        kc[IDX(nc, Z, Y, X)] = exp(s);
      }
}

/* ------------------------------------------------------------------ coarsest solve */

/* Exact solve of the interior system on one (small) level: the matrix of A over the
 * interior unknowns in lexicographic order is assembled densely, factored A = L L^T by
 * plain Cholesky, and the system A u_int = f_int + (boundary terms) is solved by forward
 * and back substitution.  The boundary nodes of u are the Dirichlet data and are left
 * unchanged.  Returns OR_ENOMEM or OR_EINVAL (matrix not positive definite) on failure. */
static int coarsest_solve(int dim, int n, double h, const double* k, const double* f,
                          double* u)
{
  const int m1 = n - 2;
  const int m = dim == 3 ? m1 * m1 * m1 : m1 * m1;
  double* A = (double*)calloc((size_t)m * m, sizeof(double));
  double* b = (double*)calloc((size_t)m, sizeof(double));
  if (!A || !b) { free(A); free(b); return OR_ENOMEM; }
  ptrdiff_t off[6];
  neighbour_offsets(n, off);
  const double ih2 = 1.0 / (h * h);
  const int z0 = dim == 3 ? 1 : 0, z1 = dim == 3 ? n - 2 : 0;
  int row = 0;
  for (int z = z0; z <= z1; ++z)
    for (int y = 1; y <= n - 2; ++y)
      for (int x = 1; x <= n - 2; ++x, ++row) {
        const size_t i = IDX(n, z, y, x);
        const int nz[6] = {z, z, z, z, z - 1, z + 1};
        const int ny[6] = {y, y, y - 1, y + 1, y, y};
        const int nx[6] = {x - 1, x + 1, x, x, x, x};
        b[row] = f[i];
        for (int j = 0; j < 2 * dim; ++j) {
          const double c = k ? 0.5 * (k[i] + k[i + off[j]]) : 1.0;
          A[(size_t)row * m + row] += c * ih2;
          const int nb_interior = nx[j] >= 1 && nx[j] <= n - 2 && ny[j] >= 1 && ny[j] <= n - 2 &&
                                  (dim == 2 || (nz[j] >= 1 && nz[j] <= n - 2));
          if (nb_interior) {
            const int col = dim == 3 ? ((nz[j] - 1) * m1 + (ny[j] - 1)) * m1 + (nx[j] - 1)
                                     : (ny[j] - 1) * m1 + (nx[j] - 1);
            A[(size_t)row * m + col] -= c * ih2;
          } else {
            b[row] += c * ih2 * u[i + off[j]];
          }
        }
      }
  /* Cholesky: lower triangle of A overwritten by L. */
  for (int j = 0; j < m; ++j) {
    double d = A[(size_t)j * m + j];
    for (int p = 0; p < j; ++p) d -= A[(size_t)j * m + p] * A[(size_t)j * m + p];
    if (!(d > 0)) { free(A); free(b); return OR_EINVAL; }
    d = sqrt(d);
    A[(size_t)j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = A[(size_t)i * m + j];
      for (int p = 0; p < j; ++p) s -= A[(size_t)i * m + p] * A[(size_t)j * m + p];
      A[(size_t)i * m + j] = s / d;
    }
  }
  /* L y = b, then L^T x = y. */
  for (int i = 0; i < m; ++i) {
    double s = b[i];
    for (int p = 0; p < i; ++p) s -= A[(size_t)i * m + p] * b[p];
    b[i] = s / A[(size_t)i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = b[i];
    for (int p = i + 1; p < m; ++p) s -= A[(size_t)p * m + i] * b[p];
    b[i] = s / A[(size_t)i * m + i];
  }
  row = 0;
  for (int z = z0; z <= z1; ++z)
    for (int y = 1; y <= n - 2; ++y)
      for (int x = 1; x <= n - 2; ++x, ++row) u[IDX(n, z, y, x)] = b[row];
  free(A);
  free(b);
  return OR_OK;
}

/* ------------------------------------------------------------------ hierarchy */

typedef struct {
  int dim, L, nu1, nu2;
  int n[MAXL];
  double h[MAXL];
  double *u[MAXL], *f[MAXL], *r[MAXL], *k[MAXL];       /* FP64 cycle data, level 0 u/f: caller's */
  float *u32[MAXL], *f32[MAXL], *r32[MAXL], *k32[MAXL]; /* FP32 inner-cycle data */
  int owns_k0;
} hierarchy;

static void hier_free(hierarchy* H)
{
  for (int l = 0; l < MAXL; ++l) {
    if (l > 0) { free(H->u[l]); free(H->f[l]); }
    if (l > 0 || H->owns_k0) free(H->k[l]);
    free(H->r[l]);
    free(H->u32[l]); free(H->f32[l]); free(H->r32[l]); free(H->k32[l]);
  }
  memset(H, 0, sizeof(*H));
}

/* Level l has n_l = (n-1)/2^l + 1 nodes per side and mesh width h_l = 2^l/(n-1): the
 * operator of every level is the same finite-difference stencil re-discretised with that
 * level's width.  Returns OR_EINVAL unless (n-1) is divisible by 2^(L-1), the coarsest
 * level keeps at least one interior node, and 2 <= L <= MAXL. */
static int hier_init(hierarchy* H, int dim, int n, int L, int nu1, int nu2, const double* k,
                     int want_f32)
{
  memset(H, 0, sizeof(*H));
  if ((dim != 2 && dim != 3) || L < 2 || L > MAXL || n < 3) return OR_EINVAL;
  if ((n - 1) % (1 << (L - 1)) != 0 || (n - 1) / (1 << (L - 1)) < 2) return OR_EINVAL;
  H->dim = dim; H->L = L; H->nu1 = nu1; H->nu2 = nu2;
  for (int l = 0; l < L; ++l) {
    H->n[l] = (n - 1) / (1 << l) + 1;
    H->h[l] = (double)(1 << l) / (double)(n - 1);
    const size_t N = node_count(dim, H->n[l]);
    H->r[l] = (double*)calloc(N, sizeof(double));
    if (l > 0) {
      H->u[l] = (double*)calloc(N, sizeof(double));
      H->f[l] = (double*)calloc(N, sizeof(double));
    }
    if (!H->r[l] || (l > 0 && (!H->u[l] || !H->f[l]))) { hier_free(H); return OR_ENOMEM; }
    if (want_f32) {
      H->u32[l] = (float*)calloc(N, sizeof(float));
      H->f32[l] = (float*)calloc(N, sizeof(float));
      H->r32[l] = (float*)calloc(N, sizeof(float));
      if (!H->u32[l] || !H->f32[l] || !H->r32[l]) { hier_free(H); return OR_ENOMEM; }
    }
  }
  if (k) {
    H->k[0] = (double*)k; /* caller's array, not owned */
    for (int l = 1; l < L; ++l) {
      H->k[l] = (double*)malloc(node_count(dim, H->n[l]) * sizeof(double));
      if (!H->k[l]) { hier_free(H); return OR_ENOMEM; }
      or_coarsen_k(dim, H->n[l - 1], H->k[l - 1], H->k[l]);
    }
    if (want_f32)
      for (int l = 0; l < L; ++l) {
        const size_t N = node_count(dim, H->n[l]);
        H->k32[l] = (float*)malloc(N * sizeof(float));
        if (!H->k32[l]) { hier_free(H); return OR_ENOMEM; }
        for (size_t i = 0; i < N; ++i) H->k32[l][i] = (float)H->k[l][i];
      }
  }
  return OR_OK;
}

/* One FP64 V(nu1,nu2)-cycle on level l for A_l u_l = f_l. */
static int vcycle_f64(hierarchy* H, int l)
{
  const int dim = H->dim, n = H->n[l];
  const double h = H->h[l];
  if (l == H->L - 1) return coarsest_solve(dim, n, h, H->k[l], H->f[l], H->u[l]);
  for (int s = 0; s < H->nu1; ++s) {
    rbgs_half_f64(dim, n, h, H->k[l], H->f[l], H->u[l], 0);
    rbgs_half_f64(dim, n, h, H->k[l], H->f[l], H->u[l], 1);
  }
  residual_f64(dim, n, h, H->k[l], H->f[l], H->u[l], H->r[l]);
  restrict_fw_f64(dim, n, H->r[l], H->f[l + 1]);
  memset(H->u[l + 1], 0, node_count(dim, H->n[l + 1]) * sizeof(double));
  const int st = vcycle_f64(H, l + 1);
  if (st) return st;
  prolong_add_f64(dim, H->n[l + 1], H->u[l + 1], H->u[l]);
  for (int s = 0; s < H->nu2; ++s) {
    rbgs_half_f64(dim, n, h, H->k[l], H->f[l], H->u[l], 0);
    rbgs_half_f64(dim, n, h, H->k[l], H->f[l], H->u[l], 1);
  }
  return OR_OK;
}

/* One FP32 V(nu1,nu2)-cycle on level l for A_l e_l = r_l with zero initial guess already
 * in u32[l]; every operation in float except the coarsest solve, which is done in double
 * on the values cast up and cast back down. */
static int vcycle_f32(hierarchy* H, int l)
{
  const int dim = H->dim, n = H->n[l];
  const float h = (float)H->h[l];
  if (l == H->L - 1) {
    const size_t N = node_count(dim, n);
    double* fd = H->r[l];
    double* ud = (double*)calloc(N, sizeof(double));
    if (!ud) return OR_ENOMEM;
    for (size_t i = 0; i < N; ++i) fd[i] = (double)H->f32[l][i];
    const int st = coarsest_solve(dim, n, H->h[l], H->k[l], fd, ud);
    for (size_t i = 0; i < N; ++i) H->u32[l][i] = (float)ud[i];
    free(ud);
    return st;
  }
  for (int s = 0; s < H->nu1; ++s) {
    rbgs_half_f32(dim, n, h, H->k32[l], H->f32[l], H->u32[l], 0);
    rbgs_half_f32(dim, n, h, H->k32[l], H->f32[l], H->u32[l], 1);
  }
  residual_f32(dim, n, h, H->k32[l], H->f32[l], H->u32[l], H->r32[l]);
  restrict_fw_f32(dim, n, H->r32[l], H->f32[l + 1]);
  memset(H->u32[l + 1], 0, node_count(dim, H->n[l + 1]) * sizeof(float));
  const int st = vcycle_f32(H, l + 1);
  if (st) return st;
  prolong_add_f32(dim, H->n[l + 1], H->u32[l + 1], H->u32[l]);
  for (int s = 0; s < H->nu2; ++s) {
    rbgs_half_f32(dim, n, h, H->k32[l], H->f32[l], H->u32[l], 0);
    rbgs_half_f32(dim, n, h, H->k32[l], H->f32[l], H->u32[l], 1);
  }
  return OR_OK;
}

/* One step of iterative refinement: r = f - A u in FP64; r32 = r / s rounded to float,
 * with s a power of two (an exact scaling that only keeps r32 far from the float range
 * limits; in float arithmetic it changes no result); e32 = one FP32 V-cycle for
 * A e = r32 from e = 0 with zero Dirichlet data; u += s * e32 in FP64. */
static int ir_step(hierarchy* H, double s)
{
  const int dim = H->dim, n = H->n[0];
  const size_t N = node_count(dim, n);
  residual_f64(dim, n, H->h[0], H->k[0], H->f[0], H->u[0], H->r[0]);
  for (size_t i = 0; i < N; ++i) {
    H->f32[0][i] = (float)(H->r[0][i] / s);
    H->u32[0][i] = 0.0f;
  }
  const int st = vcycle_f32(H, 0);
  if (st) return st;
  const int z0 = dim == 3 ? 1 : 0, z1 = dim == 3 ? n - 2 : 0;
  for (int z = z0; z <= z1; ++z)
    for (int y = 1; y <= n - 2; ++y)
      for (int x = 1; x <= n - 2; ++x) {
        const size_t i = IDX(n, z, y, x);
        H->u[0][i] += s * (double)H->u32[0][i];
      }
  return OR_OK;
}

/* ||b||_2 of the full discrete right-hand side: b = f - A u_B, where u_B is u with its
 * interior set to zero (b = f when the Dirichlet data are zero). */
static double rhs_norm(hierarchy* H)
{
  const int dim = H->dim, n = H->n[0];
  const size_t N = node_count(dim, n);
  double* ub = (double*)malloc(N * sizeof(double));
  if (!ub) return NAN;
  memcpy(ub, H->u[0], N * sizeof(double));
  const int z0 = dim == 3 ? 1 : 0, z1 = dim == 3 ? n - 2 : 0;
  for (int z = z0; z <= z1; ++z)
    for (int y = 1; y <= n - 2; ++y)
      for (int x = 1; x <= n - 2; ++x) ub[IDX(n, z, y, x)] = 0.0;
  residual_f64(dim, n, H->h[0], H->k[0], H->f[0], ub, H->r[0]);
  free(ub);
  return sqrt(interior_norm2(dim, n, H->r[0]));
}

static double residual_norm(hierarchy* H)
{
  residual_f64(H->dim, H->n[0], H->h[0], H->k[0], H->f[0], H->u[0], H->r[0]);
  return sqrt(interior_norm2(H->dim, H->n[0], H->r[0]));
}

/* Power of two nearest (in log2) to the root-mean-square of a residual with norm rn. */
static double ir_scale(double rn, int dim, int n)
{
  const double m = dim == 3 ? (double)(n - 2) * (n - 2) * (n - 2) : (double)(n - 2) * (n - 2);
  const double rms = rn / sqrt(m);
  if (!(rms > 0) || !isfinite(rms)) return 1.0;
  return ldexp(1.0, (int)lround(log2(rms)));
}

/* ------------------------------------------------------------------ exported API */

void or_apply(int dim, int n, double h, const double* k, const double* u, double* out)
{
  apply_f64(dim, n, h, k, u, out);
}
void or_residual(int dim, int n, double h, const double* k, const double* f, const double* u,
                 double* r)
{
  residual_f64(dim, n, h, k, f, u, r);
}
void or_rbgs_half(int dim, int n, double h, const double* k, const double* f, double* u,
                  int colour)
{
  rbgs_half_f64(dim, n, h, k, f, u, colour);
}
void or_restrict_fw(int dim, int nf, const double* r, double* fc)
{
  restrict_fw_f64(dim, nf, r, fc);
}
void or_prolong_add(int dim, int nc, const double* e, double* u)
{
  prolong_add_f64(dim, nc, e, u);
}
void or_residual_f32(int dim, int n, float h, const float* k, const float* f, const float* u,
                     float* r)
{
  residual_f32(dim, n, h, k, f, u, r);
}
void or_rbgs_half_f32(int dim, int n, float h, const float* k, const float* f, float* u,
                      int colour)
{
  rbgs_half_f32(dim, n, h, k, f, u, colour);
}
void or_restrict_fw_f32(int dim, int nf, const float* r, float* fc)
{
  restrict_fw_f32(dim, nf, r, fc);
}
void or_prolong_add_f32(int dim, int nc, const float* e, float* u)
{
  prolong_add_f32(dim, nc, e, u);
}
int or_coarsest_solve(int dim, int n, double h, const double* k, const double* f, double* u)
{
  return coarsest_solve(dim, n, h, k, f, u);
}
double or_interior_norm2(int dim, int n, const double* v) { return interior_norm2(dim, n, v); }

/* One FP64 V(nu1,nu2)-cycle on the finest level of an L-level hierarchy (u in/out). */
int or_vcycle(int dim, int n, int L, int nu1, int nu2, const double* k, const double* f,
              double* u)
{
  hierarchy H;
  int st = hier_init(&H, dim, n, L, nu1, nu2, k, 0);
  if (st) return st;
  H.u[0] = u;
  H.f[0] = (double*)f;
  st = vcycle_f64(&H, 0);
  H.u[0] = NULL; H.f[0] = NULL;
  hier_free(&H);
  return st;
}

/* Multigrid solve of A u = f (u in/out: initial guess in the interior, Dirichlet data on
 * the boundary).  precision 0: FP64 V-cycles; precision 1: FP32 V-cycles inside FP64
 * iterative refinement.  After every cycle the relative residual
 * ||f - A u||_2 / ||b||_2 (interior nodes; b as in rhs_norm, or 1 if ||b|| = 0) is
 * compared with tol; at most max_cycles cycles are run.  hist (nullable, max_cycles+1
 * entries) receives the relative residual before the first cycle and after each cycle.
 * Returns OR_OK, OR_ENOCONV (max_cycles reached), OR_ENAN (non-finite norm) or a setup
 * error. */
static double g_solve_seconds = 0.0;  /* wall time of the last or_solve's iteration */

static double wall_seconds(void)
{
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Wall-clock seconds of the last or_solve from the first norm to the last cycle: the
 * hierarchy's allocation and release are outside (timing only; used by the benchmark's
 * CPU baseline). */
double or_last_solve_seconds(void) { return g_solve_seconds; }

int or_solve(int dim, int n, int L, int nu1, int nu2, int max_cycles, int precision,
             const double* k, const double* f, double* u, double tol, int* cycles,
             double* relres, double* hist)
{
  hierarchy H;
  if (max_cycles < 0 || !(tol > 0)) return OR_EINVAL;
  int st = hier_init(&H, dim, n, L, nu1, nu2, k, precision == 1);
  if (st) return st;
  const double t0 = wall_seconds();
  H.u[0] = u;
  H.f[0] = (double*)f;
  double bn = rhs_norm(&H);
  if (!(bn > 0)) bn = 1.0;
  double rn = residual_norm(&H);
  double rel = rn / bn;
  int c = 0;
  if (hist) hist[0] = rel;
  while (isfinite(rel) && rel > tol && c < max_cycles) {
    if (precision == 1) st = ir_step(&H, ir_scale(rn, dim, n));
    else st = vcycle_f64(&H, 0);
    if (st) break;
    ++c;
    rn = residual_norm(&H);
    rel = rn / bn;
    if (hist) hist[c] = rel;
  }
  g_solve_seconds = wall_seconds() - t0;
  if (cycles) *cycles = c;
  if (relres) *relres = rel;
  H.u[0] = NULL; H.f[0] = NULL;
  hier_free(&H);
  if (st) return st;
  if (!isfinite(rel)) return OR_ENAN;
  if (rel > tol) return OR_ENOCONV;
  return OR_OK;
}

/* Gradient of L(u(k,f)) given u (solution of A(k) u = f) and lambda (solution of the
 * adjoint system A^T lambda = dL/du with zero boundary values; A is symmetric).
 * Implicit differentiation of A(k) u = f gives dL/df = lambda and
 * dL/dk = -lambda^T (dA/dk) u.  With arithmetic-mean faces, k_j enters the rows of j and
 * of its neighbours; collecting the terms (lambda extended by 0 to boundary nodes):
 *   dL/dk_j = -1/(2 h^2) * sum over the axis neighbours nb of j inside the grid of
 *             (lambda_j - lambda_nb) (u_j - u_nb)            for every node j,
 *   dL/df_j = lambda_j on interior nodes, 0 on boundary nodes. */
void or_grad(int dim, int n, const double* u, const double* lam, double* dk, double* df)
{
  const double h = 1.0 / (double)(n - 1);
  const double c = -1.0 / (2.0 * h * h);
  const int Zn = dim == 3 ? n : 1;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < Zn; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const size_t j = IDX(n, z, y, x);
        const int jin = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2 &&
                        (dim == 2 || (z >= 1 && z <= n - 2));
        const double lj = jin ? lam[j] : 0.0;
        const int nz[6] = {z, z, z, z, z - 1, z + 1};
        const int ny[6] = {y, y, y - 1, y + 1, y, y};
        const int nx[6] = {x - 1, x + 1, x, x, x, x};
        double s = 0;
        for (int a = 0; a < 2 * dim; ++a) {
          if (nx[a] < 0 || nx[a] >= n || ny[a] < 0 || ny[a] >= n) continue;
          if (dim == 3 && (nz[a] < 0 || nz[a] >= n)) continue;
          const size_t b = IDX(n, dim == 3 ? nz[a] : 0, ny[a], nx[a]);
          const int bin = nx[a] >= 1 && nx[a] <= n - 2 && ny[a] >= 1 && ny[a] <= n - 2 &&
                          (dim == 2 || (nz[a] >= 1 && nz[a] <= n - 2));
          const double lb = bin ? lam[b] : 0.0;
          s += (lj - lb) * (u[j] - u[b]);
        }
        dk[j] = c * s;
        df[j] = jin ? lam[j] : 0.0;
      }
}
