/*
 * fv_oracle.c -- plain CPU oracle for the paper's own benchmark solver on a uniform grid.
 *
 * TEST INFRASTRUCTURE, like mg_oracle.c: only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; it shares no code with the GPU library.
 *
 * Paper (Sect. 5, Eq. 1-2): -Laplace(u) = f on [0,1]^3 with Dirichlet data g on the
 * boundary, discretised with the cell-centred finite-volume method and solved with a
 * V(3,3) multigrid cycle whose smoother is damped Jacobi (omega = 0.8), Jacobi also serving
 * as the coarsest-grid solver (256 iterations in the benchmark of Sect. 6); the solver stops
 * when the L2 norm of the residual falls below a threshold or after a maximum number of
 * cycles.  The paper does not print the transfer operators or the boundary treatment; the
 * readings taken here:
 *   - N^3 cells (N = 2^m), cell i in 1..N per axis with centre (i - 1/2) h, h = 1/N; arrays
 *     hold (N+2)^3 values, the ghost layer (index 0 and N+1) carrying the Dirichlet value g
 *     at the centre of the adjacent boundary face;
 *   - the flux through a boundary face is (u_i - g) / (h/2): the ghost neighbour enters the
 *     7-point operator as 2 g - u_i (linear extrapolation through the face value);
 *   - (A u)_i = (1/h^2) sum over the 6 face neighbours of (u_i - v_nb), v_nb = u_nb inside,
 *     2 g - u_i across a boundary face; re-discretised with h = 2^l / N on level l;
 *   - damped Jacobi: u_new = u + omega (h^2 / 6) (f - A u), the diagonal of the interior
 *     7-point stencil;
 *   - restriction: the mean of the 8 child cells; prolongation: trilinear interpolation of
 *     the coarse cell centres (weights 3/4 and 1/4 per axis), the coarse correction
 *     extended across the boundary by its homogeneous ghost value -e (zero on the face);
 *   - the coarse-grid problem has homogeneous Dirichlet data and starts from 0; on the
 *     coarsest level the fixed number of Jacobi iterations starts from 0 as well;
 *   - the L2 residual norm is sqrt(sum over cells of r^2) (unweighted).
 *
 * Parallelism: OpenMP over z in the elementwise loops only (every cell is written by one
 * iteration, from values no iteration writes); norms are summed per plane, then serially.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define FIDX(m, z, y, x) ((((size_t)(z)) * (size_t)(m) + (size_t)(y)) * (size_t)(m) + (size_t)(x))
#define FV_MAXL 16

enum { FV_OK = 0, FV_EINVAL = 1, FV_ENOMEM = 2, FV_ENOCONV = 4, FV_ENAN = 5 };

/* Value of the face neighbour at (z, y, x) seen from cell value ui: inside the grid the
 * neighbour itself, in the ghost layer the linear extrapolation 2 g - ui. */
static double nb_value(int N, const double* u, int z, int y, int x, double ui)
{
  const int m = N + 2;
  const double v = u[FIDX(m, z, y, x)];
  const int ghost = z == 0 || z == N + 1 || y == 0 || y == N + 1 || x == 0 || x == N + 1;
  return ghost ? 2.0 * v - ui : v;
}

/* (A u) at interior cell (z, y, x): the neighbours in the order -x, +x, -y, +y, -z, +z. */
static double apply_at(int N, double h, const double* u, int z, int y, int x)
{
  const int m = N + 2;
  const double ui = u[FIDX(m, z, y, x)];
  const double v[6] = {nb_value(N, u, z, y, x - 1, ui), nb_value(N, u, z, y, x + 1, ui),
                       nb_value(N, u, z, y - 1, x, ui), nb_value(N, u, z, y + 1, x, ui),
                       nb_value(N, u, z - 1, y, x, ui), nb_value(N, u, z + 1, y, x, ui)};
  double s = 0.0;
  for (int j = 0; j < 6; ++j) s += ui - v[j];
  return s / (h * h);
}

/* out = A u on the interior cells, 0 on the ghost layer. */
void or_fv_apply(int N, double h, const double* u, double* out)
{
  const int m = N + 2;
  memset(out, 0, sizeof(double) * (size_t)m * m * m);
#pragma omp parallel for
  for (int z = 1; z <= N; ++z)
    for (int y = 1; y <= N; ++y)
      for (int x = 1; x <= N; ++x) out[FIDX(m, z, y, x)] = apply_at(N, h, u, z, y, x);
}

/* r = f - A u on the interior cells, 0 on the ghost layer. */
void or_fv_residual(int N, double h, const double* f, const double* u, double* r)
{
  const int m = N + 2;
  memset(r, 0, sizeof(double) * (size_t)m * m * m);
#pragma omp parallel for
  for (int z = 1; z <= N; ++z)
    for (int y = 1; y <= N; ++y)
      for (int x = 1; x <= N; ++x) {
        const size_t i = FIDX(m, z, y, x);
        r[i] = f[i] - apply_at(N, h, u, z, y, x);
      }
}

/* One damped Jacobi sweep, out of place: uout = u + omega (h^2/6) (f - A u) on the interior;
 * the ghost layer of uout is copied from u (the Dirichlet data). */
void or_fv_jacobi(int N, double h, double omega, const double* f, const double* u, double* uout)
{
  const int m = N + 2;
  memcpy(uout, u, sizeof(double) * (size_t)m * m * m);
#pragma omp parallel for
  for (int z = 1; z <= N; ++z)
    for (int y = 1; y <= N; ++y)
      for (int x = 1; x <= N; ++x) {
        const size_t i = FIDX(m, z, y, x);
        const double r = f[i] - apply_at(N, h, u, z, y, x);
        uout[i] = u[i] + omega * (h * h / 6.0) * r;
      }
}

/* fc = mean of the 8 children of every coarse cell (fine grid of N cells, coarse N/2);
 * the coarse ghost layer is 0. */
void or_fv_restrict(int N, const double* r, double* fc)
{
  const int m = N + 2, Nc = N / 2, mc = Nc + 2;
  memset(fc, 0, sizeof(double) * (size_t)mc * mc * mc);
#pragma omp parallel for
  for (int Z = 1; Z <= Nc; ++Z)
    for (int Y = 1; Y <= Nc; ++Y)
      for (int X = 1; X <= Nc; ++X) {
        double s = 0.0;
        for (int dz = 0; dz < 2; ++dz)
          for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
              s += r[FIDX(m, 2 * Z - 1 + dz, 2 * Y - 1 + dy, 2 * X - 1 + dx)];
        fc[FIDX(mc, Z, Y, X)] = s / 8.0;
      }
}

/* Coarse correction value at coarse index (Z, Y, X), which may lie in the ghost layer: there
 * the homogeneous extension -e of the adjacent interior cell (zero on the face). */
static double coarse_value(int Nc, const double* e, int Z, int Y, int X)
{
  const int mc = Nc + 2;
  int z = Z, y = Y, x = X;
  double sign = 1.0;
  if (z == 0) { z = 1; sign = -sign; }
  if (z == Nc + 1) { z = Nc; sign = -sign; }
  if (y == 0) { y = 1; sign = -sign; }
  if (y == Nc + 1) { y = Nc; sign = -sign; }
  if (x == 0) { x = 1; sign = -sign; }
  if (x == Nc + 1) { x = Nc; sign = -sign; }
  return sign * e[FIDX(mc, z, y, x)];
}

/* u += P e on the fine interior: fine cell i lies a quarter coarse cell from the centre of
 * its parent I = (i+1)/2, towards I-1 (i odd) or I+1 (i even); per axis the parent gets
 * 3/4 and that neighbour 1/4, and the three axes multiply. */
void or_fv_prolong_add(int Nc, const double* e, double* u)
{
  const int N = 2 * Nc, m = N + 2;
#pragma omp parallel for
  for (int z = 1; z <= N; ++z)
    for (int y = 1; y <= N; ++y)
      for (int x = 1; x <= N; ++x) {
        const int P[3] = {(z + 1) / 2, (y + 1) / 2, (x + 1) / 2};
        const int Q[3] = {(z & 1) ? P[0] - 1 : P[0] + 1, (y & 1) ? P[1] - 1 : P[1] + 1,
                          (x & 1) ? P[2] - 1 : P[2] + 1};
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
              const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
              s += w * coarse_value(Nc, e, a ? Q[0] : P[0], b ? Q[1] : P[1], c ? Q[2] : P[2]);
            }
        u[FIDX(m, z, y, x)] += s;
      }
}

/* sum of squares over the interior cells: per plane, then the planes in order */
double or_fv_norm2(int N, const double* v)
{
  const int m = N + 2;
  double* plane = (double*)malloc(sizeof(double) * (size_t)(N + 1));
  if (!plane) return NAN;
#pragma omp parallel for
  for (int z = 1; z <= N; ++z) {
    double s = 0.0;
    for (int y = 1; y <= N; ++y)
      for (int x = 1; x <= N; ++x) {
        const double t = v[FIDX(m, z, y, x)];
        s += t * t;
      }
    plane[z] = s;
  }
  double tot = 0.0;
  for (int z = 1; z <= N; ++z) tot += plane[z];
  free(plane);
  return tot;
}

/* Jacobi sweeps in place (through a scratch copy). */
static int jacobi_sweeps(int N, double h, double omega, const double* f, double* u, int sweeps)
{
  const int m = N + 2;
  const size_t cnt = (size_t)m * m * m;
  double* t = (double*)malloc(sizeof(double) * cnt);
  if (!t) return FV_ENOMEM;
  for (int s = 0; s < sweeps; ++s) {
    or_fv_jacobi(N, h, omega, f, u, t);
    memcpy(u, t, sizeof(double) * cnt);
  }
  free(t);
  return FV_OK;
}

int or_fv_jacobi_sweeps(int N, double h, double omega, const double* f, double* u, int sweeps)
{
  return jacobi_sweeps(N, h, omega, f, u, sweeps);
}

/* One V(nu1, nu2)-cycle on level l (N cells per side, mesh width h) in place; below it the
 * levels of N/2, N/4, ... cells, `levels` in all.  The coarsest level runs coarse_iters
 * Jacobi iterations from the u it is given: 0 for every coarse-grid problem, which also has
 * homogeneous Dirichlet data (its arrays are allocated zeroed). */
static int vcycle_rec(int N, double h, int levels, int nu1, int nu2, int coarse_iters,
                      double omega, const double* f, double* u)
{
  if (levels == 1) return jacobi_sweeps(N, h, omega, f, u, coarse_iters);
  int st = jacobi_sweeps(N, h, omega, f, u, nu1);
  if (st) return st;
  const int m = N + 2, Nc = N / 2, mc = Nc + 2;
  double* r = (double*)malloc(sizeof(double) * (size_t)m * m * m);
  double* fc = (double*)malloc(sizeof(double) * (size_t)mc * mc * mc);
  double* ec = (double*)calloc((size_t)mc * mc * mc, sizeof(double));
  if (!r || !fc || !ec) {
    free(r); free(fc); free(ec);
    return FV_ENOMEM;
  }
  or_fv_residual(N, h, f, u, r);
  or_fv_restrict(N, r, fc);
  st = vcycle_rec(Nc, 2.0 * h, levels - 1, nu1, nu2, coarse_iters, omega, fc, ec);
  if (!st) or_fv_prolong_add(Nc, ec, u);
  free(r); free(fc); free(ec);
  if (st) return st;
  return jacobi_sweeps(N, h, omega, f, u, nu2);
}

static int valid(int N, int levels)
{
  if (N < 2 || levels < 1 || levels > FV_MAXL) return 0;
  if (N % (1 << (levels - 1)) != 0) return 0;
  return (N >> (levels - 1)) >= 1;
}

int or_fv_vcycle(int N, int levels, int nu1, int nu2, int coarse_iters, double omega,
                 const double* f, double* u)
{
  if (!valid(N, levels) || nu1 < 0 || nu2 < 0 || coarse_iters < 0) return FV_EINVAL;
  return vcycle_rec(N, 1.0 / N, levels, nu1, nu2, coarse_iters, omega, f, u);
}

/* Cycles until the L2 residual norm is <= tol or max_cycles cycles ran.  hist[k] = the
 * residual norm after k cycles (k = 0 .. cycles).  Returns FV_ENOCONV when the tolerance was
 * not reached (u holds the last iterate; the benchmark stops at the cycle limit by design). */
int or_fv_solve(int N, int levels, int nu1, int nu2, int coarse_iters, double omega,
                const double* f, double* u, double tol, int max_cycles, int* cycles,
                double* resnorm, double* hist)
{
  if (!valid(N, levels) || max_cycles < 0) return FV_EINVAL;
  const int m = N + 2;
  const double h = 1.0 / N;
  double* r = (double*)malloc(sizeof(double) * (size_t)m * m * m);
  if (!r) return FV_ENOMEM;
  or_fv_residual(N, h, f, u, r);
  double rn = sqrt(or_fv_norm2(N, r));
  if (hist) hist[0] = rn;
  int k = 0, st = FV_OK;
  while (isfinite(rn) && rn > tol && k < max_cycles) {
    st = vcycle_rec(N, h, levels, nu1, nu2, coarse_iters, omega, f, u);
    if (st) break;
    ++k;
    or_fv_residual(N, h, f, u, r);
    rn = sqrt(or_fv_norm2(N, r));
    if (hist) hist[k] = rn;
  }
  free(r);
  if (cycles) *cycles = k;
  if (resnorm) *resnorm = rn;
  if (st) return st;
  if (!isfinite(rn)) return FV_ENAN;
  return rn <= tol ? FV_OK : FV_ENOCONV;
}
