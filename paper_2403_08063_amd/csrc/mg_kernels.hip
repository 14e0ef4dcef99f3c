// Straightforward HIP kernels of the multigrid cycle for gfx950: per-colour Gauss-Seidel
// half-sweeps, fused residual + full-weighting restriction, linear prolongation, the
// coarsest-level direct solve, deterministic residual norms, iterative-refinement casts,
// coefficient coarsening and the adjoint gradient pass.  They serve 2D grids and the
// small 3D levels; large 3D levels use the temporally blocked smoother (mg_smooth_tiled.hip).
//
// Paper: Angersbach, Kuckuk, Koestler, "Towards Code Generation for Octree-Based Multigrid
// Solvers": model problem Sect. 5 (Eq. 1-2), V-cycle Sect. 1/5, per-level re-discretised
// operators with the level's mesh width passed as a kernel scalar (Sect. 4.2-4.3).
#include "mg_kernels.h"
#include "mg_stencil.h"

#include <cmath>

namespace mgk {
namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ red-black half-sweep
// Thread t of row (y, z) updates the t-th node of the colour in that row:
// x = x0 + 2t with x0 the first interior x of the colour.
template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_rbgs_colour(T* u, const T* __restrict__ f, const T* __restrict__ k, int n, T h2,
                  int colour)
{
  const int y = blockIdx.y + 1;
  const int z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  const int x = 1 + ((1 + y + z + colour) & 1) + 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (x > n - 2) return;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  const size_t i = ((size_t)z * n + y) * (size_t)n + x;
  u[i] = gs_at<T, DIM, VAR>(f, u, k, i, sy, sz, h2);
}

// The first colour-0 half-sweep of a pre-smoothing from a zero guess: colour-0 nodes take
// the Gauss-Seidel value of the zero iterate, colour-1 nodes are set to 0 (the fill of the
// zero guess, in the same launch; boundary nodes, 0 on the coarse levels, are not written).
template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_rbgs_first_zero(T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ k,
                      int n, T h2)
{
  const int y = blockIdx.y + 1;
  const int z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int x0 = 1 + ((1 + y + z) & 1) + 2 * q, x1 = 1 + ((y + z) & 1) + 2 * q;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  const size_t row = ((size_t)z * n + y) * (size_t)n;
  if (x0 <= n - 2) u[row + x0] = gs_zero_at<T, DIM, VAR>(f, k, row + x0, sy, sz, h2);
  if (x1 <= n - 2) u[row + x1] = T(0);
}

// The first colour-0 half-sweep of a post-smoothing with the coarse-grid correction: the
// colour-1 neighbours are read as u + P ec (corrected_at), so the correction is never
// stored -- the colour-0 nodes are overwritten by this half-sweep and the colour-1 nodes by
// the next, neither reading its own old value.
template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_rbgs_first_prolong(T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ k,
                         const T* __restrict__ ec, int n, int nc, T h2)
{
  const int y = blockIdx.y + 1;
  const int z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  const int x = 1 + ((1 + y + z) & 1) + 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (x > n - 2) return;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  const size_t i = ((size_t)z * n + y) * (size_t)n + x;
  const T xm = corrected_at<T, DIM>(u, ec, n, nc, z, y, x - 1);
  const T xp = corrected_at<T, DIM>(u, ec, n, nc, z, y, x + 1);
  const T ym = corrected_at<T, DIM>(u, ec, n, nc, z, y - 1, x);
  const T yp = corrected_at<T, DIM>(u, ec, n, nc, z, y + 1, x);
  const T zm = DIM == 3 ? corrected_at<T, DIM>(u, ec, n, nc, z - 1, y, x) : T(0);
  const T zp = DIM == 3 ? corrected_at<T, DIM>(u, ec, n, nc, z + 1, y, x) : T(0);
  const T h2f = h2 * f[i];
  if (!VAR) {
    u[i] = gs_const<T, DIM>(h2f, xm, xp, ym, yp, zm, zp);
  } else {
    const T kzm = DIM == 3 ? k[i - sz] : T(0), kzp = DIM == 3 ? k[i + sz] : T(0);
    u[i] = gs_var<T, DIM>(h2f, k[i], xm, k[i - 1], xp, k[i + 1], ym, k[i - sy], yp, k[i + sy],
                          zm, kzm, zp, kzp);
  }
}

// ------------------------------------------------------------------ residual
template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_residual(const T* __restrict__ f, const T* __restrict__ u, const T* __restrict__ k,
               T* __restrict__ r, int n, T ih2)
{
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= n) return;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  const size_t i = ((size_t)z * n + y) * (size_t)n + x;
  const bool in = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2 &&
                  (DIM == 2 || (z >= 1 && z <= n - 2));
  r[i] = in ? resid_at<T, DIM, VAR>(f, u, k, i, sy, sz, ih2) : T(0);
}

// ------------------------------------------------------------------ residual + restriction
// One thread per coarse interior node (restrict_at).
template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_restrict_residual(const T* __restrict__ f, const T* __restrict__ u,
                        const T* __restrict__ k, T* __restrict__ fc, int nf, T ih2)
{
  const int nc = (nf - 1) / 2 + 1;
  const int X = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  const int Y = blockIdx.y + 1;
  const int Z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  if (X > nc - 2) return;
  fc[((size_t)Z * nc + Y) * (size_t)nc + X] = restrict_at<T, DIM, VAR>(f, u, k, nf, ih2, X, Y, Z);
}

// ------------------------------------------------------------------ prolongation
// Thread c of a fine row handles the pair x = 2c-1 (coarse c-1, c) and x = 2c (coarse c),
// which share the two coarse values of each coarse row (prolong_pair).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock)
    k_prolong_add(const T* __restrict__ e, T* __restrict__ u, int nc)
{
  const int c = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y + 1;
  const int z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  if (c > nc - 1) return;
  prolong_pair<T, DIM>(e, u, nc, c, y, z);
}

// ------------------------------------------------------------------ coarsest level

// One workgroup: assemble A (m x m, row-major) in `a`, Cholesky-factor it in place
// (right-looking: scale column j, then update the trailing lower triangle), then form
// A^-1 = L^-T L^-1 one column per thread by forward and back substitution.
__global__ void __launch_bounds__(kBlock)
    k_coarsest_factor(int dim, int n, double ih2, const double* __restrict__ k,
                      double* __restrict__ a, double* __restrict__ ainv, int* flag)
{
  const int m1 = n - 2;
  const int m = dim == 3 ? m1 * m1 * m1 : m1 * m1;
  const int tid = threadIdx.x;
  for (size_t e = tid; e < (size_t)m * m; e += blockDim.x) a[e] = 0.0;
  if (tid == 0) *flag = 0;
  __syncthreads();
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  for (int q = tid; q < m; q += blockDim.x) {
    int z, y, x;
    unknown_to_node(dim, n, q, z, y, x);
    const size_t i = ((size_t)z * n + y) * (size_t)n + x;
    const int nz[6] = {z, z, z, z, z - 1, z + 1};
    const int ny[6] = {y, y, y - 1, y + 1, y, y};
    const int nx[6] = {x - 1, x + 1, x, x, x, x};
    const ptrdiff_t off[6] = {-1, 1, -(ptrdiff_t)sy, (ptrdiff_t)sy, -(ptrdiff_t)sz, (ptrdiff_t)sz};
    for (int j = 0; j < 2 * dim; ++j) {
      const double c = k ? 0.5 * (k[i] + k[i + off[j]]) : 1.0;
      a[(size_t)q * m + q] += c * ih2;
      const bool nb_in = nx[j] >= 1 && nx[j] <= n - 2 && ny[j] >= 1 && ny[j] <= n - 2 &&
                         (dim == 2 || (nz[j] >= 1 && nz[j] <= n - 2));
      if (nb_in) {
        const int col = dim == 3 ? ((nz[j] - 1) * m1 + (ny[j] - 1)) * m1 + (nx[j] - 1)
                                 : (ny[j] - 1) * m1 + (nx[j] - 1);
        a[(size_t)q * m + col] -= c * ih2;
      }
    }
  }
  __syncthreads();
  __shared__ double piv;
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      const double d = a[(size_t)j * m + j];
      if (!(d > 0.0)) *flag = 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      a[(size_t)j * m + j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += blockDim.x) a[(size_t)i * m + j] /= piv;
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += blockDim.x) {
      const double lij = a[(size_t)i * m + j];
      for (int p = j + 1; p <= i; ++p) a[(size_t)i * m + p] -= lij * a[(size_t)p * m + j];
    }
    __syncthreads();
  }
  // column c of A^-1: solve L y = e_c, then L^T x = y; stored in column c of ainv
  for (int c = tid; c < m; c += blockDim.x) {
    for (int i = 0; i < m; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int p = c; p < i; ++p) s -= a[(size_t)i * m + p] * ainv[(size_t)p * m + c];
      ainv[(size_t)i * m + c] = (i < c) ? 0.0 : s / a[(size_t)i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = ainv[(size_t)i * m + c];
      for (int p = i + 1; p < m; ++p) s -= a[(size_t)p * m + i] * ainv[(size_t)p * m + c];
      ainv[(size_t)i * m + c] = s / a[(size_t)i * m + i];
    }
  }
}

// One workgroup: interior of u = ainv * interior of f (coarsest_apply).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_coarsest_solve(int dim, int n, const double* __restrict__ ainv, const T* __restrict__ f,
                     T* __restrict__ u)
{
  __shared__ double b[1024];
  coarsest_apply<T>(dim, n, ainv, f, u, b);
}

// ------------------------------------------------------------------ reductions
// Wavefront (64 lanes) sum by butterfly shuffles, then across the waves of the block in
// LDS.  Fixed order: bitwise reproducible for a fixed launch shape.
__device__ __forceinline__ double block_sum(double v)
{
  __shared__ double part[kBlock / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
  return s;  // valid in thread 0
}

__device__ __forceinline__ void interior_coords(int dim, int n, size_t t, int& z, int& y, int& x)
{
  const size_t m1 = (size_t)(n - 2);
  x = 1 + (int)(t % m1);
  y = 1 + (int)((t / m1) % m1);
  z = dim == 3 ? 1 + (int)(t / (m1 * m1)) : 0;
}

// mode 0: r = f - A u; mode 1: r = f - A u_B (interior of u taken as 0).
template <int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_resid_norm2(const double* __restrict__ f, const double* __restrict__ u,
                  const double* __restrict__ k, int n, double ih2, int mode,
                  double* __restrict__ partial)
{
  const size_t m1 = (size_t)(n - 2);
  const size_t M = DIM == 3 ? m1 * m1 * m1 : m1 * m1;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < M;
       t += (size_t)gridDim.x * blockDim.x) {
    int z, y, x;
    interior_coords(DIM, n, t, z, y, x);
    const size_t i = ((size_t)z * n + y) * (size_t)n + x;
    double r;
    if (mode == 0) {
      r = resid_at<double, DIM, VAR>(f, u, k, i, sy, sz, ih2);
    } else {
      auto ub = [&](int zz, int yy, int xx) -> double {
        const bool in = xx >= 1 && xx <= n - 2 && yy >= 1 && yy <= n - 2 &&
                        (DIM == 2 || (zz >= 1 && zz <= n - 2));
        return in ? 0.0 : u[((size_t)zz * n + yy) * (size_t)n + xx];
      };
      const double xm = ub(z, y, x - 1), xp = ub(z, y, x + 1), ym = ub(z, y - 1, x),
                   yp = ub(z, y + 1, x);
      const double zm = DIM == 3 ? ub(z - 1, y, x) : 0.0, zp = DIM == 3 ? ub(z + 1, y, x) : 0.0;
      if (!VAR) {
        r = f[i] - au_const<double, DIM>(ih2, 0.0, xm, xp, ym, yp, zm, zp);
      } else {
        const double kzm = DIM == 3 ? k[i - sz] : 0.0, kzp = DIM == 3 ? k[i + sz] : 0.0;
        r = f[i] - au_var<double, DIM>(ih2, 0.0, k[i], xm, k[i - 1], xp, k[i + 1], ym,
                                       k[i - sy], yp, k[i + sy], zm, kzm, zp, kzp);
      }
    }
    acc += r * r;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
    k_sum_partials(const double* __restrict__ partial, int count, double* __restrict__ out)
{
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) out[0] = s;
}

// ------------------------------------------------------------------ iterative refinement
template <int DIM, bool VAR>
__global__ void __launch_bounds__(kBlock)
    k_ir_residual(const double* __restrict__ f, const double* __restrict__ u,
                  const double* __restrict__ k, int n, double ih2, double inv_scale,
                  float* __restrict__ r32, double* __restrict__ partial)
{
  const size_t m1 = (size_t)(n - 2);
  const size_t M = DIM == 3 ? m1 * m1 * m1 : m1 * m1;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < M;
       t += (size_t)gridDim.x * blockDim.x) {
    int z, y, x;
    interior_coords(DIM, n, t, z, y, x);
    const size_t i = ((size_t)z * n + y) * (size_t)n + x;
    const double r = resid_at<double, DIM, VAR>(f, u, k, i, sy, sz, ih2);
    r32[i] = (float)(r * inv_scale);
    acc += r * r;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock)
    k_ir_update(const float* __restrict__ e, double* __restrict__ u, int n, double scale)
{
  const int x = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y + 1;
  const int z = DIM == 3 ? (int)blockIdx.z + 1 : 0;
  if (x > n - 2) return;
  const size_t i = ((size_t)z * n + y) * (size_t)n + x;
  u[i] = u[i] + scale * (double)e[i];
}

// ------------------------------------------------------------------ coefficients
template <int DIM>
__global__ void __launch_bounds__(kBlock)
    k_coarsen_k(const double* __restrict__ k, double* __restrict__ kc, int nf)
{
  const int nc = (nf - 1) / 2 + 1;
  const int X = blockIdx.x * blockDim.x + threadIdx.x;
  const int Y = blockIdx.y;
  const int Z = DIM == 3 ? (int)blockIdx.z : 0;
  if (X >= nc) return;
  const bool in = X >= 1 && X <= nc - 2 && Y >= 1 && Y <= nc - 2 &&
                  (DIM == 2 || (Z >= 1 && Z <= nc - 2));
  const int fz = DIM == 3 ? 2 * Z : 0;
  const size_t out = ((size_t)Z * nc + Y) * (size_t)nc + X;
  if (!in) {
    kc[out] = k[((size_t)fz * nf + 2 * Y) * (size_t)nf + 2 * X];
    return;
  }
  const double w[3] = {0.25, 0.5, 0.25};
  double s = 0.0;
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox)
        s += w[ox + 1] * w[oy + 1] * (DIM == 3 ? w[oz + 1] : 1.0) *
             log(k[((size_t)(fz + oz) * nf + (2 * Y + oy)) * (size_t)nf + (2 * X + ox)]);
  kc[out] = exp(s);
}

__global__ void __launch_bounds__(kBlock)
    k_cast_f32(const double* __restrict__ src, float* __restrict__ dst, size_t count)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ------------------------------------------------------------------ adjoint gradient
// dk_j = -1/(2h^2) sum_{axis neighbours m in the grid} (lam_j - lam_m)(u_j - u_m) with lam
// read as 0 on boundary nodes; df_j = lam_j on interior nodes, 0 on the boundary.
// One wave per grid row (kBlock / 64 rows per workgroup), stepping along x by 64: rows of
// n = 2^m + 1 nodes leave one lane of the last step busy instead of most of a workgroup idle.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
    k_grad(const double* __restrict__ u, const double* __restrict__ lam, double* __restrict__ dk,
           double* __restrict__ df, int n, double c)
{
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);  // y + n z
  const int rows = DIM == 3 ? n * n : n;
  if (row >= rows) return;
  const int y = row % n;
  const int z = DIM == 3 ? row / n : 0;
  auto inside = [&](int zz, int yy, int xx) {
    return xx >= 1 && xx <= n - 2 && yy >= 1 && yy <= n - 2 &&
           (DIM == 2 || (zz >= 1 && zz <= n - 2));
  };
  for (int x = lane; x < n; x += 64) {
    const size_t j = ((size_t)z * n + y) * (size_t)n + x;
    const bool jin = inside(z, y, x);
    const double lj = jin ? lam[j] : 0.0;
    const double uj = u[j];
    if (dk) {
      const int nz[6] = {z, z, z, z, z - 1, z + 1};
      const int ny[6] = {y, y, y - 1, y + 1, y, y};
      const int nx[6] = {x - 1, x + 1, x, x, x, x};
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 2 * DIM; ++a) {
        if (nx[a] < 0 || nx[a] >= n || ny[a] < 0 || ny[a] >= n) continue;
        if (DIM == 3 && (nz[a] < 0 || nz[a] >= n)) continue;
        const size_t b = ((size_t)(DIM == 3 ? nz[a] : 0) * n + ny[a]) * (size_t)n + nx[a];
        const double lb = inside(nz[a], ny[a], nx[a]) ? lam[b] : 0.0;
        s += (lj - lb) * (uj - u[b]);
      }
      dk[j] = c * s;
    }
    if (df) df[j] = jin ? lj : 0.0;
  }
}

// The 3D gradient pass marching along z: a workgroup covers 64 x 4 nodes of a plane and
// kGradZ planes; every thread keeps u and lambda of the planes z-1, z, z+1 in registers, so
// each node is fetched from HBM once, its in-plane neighbours from the caches.  Same terms in
// the same order as k_grad.
constexpr int kGradZ = 32;

__global__ void __launch_bounds__(kBlock)
    k_grad3_march(const double* __restrict__ u, const double* __restrict__ lam,
                  double* __restrict__ dk, double* __restrict__ df, int n, double c)
{
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int z0 = blockIdx.z * kGradZ, z1 = min(z0 + kGradZ, n);
  if (x >= n || y >= n) return;  // no barrier below
  const size_t plane = (size_t)n * n, col = (size_t)y * n + x;
  auto inside = [&](int zz, int yy, int xx) {
    return xx >= 1 && xx <= n - 2 && yy >= 1 && yy <= n - 2 && zz >= 1 && zz <= n - 2;
  };
  auto lam_at = [&](int zz, int yy, int xx, size_t i) { return inside(zz, yy, xx) ? lam[i] : 0.0; };
  double um = 0.0, lm = 0.0;  // plane z-1
  if (z0 > 0) {
    um = u[(size_t)(z0 - 1) * plane + col];
    lm = lam_at(z0 - 1, y, x, (size_t)(z0 - 1) * plane + col);
  }
  double uc = u[(size_t)z0 * plane + col], lc = lam_at(z0, y, x, (size_t)z0 * plane + col);
  for (int z = z0; z < z1; ++z) {
    const size_t j = (size_t)z * plane + col;
    double up = 0.0, lp = 0.0;  // plane z+1
    if (z + 1 < n) {
      up = u[j + plane];
      lp = lam_at(z + 1, y, x, j + plane);
    }
    if (dk) {
      double s = 0.0;
      if (x - 1 >= 0) s += (lc - lam_at(z, y, x - 1, j - 1)) * (uc - u[j - 1]);
      if (x + 1 < n) s += (lc - lam_at(z, y, x + 1, j + 1)) * (uc - u[j + 1]);
      if (y - 1 >= 0) s += (lc - lam_at(z, y - 1, x, j - n)) * (uc - u[j - n]);
      if (y + 1 < n) s += (lc - lam_at(z, y + 1, x, j + n)) * (uc - u[j + n]);
      if (z - 1 >= 0) s += (lc - lm) * (uc - um);
      if (z + 1 < n) s += (lc - lp) * (uc - up);
      dk[j] = c * s;
    }
    if (df) df[j] = inside(z, y, x) ? lc : 0.0;
    um = uc;
    lm = lc;
    uc = up;
    lc = lp;
  }
}

// ------------------------------------------------------------------ small helpers
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ p, size_t count, T v)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_copy(const T* __restrict__ s, T* __restrict__ d, size_t count)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// Boundary nodes as the union of the 2d faces: face f, in-face coordinates (a, b).
__device__ __forceinline__ bool face_node(int dim, int n, int face, int a, int b, size_t& i)
{
  int z = 0, y, x;
  if (dim == 2) {
    if (b != 0) return false;
    switch (face) {
      case 0: y = 0; x = a; break;
      case 1: y = n - 1; x = a; break;
      case 2: y = a; x = 0; break;
      default: y = a; x = n - 1; break;
    }
  } else {
    switch (face) {
      case 0: z = 0; y = b; x = a; break;
      case 1: z = n - 1; y = b; x = a; break;
      case 2: z = b; y = 0; x = a; break;
      case 3: z = b; y = n - 1; x = a; break;
      case 4: z = b; y = a; x = 0; break;
      default: z = b; y = a; x = n - 1; break;
    }
  }
  i = ((size_t)z * n + y) * (size_t)n + x;
  return true;
}

__global__ void __launch_bounds__(kBlock)
    k_boundary(const double* __restrict__ src, double* __restrict__ dst, int dim, int n)
{
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const int face = blockIdx.z;
  if (a >= n) return;
  size_t i;
  if (!face_node(dim, n, face, a, b, i)) return;
  dst[i] = src ? src[i] : 0.0;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

inline int grid_for(size_t count)
{
  const size_t g = (count + kBlock - 1) / kBlock;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

// ================================================================== launchers
template <typename T>
void rbgs_colour(hipStream_t s, int dim, int n, double h, const T* k, const T* f, T* u,
                 int colour)
{
  const int half = (n - 1) / 2;  // nodes of one colour in a row, rounded up
  const int bx = half >= 256 ? 256 : (half > 64 ? 128 : 64);
  const dim3 grid(cdiv(half, bx), n - 2, dim == 3 ? n - 2 : 1);
  const T h2 = (T)(h * h);
  if (dim == 3) {
    if (k) k_rbgs_colour<T, 3, true><<<grid, bx, 0, s>>>(u, f, k, n, h2, colour);
    else k_rbgs_colour<T, 3, false><<<grid, bx, 0, s>>>(u, f, k, n, h2, colour);
  } else {
    if (k) k_rbgs_colour<T, 2, true><<<grid, bx, 0, s>>>(u, f, k, n, h2, colour);
    else k_rbgs_colour<T, 2, false><<<grid, bx, 0, s>>>(u, f, k, n, h2, colour);
  }
}

template <typename T>
void rbgs_first(hipStream_t s, int dim, int n, double h, const T* k, const T* f, T* u,
                const T* ec)
{
  const int half = (n - 1) / 2;
  const int bx = half >= 256 ? 256 : (half > 64 ? 128 : 64);
  const dim3 grid(cdiv(half, bx), n - 2, dim == 3 ? n - 2 : 1);
  const T h2 = (T)(h * h);
  const int nc = (n - 1) / 2 + 1;
  if (ec) {
    if (dim == 3) {
      if (k) k_rbgs_first_prolong<T, 3, true><<<grid, bx, 0, s>>>(u, f, k, ec, n, nc, h2);
      else k_rbgs_first_prolong<T, 3, false><<<grid, bx, 0, s>>>(u, f, k, ec, n, nc, h2);
    } else {
      if (k) k_rbgs_first_prolong<T, 2, true><<<grid, bx, 0, s>>>(u, f, k, ec, n, nc, h2);
      else k_rbgs_first_prolong<T, 2, false><<<grid, bx, 0, s>>>(u, f, k, ec, n, nc, h2);
    }
  } else {
    if (dim == 3) {
      if (k) k_rbgs_first_zero<T, 3, true><<<grid, bx, 0, s>>>(u, f, k, n, h2);
      else k_rbgs_first_zero<T, 3, false><<<grid, bx, 0, s>>>(u, f, k, n, h2);
    } else {
      if (k) k_rbgs_first_zero<T, 2, true><<<grid, bx, 0, s>>>(u, f, k, n, h2);
      else k_rbgs_first_zero<T, 2, false><<<grid, bx, 0, s>>>(u, f, k, n, h2);
    }
  }
}

template <typename T>
void residual(hipStream_t s, int dim, int n, double h, const T* k, const T* f, const T* u, T* r)
{
  const int bx = n >= 256 ? 256 : 64;
  const dim3 grid(cdiv(n, bx), n, dim == 3 ? n : 1);
  const T ih2 = (T)(1.0 / (h * h));
  if (dim == 3) {
    if (k) k_residual<T, 3, true><<<grid, bx, 0, s>>>(f, u, k, r, n, ih2);
    else k_residual<T, 3, false><<<grid, bx, 0, s>>>(f, u, k, r, n, ih2);
  } else {
    if (k) k_residual<T, 2, true><<<grid, bx, 0, s>>>(f, u, k, r, n, ih2);
    else k_residual<T, 2, false><<<grid, bx, 0, s>>>(f, u, k, r, n, ih2);
  }
}

template <typename T>
void restrict_residual(hipStream_t s, int dim, int nf, double h, const T* k, const T* f,
                       const T* u, T* fc)
{
  const int nc = (nf - 1) / 2 + 1;
  const int cnt = nc - 2;
  const int bx = cnt >= 256 ? 256 : (cnt > 64 ? 128 : 64);
  const dim3 grid(cdiv(cnt, bx), nc - 2, dim == 3 ? nc - 2 : 1);
  const T ih2 = (T)(1.0 / (h * h));
  if (dim == 3) {
    if (k) k_restrict_residual<T, 3, true><<<grid, bx, 0, s>>>(f, u, k, fc, nf, ih2);
    else k_restrict_residual<T, 3, false><<<grid, bx, 0, s>>>(f, u, k, fc, nf, ih2);
  } else {
    if (k) k_restrict_residual<T, 2, true><<<grid, bx, 0, s>>>(f, u, k, fc, nf, ih2);
    else k_restrict_residual<T, 2, false><<<grid, bx, 0, s>>>(f, u, k, fc, nf, ih2);
  }
}

template <typename T>
void prolong_add(hipStream_t s, int dim, int nc, const T* ec, T* u)
{
  const int nf = 2 * (nc - 1) + 1;
  const int cnt = nc - 1;  // fine x pairs per row
  const int bx = cnt >= 256 ? 256 : (cnt > 64 ? 128 : 64);
  const dim3 grid(cdiv(cnt, bx), nf - 2, dim == 3 ? nf - 2 : 1);
  if (dim == 3) k_prolong_add<T, 3><<<grid, bx, 0, s>>>(ec, u, nc);
  else k_prolong_add<T, 2><<<grid, bx, 0, s>>>(ec, u, nc);
}

void coarsest_factor(hipStream_t s, int dim, int n, double h, const double* k, double* work,
                     double* ainv, int* flag)
{
  k_coarsest_factor<<<1, kBlock, 0, s>>>(dim, n, 1.0 / (h * h), k, work, ainv, flag);
}

template <typename T>
void coarsest_solve(hipStream_t s, int dim, int n, const double* ainv, const T* f, T* u)
{
  k_coarsest_solve<T><<<1, kBlock, 0, s>>>(dim, n, ainv, f, u);
}

void resid_norm2(hipStream_t s, int dim, int n, double h, const double* k, const double* f,
                 const double* u, int mode, double* partial, double* out)
{
  const double ih2 = 1.0 / (h * h);
  if (dim == 3) {
    if (k) k_resid_norm2<3, true><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, mode, partial);
    else k_resid_norm2<3, false><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, mode, partial);
  } else {
    if (k) k_resid_norm2<2, true><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, mode, partial);
    else k_resid_norm2<2, false><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, mode, partial);
  }
  k_sum_partials<<<1, kBlock, 0, s>>>(partial, kNormBlocks, out);
}

void ir_residual(hipStream_t s, int dim, int n, double h, const double* k, const double* f,
                 const double* u, double inv_scale, float* r32, double* partial, double* out)
{
  const double ih2 = 1.0 / (h * h);
  if (dim == 3) {
    if (k) k_ir_residual<3, true><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, inv_scale, r32, partial);
    else k_ir_residual<3, false><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, inv_scale, r32, partial);
  } else {
    if (k) k_ir_residual<2, true><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, inv_scale, r32, partial);
    else k_ir_residual<2, false><<<kNormBlocks, kBlock, 0, s>>>(f, u, k, n, ih2, inv_scale, r32, partial);
  }
  k_sum_partials<<<1, kBlock, 0, s>>>(partial, kNormBlocks, out);
}

void ir_update(hipStream_t s, int dim, int n, double scale, const float* e32, double* u)
{
  const int cnt = n - 2;
  const int bx = cnt >= 256 ? 256 : 64;
  const dim3 grid(cdiv(cnt, bx), n - 2, dim == 3 ? n - 2 : 1);
  if (dim == 3) k_ir_update<3><<<grid, bx, 0, s>>>(e32, u, n, scale);
  else k_ir_update<2><<<grid, bx, 0, s>>>(e32, u, n, scale);
}

void coarsen_k(hipStream_t s, int dim, int nf, const double* k, double* kc)
{
  const int nc = (nf - 1) / 2 + 1;
  const int bx = nc >= 256 ? 256 : 64;
  const dim3 grid(cdiv(nc, bx), nc, dim == 3 ? nc : 1);
  if (dim == 3) k_coarsen_k<3><<<grid, bx, 0, s>>>(k, kc, nf);
  else k_coarsen_k<2><<<grid, bx, 0, s>>>(k, kc, nf);
}

void cast_to_f32(hipStream_t s, size_t count, const double* src, float* dst)
{
  k_cast_f32<<<grid_for(count), kBlock, 0, s>>>(src, dst, count);
}

void grad(hipStream_t s, int dim, int n, const double* u, const double* lam, double* dk,
          double* df)
{
  const double h = 1.0 / (double)(n - 1);
  const double c = -1.0 / (2.0 * h * h);
  if (dim == 3) {
    const dim3 grid(cdiv(n, 64), cdiv(n, 4), cdiv(n, kGradZ));
    k_grad3_march<<<grid, kBlock, 0, s>>>(u, lam, dk, df, n, c);
  } else {
    k_grad<2><<<dim3(cdiv(n, kBlock / 64)), kBlock, 0, s>>>(u, lam, dk, df, n, c);
  }
}

template <typename T>
void fill(hipStream_t s, size_t count, T value, T* p)
{
  if (count) k_fill<T><<<grid_for(count), kBlock, 0, s>>>(p, count, value);
}

template <typename T>
void copy(hipStream_t s, size_t count, const T* src, T* dst)
{
  if (count) k_copy<T><<<grid_for(count), kBlock, 0, s>>>(src, dst, count);
}

void copy_boundary(hipStream_t s, int dim, int n, const double* src, double* dst)
{
  const int bx = n >= 256 ? 256 : 64;
  const dim3 grid(cdiv(n, bx), dim == 3 ? n : 1, 2 * dim);
  k_boundary<<<grid, bx, 0, s>>>(src, dst, dim, n);
}

void zero_boundary(hipStream_t s, int dim, int n, double* p)
{
  copy_boundary(s, dim, n, nullptr, p);
}

// explicit instantiations
template void rbgs_colour<double>(hipStream_t, int, int, double, const double*, const double*, double*, int);
template void rbgs_colour<float>(hipStream_t, int, int, double, const float*, const float*, float*, int);
template void rbgs_first<double>(hipStream_t, int, int, double, const double*, const double*, double*, const double*);
template void rbgs_first<float>(hipStream_t, int, int, double, const float*, const float*, float*, const float*);
template void residual<double>(hipStream_t, int, int, double, const double*, const double*, const double*, double*);
template void residual<float>(hipStream_t, int, int, double, const float*, const float*, const float*, float*);
template void restrict_residual<double>(hipStream_t, int, int, double, const double*, const double*, const double*, double*);
template void restrict_residual<float>(hipStream_t, int, int, double, const float*, const float*, const float*, float*);
template void prolong_add<double>(hipStream_t, int, int, const double*, double*);
template void prolong_add<float>(hipStream_t, int, int, const float*, float*);
template void coarsest_solve<double>(hipStream_t, int, int, const double*, const double*, double*);
template void coarsest_solve<float>(hipStream_t, int, int, const double*, const float*, float*);
template void fill<double>(hipStream_t, size_t, double, double*);
template void fill<float>(hipStream_t, size_t, float, float*);
template void copy<double>(hipStream_t, size_t, const double*, double*);
template void copy<float>(hipStream_t, size_t, const float*, float*);

}  // namespace mgk
