// Point formulas of the finite-difference operator shared by every kernel, so that all
// kernels evaluate them with the same operations in the same order (bitwise-identical
// results between the straightforward and the temporally blocked kernels).  The library is
// compiled without floating-point contraction.
//
// Operator (paper Sect. 5, Eq. 1; variable coefficients Sect. 7): at an interior node i
// with axis neighbours in the order -x, +x, -y, +y, -z, +z,
//   (A u)_i = (2d u_i - sum_nb u_nb) / h^2                         (constant coefficient)
//   (A u)_i = sum_nb c_nb (u_i - u_nb) / h^2, c_nb = (k_i + k_nb)/2  (variable coefficient)
// Red-black Gauss-Seidel sets u_i to the value that zeroes its own residual.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace mgk {

__device__ __forceinline__ size_t at3(int n, int z, int y, int x)
{
  return ((size_t)z * (size_t)n + (size_t)y) * (size_t)n + (size_t)x;
}

// Gauss-Seidel value, constant coefficient: (h^2 f_i + sum_nb u_nb) * (1/(2d)).
template <typename T, int DIM>
__device__ __forceinline__ T gs_const(T h2f, T xm, T xp, T ym, T yp, T zm, T zp)
{
  T s = xm + xp;
  s = s + ym;
  s = s + yp;
  if (DIM == 3) {
    s = s + zm;
    s = s + zp;
  }
  const T inv = DIM == 3 ? T(1) / T(6) : T(0.25);
  return (h2f + s) * inv;
}

// Gauss-Seidel value, variable coefficient: (h^2 f_i + sum c_nb u_nb) / sum c_nb.
template <typename T, int DIM>
__device__ __forceinline__ T gs_var(T h2f, T ki, T xm, T kxm, T xp, T kxp, T ym, T kym, T yp,
                                    T kyp, T zm, T kzm, T zp, T kzp)
{
  T c = T(0.5) * (ki + kxm);
  T num = c * xm;
  T den = c;
  c = T(0.5) * (ki + kxp);
  num = num + c * xp;
  den = den + c;
  c = T(0.5) * (ki + kym);
  num = num + c * ym;
  den = den + c;
  c = T(0.5) * (ki + kyp);
  num = num + c * yp;
  den = den + c;
  if (DIM == 3) {
    c = T(0.5) * (ki + kzm);
    num = num + c * zm;
    den = den + c;
    c = T(0.5) * (ki + kzp);
    num = num + c * zp;
    den = den + c;
  }
  return (h2f + num) / den;
}

// (A u)_i, constant coefficient.
template <typename T, int DIM>
__device__ __forceinline__ T au_const(T ih2, T ui, T xm, T xp, T ym, T yp, T zm, T zp)
{
  T s = xm + xp;
  s = s + ym;
  s = s + yp;
  if (DIM == 3) {
    s = s + zm;
    s = s + zp;
  }
  return (T(2 * DIM) * ui - s) * ih2;
}

// (A u)_i, variable coefficient.
template <typename T, int DIM>
__device__ __forceinline__ T au_var(T ih2, T ui, T ki, T xm, T kxm, T xp, T kxp, T ym, T kym,
                                    T yp, T kyp, T zm, T kzm, T zp, T kzp)
{
  T s = (T(0.5) * (ki + kxm)) * (ui - xm);
  s = s + (T(0.5) * (ki + kxp)) * (ui - xp);
  s = s + (T(0.5) * (ki + kym)) * (ui - ym);
  s = s + (T(0.5) * (ki + kyp)) * (ui - yp);
  if (DIM == 3) {
    s = s + (T(0.5) * (ki + kzm)) * (ui - zm);
    s = s + (T(0.5) * (ki + kzp)) * (ui - zp);
  }
  return s * ih2;
}

// Residual f_i - (A u)_i at interior node i of an array with strides (1, sy, sz).
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T resid_at(const T* __restrict__ f, const T* __restrict__ u,
                                      const T* __restrict__ k, size_t i, size_t sy, size_t sz,
                                      T ih2)
{
  const T ui = u[i];
  const T xm = u[i - 1], xp = u[i + 1], ym = u[i - sy], yp = u[i + sy];
  const T zm = DIM == 3 ? u[i - sz] : T(0), zp = DIM == 3 ? u[i + sz] : T(0);
  if (!VAR) return f[i] - au_const<T, DIM>(ih2, ui, xm, xp, ym, yp, zm, zp);
  const T kzm = DIM == 3 ? k[i - sz] : T(0), kzp = DIM == 3 ? k[i + sz] : T(0);
  return f[i] - au_var<T, DIM>(ih2, ui, k[i], xm, k[i - 1], xp, k[i + 1], ym, k[i - sy], yp,
                               k[i + sy], zm, kzm, zp, kzp);
}

// Gauss-Seidel value at interior node i read from global memory.
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T gs_at(const T* __restrict__ f, const T* u, const T* __restrict__ k,
                                   size_t i, size_t sy, size_t sz, T h2)
{
  const T xm = u[i - 1], xp = u[i + 1], ym = u[i - sy], yp = u[i + sy];
  const T zm = DIM == 3 ? u[i - sz] : T(0), zp = DIM == 3 ? u[i + sz] : T(0);
  const T h2f = h2 * f[i];
  if (!VAR) return gs_const<T, DIM>(h2f, xm, xp, ym, yp, zm, zp);
  const T kzm = DIM == 3 ? k[i - sz] : T(0), kzp = DIM == 3 ? k[i + sz] : T(0);
  return gs_var<T, DIM>(h2f, k[i], xm, k[i - 1], xp, k[i + 1], ym, k[i - sy], yp, k[i + sy],
                        zm, kzm, zp, kzp);
}

// Gauss-Seidel value at interior node i of a zero iterate: gs_at with every neighbour 0.
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T gs_zero_at(const T* __restrict__ f, const T* __restrict__ k,
                                        size_t i, size_t sy, size_t sz, T h2)
{
  const T h2f = h2 * f[i];
  if (!VAR) return gs_const<T, DIM>(h2f, T(0), T(0), T(0), T(0), T(0), T(0));
  const T kzm = DIM == 3 ? k[i - sz] : T(0), kzp = DIM == 3 ? k[i + sz] : T(0);
  return gs_var<T, DIM>(h2f, k[i], T(0), k[i - 1], T(0), k[i + 1], T(0), k[i - sy], T(0),
                        k[i + sy], T(0), kzm, T(0), kzp);
}

// Full weighting of the fine residual around coarse interior node (X, Y, Z): the 3^d fine
// residuals around 2I combined with weights prod_a w(o_a), w(0) = 1/2, w(+-1) = 1/4, summed
// in the loop order z, y, x.
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T restrict_at(const T* __restrict__ f, const T* __restrict__ u,
                                         const T* __restrict__ k, int nf, T ih2, int X, int Y,
                                         int Z)
{
  const size_t sy = (size_t)nf, sz = (size_t)nf * nf;
  const T w[3] = {T(0.25), T(0.5), T(0.25)};
  T s = T(0);
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const int fz = DIM == 3 ? 2 * Z + oz : 0;
        const size_t i = ((size_t)fz * nf + (2 * Y + oy)) * (size_t)nf + (2 * X + ox);
        const T wt = w[ox + 1] * w[oy + 1] * (DIM == 3 ? w[oz + 1] : T(1));
        s = s + wt * resid_at<T, DIM, VAR>(f, u, k, i, sy, sz, ih2);
      }
  return s;
}

// u += P e for the fine pair x = 2c-1, 2c of row (y, z), c in 1..nc-1: along each axis an
// even index 2I takes coarse I with weight 1, an odd index 2I+1 takes I and I+1 with weight
// 1/2; terms summed in the loop order z, y, x.
template <typename T, int DIM>
__device__ __forceinline__ void prolong_pair(const T* __restrict__ e, T* __restrict__ u, int nc,
                                             int c, int y, int z)
{
  const int nf = 2 * (nc - 1) + 1;
  const int mz = DIM == 3 ? 1 + (z & 1) : 1, my = 1 + (y & 1);
  const int cz0 = DIM == 3 ? z >> 1 : 0, cy0 = y >> 1;
  const T wz = DIM == 3 ? ((z & 1) ? T(0.5) : T(1)) : T(1);
  const T wy = (y & 1) ? T(0.5) : T(1);
  T sodd = T(0), seven = T(0);  // x = 2c-1 and x = 2c
  for (int a = 0; a < mz; ++a)
    for (int b = 0; b < my; ++b) {
      const size_t row = ((size_t)(cz0 + a) * nc + (cy0 + b)) * (size_t)nc;
      const T e0 = e[row + c - 1], e1 = e[row + c];
      sodd = sodd + (wz * wy * T(0.5)) * e0;
      sodd = sodd + (wz * wy * T(0.5)) * e1;
      seven = seven + (wz * wy * T(1)) * e1;
    }
  const size_t i = ((size_t)z * nf + y) * (size_t)nf + (2 * c - 1);
  u[i] = u[i] + sodd;
  if (2 * c <= nf - 2) u[i + 1] = u[i + 1] + seven;
}

// u + P e at fine node (z, y, x) of a level with nf nodes per side (boundary nodes: u): the
// terms prolong_pair adds to that node, in its order.
template <typename T, int DIM>
__device__ __forceinline__ T corrected_at(const T* u, const T* __restrict__ e, int nf, int nc,
                                          int z, int y, int x)
{
  const size_t i = ((size_t)z * nf + y) * (size_t)nf + x;
  if (x < 1 || x > nf - 2 || y < 1 || y > nf - 2 || (DIM == 3 && (z < 1 || z > nf - 2)))
    return u[i];
  const int mz = DIM == 3 ? 1 + (z & 1) : 1, my = 1 + (y & 1);
  const int cz0 = DIM == 3 ? z >> 1 : 0, cy0 = y >> 1;
  const T wz = DIM == 3 ? ((z & 1) ? T(0.5) : T(1)) : T(1);
  const T wy = (y & 1) ? T(0.5) : T(1);
  const int c = (x + 1) >> 1;  // x = 2c-1 (odd) or 2c (even)
  T s = T(0);
  for (int a = 0; a < mz; ++a)
    for (int b = 0; b < my; ++b) {
      const size_t row = ((size_t)(cz0 + a) * nc + (cy0 + b)) * (size_t)nc;
      if (x & 1) {
        s = s + (wz * wy * T(0.5)) * e[row + c - 1];
        s = s + (wz * wy * T(0.5)) * e[row + c];
      } else {
        s = s + (wz * wy * T(1)) * e[row + c];
      }
    }
  return u[i] + s;
}

// Interior unknown q of a level with n nodes per side <-> node (z, y, x), lexicographic.
__device__ __forceinline__ void unknown_to_node(int dim, int n, int q, int& z, int& y, int& x)
{
  const int m1 = n - 2;
  x = 1 + q % m1;
  y = 1 + (q / m1) % m1;
  z = dim == 3 ? 1 + q / (m1 * m1) : 0;
}

// Coarsest solve by one workgroup: b (shared, >= m doubles) = interior of f in double,
// u_q = sum_c ainv[c][q] b_c (ainv symmetric: column access keeps a wavefront's reads
// contiguous).  Ends with the workgroup synchronised.
template <typename T>
__device__ __forceinline__ void coarsest_apply(int dim, int n, const double* __restrict__ ainv,
                                               const T* __restrict__ f, T* __restrict__ u,
                                               double* b)
{
  const int m1 = n - 2;
  const int m = dim == 3 ? m1 * m1 * m1 : m1 * m1;
  for (int q = threadIdx.x; q < m; q += blockDim.x) {
    int z, y, x;
    unknown_to_node(dim, n, q, z, y, x);
    b[q] = (double)f[((size_t)z * n + y) * (size_t)n + x];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < m; q += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += ainv[(size_t)c * m + q] * b[c];
    int z, y, x;
    unknown_to_node(dim, n, q, z, y, x);
    u[((size_t)z * n + y) * (size_t)n + x] = (T)s;
  }
  __syncthreads();
}

}  // namespace mgk
