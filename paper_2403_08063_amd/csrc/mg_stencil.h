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

}  // namespace mgk
