// Coarse tail of the V-cycle in one launch.
//
// Below a few ten thousand interior nodes per level a kernel launch costs more than the
// work it carries (the V-cycle's coarse levels are launch-latency bound, the GPU analogue
// of the coarse-grid overhead the paper measures in Sect. 6).  One workgroup of 1024
// threads therefore runs the complete V(nu1, nu2)-cycle on all levels from `first` down to
// the coarsest, with workgroup barriers between the dependent phases: zero guess,
// red-black half-sweeps, residual + full-weighting restriction, the coarsest solve,
// prolongation + correction, post-smoothing.  Every phase evaluates the same point
// formulas in the same order as the multi-kernel path (mg_stencil.h), so the result is
// bitwise identical to launching the per-level kernels.
#include "mg_kernels.h"
#include "mg_stencil.h"

namespace mgk {
namespace {

constexpr int kTailThreads = 1024;

// Work items of a phase: an nx x ny (x nz) box, enumerated over power-of-two padded x and
// y extents so that a thread index splits into coordinates by shifts and masks (an integer
// division costs tens of instructions, more than a tail phase's arithmetic).
__device__ __forceinline__ int ceil_log2(int v) { return v <= 1 ? 0 : 32 - __clz(v - 1); }

template <typename F>
__device__ __forceinline__ void for_box(int nx, int ny, int nz, F&& body)
{
  const int lx = ceil_log2(nx), ly = ceil_log2(ny);
  const int total = (1 << (lx + ly)) * nz;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int x = t & ((1 << lx) - 1), y = (t >> lx) & ((1 << ly) - 1), z = t >> (lx + ly);
    if (x < nx && y < ny) body(x, y, z);
  }
}

template <typename T, int DIM, bool VAR>
__device__ void tail_half_sweep(const TailLevel<T>& L, int colour)
{
  const int n = L.n;
  const int half = (n - 1) / 2;  // nodes of one colour in a row, rounded up
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  for_box(half, n - 2, DIM == 3 ? n - 2 : 1, [&](int q, int yy, int zz) {
    const int y = 1 + yy;
    const int z = DIM == 3 ? 1 + zz : 0;
    const int x = 1 + ((1 + y + z + colour) & 1) + 2 * q;
    if (x > n - 2) return;
    const size_t i = ((size_t)z * n + y) * (size_t)n + x;
    L.u[i] = gs_at<T, DIM, VAR>(L.f, L.u, L.k, i, sy, sz, L.h2);
  });
  __syncthreads();
}

template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kTailThreads) k_tail(TailArgs<T> a)
{
  __shared__ double b[1024];
  const int last = a.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const TailLevel<T>& L = a.lv[l];
    const size_t N = DIM == 3 ? (size_t)L.n * L.n * L.n : (size_t)L.n * L.n;
    for (size_t i = threadIdx.x; i < N; i += blockDim.x) L.u[i] = T(0);
    __syncthreads();
    for (int s = 0; s < a.nu1; ++s) {
      tail_half_sweep<T, DIM, VAR>(L, 0);
      tail_half_sweep<T, DIM, VAR>(L, 1);
    }
    const TailLevel<T>& C = a.lv[l + 1];
    const int nc = C.n, mc = nc - 2;
    const int cnt = DIM == 3 ? mc * mc * mc : mc * mc;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int X = 1 + t % mc;
      const int Y = 1 + (t / mc) % mc;
      const int Z = DIM == 3 ? 1 + t / (mc * mc) : 0;
      C.f[((size_t)Z * nc + Y) * (size_t)nc + X] =
          restrict_at<T, DIM, VAR>(L.f, L.u, L.k, L.n, L.ih2, X, Y, Z);
    }
    __syncthreads();
  }
  coarsest_apply<T>(DIM, a.lv[last].n, a.ainv, a.lv[last].f, a.lv[last].u, b);
  for (int l = last - 1; l >= 0; --l) {
    const TailLevel<T>& L = a.lv[l];
    const TailLevel<T>& C = a.lv[l + 1];
    const int nc = C.n, mf = L.n - 2;
    const int rows = DIM == 3 ? mf * mf : mf;
    const int pairs = nc - 1;
    for (int t = threadIdx.x; t < rows * pairs; t += blockDim.x) {
      const int r = t / pairs, c = 1 + (t - r * pairs);
      const int y = 1 + r % mf;
      const int z = DIM == 3 ? 1 + r / mf : 0;
      prolong_pair<T, DIM>(C.u, L.u, nc, c, y, z);
    }
    __syncthreads();
    for (int s = 0; s < a.nu2; ++s) {
      tail_half_sweep<T, DIM, VAR>(L, 0);
      tail_half_sweep<T, DIM, VAR>(L, 1);
    }
  }
}

// The same cycle with the levels staged in LDS (dynamic): per level u, f and, with a
// variable coefficient, k (n^dim values each, in that order).  Every dependent phase then
// reads LDS instead of L2 after its barrier; the staging copies the first level's f and
// every level's k, zeroes every u (the zero guesses, boundaries included), and the first
// level's u is written back at the end.
template <typename T, int DIM, bool VAR>
__device__ __forceinline__ TailLevel<T> lds_level(unsigned char* base, const TailArgs<T>& a, int l)
{
  size_t off = 0;
  for (int q = 0; q < l; ++q) {
    const size_t n = (size_t)a.lv[q].n;
    off += (DIM == 3 ? n * n * n : n * n) * (VAR ? 3 : 2);
  }
  const size_t n = (size_t)a.lv[l].n;
  const size_t N = DIM == 3 ? n * n * n : n * n;
  T* p = reinterpret_cast<T*>(base) + off;
  return {p, p + N, VAR ? p + 2 * N : nullptr, a.lv[l].n, a.lv[l].h2, a.lv[l].ih2};
}

template <typename T, int DIM, bool VAR>
__global__ void __launch_bounds__(kTailThreads) k_tail_lds(TailArgs<T> a)
{
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ double b[1024];
  const int last = a.nlev - 1;
  for (int l = 0; l <= last; ++l) {
    const TailLevel<T> L = lds_level<T, DIM, VAR>(tail_lds, a, l);
    const TailLevel<T>& G = a.lv[l];
    const size_t N = DIM == 3 ? (size_t)L.n * L.n * L.n : (size_t)L.n * L.n;
    for (size_t i = threadIdx.x; i < N; i += blockDim.x) {
      L.u[i] = T(0);
      L.f[i] = l == 0 ? G.f[i] : T(0);
      if constexpr (VAR) const_cast<T*>(L.k)[i] = G.k[i];
    }
  }
  __syncthreads();
  for (int l = 0; l < last; ++l) {
    const TailLevel<T> L = lds_level<T, DIM, VAR>(tail_lds, a, l);
    for (int s = 0; s < a.nu1; ++s) {
      tail_half_sweep<T, DIM, VAR>(L, 0);
      tail_half_sweep<T, DIM, VAR>(L, 1);
    }
    const TailLevel<T> C = lds_level<T, DIM, VAR>(tail_lds, a, l + 1);
    const int nc = C.n, mc = nc - 2;
    for_box(mc, mc, DIM == 3 ? mc : 1, [&](int xx, int yy, int zz) {
      const int X = 1 + xx, Y = 1 + yy, Z = DIM == 3 ? 1 + zz : 0;
      C.f[((size_t)Z * nc + Y) * (size_t)nc + X] =
          restrict_at<T, DIM, VAR>(L.f, L.u, L.k, L.n, L.ih2, X, Y, Z);
    });
    __syncthreads();
  }
  {
    const TailLevel<T> Lc = lds_level<T, DIM, VAR>(tail_lds, a, last);
    coarsest_apply<T>(DIM, Lc.n, a.ainv, Lc.f, Lc.u, b);
  }
  for (int l = last - 1; l >= 0; --l) {
    const TailLevel<T> L = lds_level<T, DIM, VAR>(tail_lds, a, l);
    const TailLevel<T> C = lds_level<T, DIM, VAR>(tail_lds, a, l + 1);
    const int nc = C.n, mf = L.n - 2;
    for_box(nc - 1, mf, DIM == 3 ? mf : 1, [&](int cc, int yy, int zz) {
      prolong_pair<T, DIM>(C.u, L.u, nc, 1 + cc, 1 + yy, DIM == 3 ? 1 + zz : 0);
    });
    __syncthreads();
    for (int s = 0; s < a.nu2; ++s) {
      tail_half_sweep<T, DIM, VAR>(L, 0);
      tail_half_sweep<T, DIM, VAR>(L, 1);
    }
  }
  const TailLevel<T> L0 = lds_level<T, DIM, VAR>(tail_lds, a, 0);
  const size_t N0 = DIM == 3 ? (size_t)L0.n * L0.n * L0.n : (size_t)L0.n * L0.n;
  for (size_t i = threadIdx.x; i < N0; i += blockDim.x) a.lv[0].u[i] = L0.u[i];
}

// LDS of the staged levels, bytes
template <typename T>
size_t tail_lds_bytes(int dim, const TailArgs<T>& a)
{
  const bool var = a.lv[0].k != nullptr;
  size_t vals = 0;
  for (int q = 0; q < a.nlev; ++q) {
    const size_t n = (size_t)a.lv[q].n;
    vals += (dim == 3 ? n * n * n : n * n) * (var ? 3 : 2);
  }
  return vals * sizeof(T);
}

// dynamic LDS the staged tail may take next to its static 8 KB (gfx950: 160 KB per CU)
constexpr size_t kTailLdsMax = 144 * 1024;

template <typename Kernel>
bool allow_lds(Kernel kern, size_t bytes)
{
  if (bytes > kTailLdsMax) return false;
  static int granted[64] = {0};  // per device: 1 granted, -1 refused
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  if (granted[dev] == 0)
    granted[dev] = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kTailLdsMax) == hipSuccess ? 1 : -1;
  return granted[dev] == 1;
}

template <typename T, int DIM, bool VAR>
void launch_tail(hipStream_t s, const TailArgs<T>& a)
{
  const size_t bytes = tail_lds_bytes<T>(DIM, a);
  auto kl = k_tail_lds<T, DIM, VAR>;
  if (allow_lds(kl, bytes)) kl<<<1, kTailThreads, bytes, s>>>(a);
  else k_tail<T, DIM, VAR><<<1, kTailThreads, 0, s>>>(a);
}

}  // namespace

bool tail_fits(int dim, int n)
{
  const long long m = n - 2;
  return (dim == 3 ? m * m * m : m * m) <= kTailMaxNodes;
}

template <typename T>
void tail_cycle(hipStream_t s, int dim, const TailArgs<T>& a)
{
  const bool var = a.lv[0].k != nullptr;
  if (dim == 3) {
    if (var) launch_tail<T, 3, true>(s, a);
    else launch_tail<T, 3, false>(s, a);
  } else {
    if (var) launch_tail<T, 2, true>(s, a);
    else launch_tail<T, 2, false>(s, a);
  }
}

template void tail_cycle<double>(hipStream_t, int, const TailArgs<double>&);
template void tail_cycle<float>(hipStream_t, int, const TailArgs<float>&);

}  // namespace mgk
