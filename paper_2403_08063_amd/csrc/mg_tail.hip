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

template <typename T, int DIM, bool VAR>
__device__ void tail_half_sweep(const TailLevel<T>& L, int colour)
{
  const int n = L.n;
  const int half = (n - 1) / 2;  // nodes of one colour in a row, rounded up
  const int rows = DIM == 3 ? (n - 2) * (n - 2) : n - 2;
  const size_t sy = (size_t)n, sz = (size_t)n * n;
  for (int t = threadIdx.x; t < rows * half; t += blockDim.x) {
    const int r = t / half, q = t - r * half;
    const int y = 1 + r % (n - 2);
    const int z = DIM == 3 ? 1 + r / (n - 2) : 0;
    const int x = 1 + ((1 + y + z + colour) & 1) + 2 * q;
    if (x > n - 2) continue;
    const size_t i = ((size_t)z * n + y) * (size_t)n + x;
    L.u[i] = gs_at<T, DIM, VAR>(L.f, L.u, L.k, i, sy, sz, L.h2);
  }
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
    if (var) k_tail<T, 3, true><<<1, kTailThreads, 0, s>>>(a);
    else k_tail<T, 3, false><<<1, kTailThreads, 0, s>>>(a);
  } else {
    if (var) k_tail<T, 2, true><<<1, kTailThreads, 0, s>>>(a);
    else k_tail<T, 2, false><<<1, kTailThreads, 0, s>>>(a);
  }
}

template void tail_cycle<double>(hipStream_t, int, const TailArgs<double>&);
template void tail_cycle<float>(hipStream_t, int, const TailArgs<float>&);

}  // namespace mgk
