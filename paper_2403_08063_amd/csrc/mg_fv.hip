// Cell-centred finite-volume multigrid: the paper's own benchmark solver (Sect. 5: the
// Poisson problem of Eq. 1-2, cell-centred FVM, V(3,3) with a damped Jacobi smoother,
// omega = 0.8, Jacobi also as the coarsest-grid solver; Sect. 6: 256 coarsest iterations)
// on a uniform grid, behind the C ABI of include/mg_fv.h.
//
// Levels of N >= 128 cells per side smooth with the exact-partition streaming pass
// (fv_jacobi_tiled, mg_resid_tiled.hip: one read of u and f and one write per sweep, the
// paper's 24 bytes per cell update); smaller levels with one thread per cell.  The
// transfers run one thread per output cell; the coarsest level runs its fixed number of
// Jacobi iterations inside one workgroup, with the level held in LDS.  Every kernel
// evaluates a cell's update with the operations, in the order, of the plain definition
// (neighbours -x, +x, -y, +y, -z, +z; ghost neighbour 2 g - u_i; N a power of two, so the
// multiplication by 1/h^2 equals the division by h^2).
#include "../../include/mg_fv.h"
#include "mg_kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>

namespace {

constexpr int kFvMaxLevels = 16;
constexpr int kFvMaxN = 2048;
constexpr int kFvCoarseLds = 16;  // coarsest levels up to 16^3 cells run in one workgroup
constexpr size_t kFvAlign = 256;
constexpr int kFvNormBlocks = 1024;

thread_local char g_fv_err[512] = "no error";

struct FvLevel {
  int N = 0;
  size_t cnt = 0;  // (N+2)^3
  double h = 0;
  double *u = nullptr, *f = nullptr, *t = nullptr;
};

}  // namespace

struct mgfv_ctx {
  mgfv_grid g{};
  hipStream_t s = nullptr;
  FvLevel lv[kFvMaxLevels];
  double* partial = nullptr;
  double* scal = nullptr;
  char err[512] = "no error";
};

namespace {

mg_status fv_fail(mgfv_ctx* c, mg_status st, const char* fmt, ...)
{
  char* buf = c ? c->err : g_fv_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
  return st;
}

mg_status fv_validate(const mgfv_grid* g)
{
  if (!g) return fv_fail(nullptr, MG_EINVAL, "grid description is NULL");
  if (g->N < 4 || g->N > kFvMaxN || (g->N & (g->N - 1)) != 0)
    return fv_fail(nullptr, MG_EINVAL, "N must be a power of two in [4, %d] (got %d)", kFvMaxN, g->N);
  if (g->levels < 1 || g->levels > kFvMaxLevels)
    return fv_fail(nullptr, MG_EINVAL, "levels must be in [1, %d] (got %d)", kFvMaxLevels, g->levels);
  if ((g->N >> (g->levels - 1)) < 2)
    return fv_fail(nullptr, MG_EINVAL, "the coarsest level has fewer than 2 cells per side");
  if (g->nu1 < 0 || g->nu2 < 0) return fv_fail(nullptr, MG_EINVAL, "nu1, nu2 must be >= 0");
  if (g->coarse_iters < 0) return fv_fail(nullptr, MG_EINVAL, "coarse_iters must be >= 0");
  if (!(g->omega > 0.0 && g->omega < 2.0))
    return fv_fail(nullptr, MG_EINVAL, "omega must be in (0, 2)");
  if (g->max_cycles < 1) return fv_fail(nullptr, MG_EINVAL, "max_cycles must be >= 1");
  return MG_OK;
}

struct FvCarver {
  char* base;
  size_t off = 0;
  double* take(size_t count)
  {
    off = (off + kFvAlign - 1) / kFvAlign * kFvAlign;
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += count * sizeof(double);
    return p;
  }
};

void fv_layout(const mgfv_grid* g, FvCarver& cv, mgfv_ctx* c)
{
  FvLevel tmp[kFvMaxLevels];
  FvLevel* lv = c ? c->lv : tmp;
  for (int l = 0; l < g->levels; ++l) {
    FvLevel& L = lv[l];
    L.N = g->N >> l;
    L.cnt = (size_t)(L.N + 2) * (L.N + 2) * (L.N + 2);
    L.h = (double)(1 << l) / (double)g->N;
    L.t = cv.take(L.cnt);
    if (l > 0) {
      L.u = cv.take(L.cnt);
      L.f = cv.take(L.cnt);
    }
  }
  double* partial = cv.take(mgk::kStreamPartials);
  double* scal = cv.take(8);
  if (c) {
    c->partial = partial;
    c->scal = scal;
  }
}

mg_status fv_hip(mgfv_ctx* c, hipError_t e, const char* what)
{
  if (e == hipSuccess) return MG_OK;
  return fv_fail(c, MG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

mg_status fv_launch_check(mgfv_ctx* c, const char* what) { return fv_hip(c, hipGetLastError(), what); }

// ---------------------------------------------------------------- per-cell arithmetic
__device__ __forceinline__ size_t fidx(int m, int z, int y, int x)
{
  return ((size_t)z * (size_t)m + (size_t)y) * (size_t)m + (size_t)x;
}

// (A u) at interior cell (z, y, x) of a level with N cells per side
__device__ __forceinline__ double fv_apply_at(int N, double ih2, const double* __restrict__ u,
                                              int z, int y, int x)
{
  const int m = N + 2;
  const size_t i = fidx(m, z, y, x);
  const size_t sy = (size_t)m, sz = (size_t)m * m;
  const double ui = u[i];
  const double v0 = x == 1 ? 2.0 * u[i - 1] - ui : u[i - 1];
  const double v1 = x == N ? 2.0 * u[i + 1] - ui : u[i + 1];
  const double v2 = y == 1 ? 2.0 * u[i - sy] - ui : u[i - sy];
  const double v3 = y == N ? 2.0 * u[i + sy] - ui : u[i + sy];
  const double v4 = z == 1 ? 2.0 * u[i - sz] - ui : u[i - sz];
  const double v5 = z == N ? 2.0 * u[i + sz] - ui : u[i + sz];
  double s = ui - v0;
  s = s + (ui - v1);
  s = s + (ui - v2);
  s = s + (ui - v3);
  s = s + (ui - v4);
  s = s + (ui - v5);
  return s * ih2;
}

// One-thread-per-entry kernels run on a 3D grid: x from blockIdx.x and the thread, y and z
// from blockIdx.y and blockIdx.z (no index division).
constexpr int kFvRowThreads = 128;

dim3 grid3(int xs, int ys, int zs) { return dim3((unsigned)((xs + kFvRowThreads - 1) / kFvRowThreads), ys, zs); }

// zero: u is identically 0, ghost layer included, and is not read (A u = +0)
__global__ void __launch_bounds__(kFvRowThreads)
    k_fv_jacobi(int N, double ih2, double coef, const double* __restrict__ f,
                const double* __restrict__ u, double* __restrict__ uout, int zero)
{
  const int x = 1 + blockIdx.x * kFvRowThreads + threadIdx.x, y = 1 + blockIdx.y, z = 1 + blockIdx.z;
  if (x > N) return;
  const size_t i = fidx(N + 2, z, y, x);
  const double r = f[i] - (zero ? 0.0 : fv_apply_at(N, ih2, u, z, y, x));
  uout[i] = (zero ? 0.0 : u[i]) + coef * r;
}

// r on all (N+2)^3 entries: f - A u on the cells, 0 on the ghost layer
__global__ void __launch_bounds__(kFvRowThreads)
    k_fv_residual(int N, double ih2, const double* __restrict__ f, const double* __restrict__ u,
                  double* __restrict__ r)
{
  const int m = N + 2;
  const int x = blockIdx.x * kFvRowThreads + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= m) return;
  const size_t t = fidx(m, z, y, x);
  const bool cell = x >= 1 && x <= N && y >= 1 && y <= N && z >= 1 && z <= N;
  r[t] = cell ? f[t] - fv_apply_at(N, ih2, u, z, y, x) : 0.0;
}

// fc on all (Nc+2)^3 entries: the mean of the 8 children's residuals, 0 on the ghost layer
__global__ void __launch_bounds__(kFvRowThreads)
    k_fv_restrict(int Nc, double ih2, const double* __restrict__ f, const double* __restrict__ u,
                  double* __restrict__ fc)
{
  const int mc = Nc + 2, N = 2 * Nc, m = N + 2;
  const int X = blockIdx.x * kFvRowThreads + threadIdx.x, Y = blockIdx.y, Z = blockIdx.z;
  if (X >= mc) return;
  const size_t t = fidx(mc, Z, Y, X);
  if (X < 1 || X > Nc || Y < 1 || Y > Nc || Z < 1 || Z > Nc) {
    fc[t] = 0.0;
    return;
  }
  double s = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int z = 2 * Z - 1 + dz, y = 2 * Y - 1 + dy, x = 2 * X - 1 + dx;
        s += f[fidx(m, z, y, x)] - fv_apply_at(N, ih2, u, z, y, x);
      }
  fc[t] = s / 8.0;
}

// coarse correction at (Z, Y, X), possibly in the ghost layer: the homogeneous extension
__device__ __forceinline__ double fv_coarse_value(int Nc, const double* __restrict__ e, int Z,
                                                  int Y, int X)
{
  double sign = 1.0;
  if (Z == 0) { Z = 1; sign = -sign; }
  if (Z == Nc + 1) { Z = Nc; sign = -sign; }
  if (Y == 0) { Y = 1; sign = -sign; }
  if (Y == Nc + 1) { Y = Nc; sign = -sign; }
  if (X == 0) { X = 1; sign = -sign; }
  if (X == Nc + 1) { X = Nc; sign = -sign; }
  return sign * e[fidx(Nc + 2, Z, Y, X)];
}

// u += P e on the fine cells: per axis 3/4 from the parent, 1/4 from its neighbour on the
// fine cell's side.  One thread per fine column pair (2X-1, 2X), the two children of coarse
// column X: they share the parent's y and z weights and need the coarse columns X-1, X, X+1;
// each cell sums its 8 terms in the order z, y, x (parent first).
__global__ void __launch_bounds__(kFvRowThreads)
    k_fv_prolong(int Nc, const double* __restrict__ e, double* __restrict__ u)
{
  const int N = 2 * Nc;
  const int X = 1 + blockIdx.x * kFvRowThreads + threadIdx.x, y = 1 + blockIdx.y, z = 1 + blockIdx.z;
  if (X > Nc) return;
  const int P0 = (z + 1) / 2, P1 = (y + 1) / 2;
  const int Q0 = (z & 1) ? P0 - 1 : P0 + 1, Q1 = (y & 1) ? P1 - 1 : P1 + 1;
  double v[2][2][3];  // [z: parent, side][y: parent, side][x: X-1, X, X+1]
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int d = 0; d < 3; ++d) v[a][b][d] = fv_coarse_value(Nc, e, a ? Q0 : P0, b ? Q1 : P1, X - 1 + d);
  double s0 = 0.0, s1 = 0.0;  // cells 2X-1 (side X-1) and 2X (side X+1)
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
        s0 += w * v[a][b][c ? 0 : 1];
        s1 += w * v[a][b][c ? 2 : 1];
      }
  const size_t i = fidx(N + 2, z, y, 2 * X - 1);
  u[i] += s0;
  u[i + 1] += s1;
}

// per-block sums of (f - A u)^2 over the cells (fixed grid: the summation order does not
// depend on the device), then one fixed-order sum
__global__ void __launch_bounds__(256)
    k_fv_norm2_blocks(int N, double ih2, const double* __restrict__ f, const double* __restrict__ u,
                      double* __restrict__ partial)
{
  __shared__ double part[4];
  const size_t total = (size_t)N * N * N;
  const int lg = __builtin_ctz((unsigned)N);  // N is a power of two
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int x = 1 + (int)(t & (size_t)(N - 1)), y = 1 + (int)((t >> lg) & (size_t)(N - 1));
    const int z = 1 + (int)(t >> (2 * lg));
    const double r = f[fidx(N + 2, z, y, x)] - fv_apply_at(N, ih2, u, z, y, x);
    acc += r * r;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ void __launch_bounds__(256)
    k_fv_sum(const double* __restrict__ partial, int count, double* __restrict__ out)
{
  __shared__ double part[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (part[0] + part[1]) + (part[2] + part[3]);
}

// The coarsest-grid solver: `iters` Jacobi iterations on a level of N <= 16 cells per side
// inside one workgroup, the level (ghosts included) in two LDS buffers.
constexpr int kFvCoarseThreads = 1024;
constexpr int kFvCoarseMax = (kFvCoarseLds + 2) * (kFvCoarseLds + 2) * (kFvCoarseLds + 2);

__global__ void __launch_bounds__(kFvCoarseThreads)
    k_fv_coarse(int N, double ih2, double coef, int iters, const double* __restrict__ f,
                double* __restrict__ u, int zero)
{
  __shared__ double buf[2][kFvCoarseMax];
  const int m = N + 2;
  const int cnt = m * m * m, cells = N * N * N;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) buf[0][i] = buf[1][i] = zero ? 0.0 : u[i];
  __syncthreads();
  int cur = 0;
  for (int it = 0; it < iters; ++it) {
    const double* src = buf[cur];
    double* dst = buf[1 - cur];
    for (int t = threadIdx.x; t < cells; t += blockDim.x) {
      const int x = 1 + t % N, y = 1 + (t / N) % N, z = 1 + t / (N * N);
      const int i = (z * m + y) * m + x;
      const double r = f[i] - fv_apply_at(N, ih2, src, z, y, x);
      dst[i] = src[i] + coef * r;
    }
    __syncthreads();
    cur = 1 - cur;
  }
  for (int t = threadIdx.x; t < cells; t += blockDim.x) {
    const int x = 1 + t % N, y = 1 + (t / N) % N, z = 1 + t / (N * N);
    const int i = (z * m + y) * m + x;
    u[i] = buf[cur][i];
  }
}

// ---------------------------------------------------------------- level operations
double jacobi_coef(const mgfv_ctx* c, const FvLevel& L) { return c->g.omega * (L.h * L.h / 6.0); }

// `sweeps` Jacobi sweeps on level l from u (alternating with t, whose ghost layer equals
// u's); returns the buffer that holds the result.  zero: u is 0 (a coarse level's zero
// correction, ghost layer 0) and is not read: the first sweep reads 0 instead.
double* smooth(mgfv_ctx* c, int l, double* u, double* t, const double* f, int sweeps,
               bool zero = false)
{
  const FvLevel& L = c->lv[l];
  const double ih2 = 1.0 / (L.h * L.h);
  double *cur = u, *oth = t;
  for (int s = 0; s < sweeps; ++s) {
    const bool z0 = zero && s == 0;
    if (mgk::fv_tiled_supported(L.N))
      mgk::fv_jacobi_tiled(c->s, L.N, L.h, c->g.omega, f, cur, oth, c->partial, z0);
    else
      k_fv_jacobi<<<grid3(L.N, L.N, L.N), kFvRowThreads, 0, c->s>>>(L.N, ih2, jacobi_coef(c, L),
                                                                   f, cur, oth, z0 ? 1 : 0);
    double* x = cur;
    cur = oth;
    oth = x;
  }
  return cur;
}

// zero: u is 0 (not read)
void coarse_solve(mgfv_ctx* c, int l, const double* f, double* u, bool zero = false)
{
  const FvLevel& L = c->lv[l];
  const double ih2 = 1.0 / (L.h * L.h);
  if (L.N <= kFvCoarseLds) {
    k_fv_coarse<<<1, kFvCoarseThreads, 0, c->s>>>(L.N, ih2, jacobi_coef(c, L), c->g.coarse_iters, f, u,
                                                   zero ? 1 : 0);
    return;
  }
  if (zero && c->g.coarse_iters == 0) mgk::fill<double>(c->s, L.cnt, 0.0, u);
  double* r = smooth(c, l, u, L.t, f, c->g.coarse_iters, zero);
  if (r != u) mgk::copy<double>(c->s, L.cnt, r, u);
}

// fc = restriction of f - A u; the streaming pass (N >= 128) leaves fc's ghost layer as it
// is (zero in the workspace), the per-cell kernel writes it as 0
void restrict_residual(mgfv_ctx* c, int l, const double* f, const double* u, double* fc)
{
  const FvLevel& L = c->lv[l];
  const int Nc = L.N / 2;
  if (mgk::fv_tiled_supported(L.N)) {
    mgk::fv_restrict_tiled(c->s, L.N, L.h, f, u, fc, c->partial);
    return;
  }
  k_fv_restrict<<<grid3(Nc + 2, Nc + 2, Nc + 2), kFvRowThreads, 0, c->s>>>(Nc, 1.0 / (L.h * L.h),
                                                                          f, u, fc);
}

void prolong(mgfv_ctx* c, int l, const double* ec, double* u)
{
  const FvLevel& L = c->lv[l];
  k_fv_prolong<<<grid3(L.N / 2, L.N, L.N), kFvRowThreads, 0, c->s>>>(L.N / 2, ec, u);
}

void norm2(mgfv_ctx* c, const double* f, const double* u)
{
  const FvLevel& L = c->lv[0];
  if (mgk::fv_tiled_supported(L.N)) {
    mgk::fv_norm2_tiled(c->s, L.N, L.h, f, u, c->partial, c->scal);
    return;
  }
  k_fv_norm2_blocks<<<kFvNormBlocks, 256, 0, c->s>>>(L.N, 1.0 / (L.h * L.h), f, u, c->partial);
  k_fv_sum<<<1, 256, 0, c->s>>>(c->partial, kFvNormBlocks, c->scal);
}

// One V-cycle on level l from (u, t); returns the buffer holding the result.  zero: the
// iterate is 0 (a coarse level's correction, with zero Dirichlet data) and is not read --
// the first sweep starts from 0 instead of a filled array.
double* cycle(mgfv_ctx* c, int l, double* u, double* t, const double* f, bool zero = false)
{
  if (l == c->g.levels - 1) {
    coarse_solve(c, l, f, u, zero);
    return u;
  }
  if (zero && c->g.nu1 == 0) {
    mgk::fill<double>(c->s, c->lv[l].cnt, 0.0, u);
    zero = false;
  }
  double* cur = smooth(c, l, u, t, f, c->g.nu1, zero);
  FvLevel& C = c->lv[l + 1];
  restrict_residual(c, l, f, cur, C.f);
  double* ec = cycle(c, l + 1, C.u, C.t, C.f, true);  // zero correction, zero Dirichlet data
  double* oth = cur == u ? t : u;
  const FvLevel& F = c->lv[l];
  if (c->g.nu2 > 0 && mgk::fv_tiled_supported(F.N)) {
    // the correction enters the first post-smoothing sweep: u + P e is never stored
    mgk::fv_jacobi_prolong_tiled(c->s, F.N, F.h, c->g.omega, f, cur, ec, oth, c->partial);
    return smooth(c, l, oth, cur, f, c->g.nu2 - 1);
  }
  prolong(c, l, ec, cur);
  return smooth(c, l, cur, oth, f, c->g.nu2);
}

mg_status read_norm(mgfv_ctx* c, double* out)
{
  if (mg_status st = fv_hip(c, hipMemcpyAsync(out, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s),
                            "reading the norm"))
    return st;
  return fv_hip(c, hipStreamSynchronize(c->s), "stream synchronisation");
}

mg_status level_args(mgfv_ctx* c, int level, bool coarser)
{
  if (!c) return fv_fail(nullptr, MG_EINVAL, "context is NULL");
  if (level < 0 || level >= c->g.levels || (coarser && level + 1 >= c->g.levels))
    return fv_fail(c, MG_EINVAL, "level %d out of range", level);
  return MG_OK;
}

mg_status vcycle_impl(mgfv_ctx* c, const double* f, double* u)
{
  FvLevel& L0 = c->lv[0];
  mgk::copy_boundary(c->s, 3, L0.N + 2, u, L0.t);
  double* r = cycle(c, 0, u, L0.t, f);
  if (r != u) mgk::copy<double>(c->s, L0.cnt, r, u);
  return fv_launch_check(c, "V-cycle");
}

}  // namespace

// ================================================================== C ABI
extern "C" {

size_t mgfv_workspace_bytes(const mgfv_grid* grid)
{
  if (fv_validate(grid) != MG_OK) return 0;
  FvCarver cv{nullptr};
  fv_layout(grid, cv, nullptr);
  return cv.off + kFvAlign;
}

mg_status mgfv_setup(const mgfv_grid* grid, void* workspace, size_t bytes, void* stream,
                     mgfv_ctx** out)
{
  if (!out) return fv_fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (mg_status st = fv_validate(grid)) return st;
  if (!workspace) return fv_fail(nullptr, MG_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kFvAlign != 0)
    return fv_fail(nullptr, MG_EINVAL, "workspace must be %zu-byte aligned", kFvAlign);
  const size_t need = mgfv_workspace_bytes(grid);
  if (bytes < need)
    return fv_fail(nullptr, MG_ENOMEM, "workspace of %zu bytes < %zu required", bytes, need);
  mgfv_ctx* c = new (std::nothrow) mgfv_ctx;
  if (!c) return fv_fail(nullptr, MG_ENOMEM, "host allocation of the context failed");
  c->g = *grid;
  c->s = static_cast<hipStream_t>(stream);
  FvCarver cv{static_cast<char*>(workspace)};
  fv_layout(grid, cv, c);
  // coarse ghost layers (zero Dirichlet data of the corrections) are never written after this
  mgk::fill<double>(c->s, need / sizeof(double), 0.0, static_cast<double*>(workspace));
  if (mg_status st = fv_launch_check(c, "setup")) {
    snprintf(g_fv_err, sizeof g_fv_err, "%s", c->err);
    delete c;
    return st;
  }
  *out = c;
  return MG_OK;
}

void mgfv_destroy(mgfv_ctx* c) { delete c; }

const char* mgfv_last_error(const mgfv_ctx* c) { return c ? c->err : g_fv_err; }

mg_status mgfv_jacobi(mgfv_ctx* c, int level, const double* f, double* u, int sweeps)
{
  if (mg_status st = level_args(c, level, false)) return st;
  if (!f || !u || sweeps < 0) return fv_fail(c, MG_EINVAL, "bad smoothing arguments");
  FvLevel& L = c->lv[level];
  mgk::copy_boundary(c->s, 3, L.N + 2, u, L.t);
  double* r = smooth(c, level, u, L.t, f, sweeps);
  if (r != u) mgk::copy<double>(c->s, L.cnt, r, u);
  return fv_launch_check(c, "Jacobi");
}

mg_status mgfv_residual(mgfv_ctx* c, int level, const double* f, const double* u, double* r)
{
  if (mg_status st = level_args(c, level, false)) return st;
  if (!f || !u || !r) return fv_fail(c, MG_EINVAL, "f, u and r must be non-NULL");
  const FvLevel& L = c->lv[level];
  k_fv_residual<<<grid3(L.N + 2, L.N + 2, L.N + 2), kFvRowThreads, 0, c->s>>>(L.N, 1.0 / (L.h * L.h),
                                                                             f, u, r);
  return fv_launch_check(c, "residual");
}

mg_status mgfv_restrict_residual(mgfv_ctx* c, int level, const double* f, const double* u,
                                 double* fc)
{
  if (mg_status st = level_args(c, level, true)) return st;
  if (!f || !u || !fc) return fv_fail(c, MG_EINVAL, "f, u and fc must be non-NULL");
  if (mgk::fv_tiled_supported(c->lv[level].N)) mgk::zero_boundary(c->s, 3, c->lv[level + 1].N + 2, fc);
  restrict_residual(c, level, f, u, fc);
  return fv_launch_check(c, "restriction");
}

mg_status mgfv_prolong_correct(mgfv_ctx* c, int level, const double* ec, double* u)
{
  if (mg_status st = level_args(c, level, true)) return st;
  if (!ec || !u) return fv_fail(c, MG_EINVAL, "ec and u must be non-NULL");
  prolong(c, level, ec, u);
  return fv_launch_check(c, "prolongation");
}

mg_status mgfv_coarse_solve(mgfv_ctx* c, const double* f, double* u)
{
  if (!c) return fv_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return fv_fail(c, MG_EINVAL, "f and u must be non-NULL");
  const int l = c->g.levels - 1;
  FvLevel& L = c->lv[l];
  if (L.N > kFvCoarseLds) mgk::copy_boundary(c->s, 3, L.N + 2, u, L.t);
  coarse_solve(c, l, f, u);
  return fv_launch_check(c, "coarsest solve");
}

mg_status mgfv_residual_norm2(mgfv_ctx* c, const double* f, const double* u, double* out)
{
  if (!c) return fv_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u || !out) return fv_fail(c, MG_EINVAL, "f, u and out must be non-NULL");
  norm2(c, f, u);
  if (mg_status st = fv_launch_check(c, "norm")) return st;
  return read_norm(c, out);
}

mg_status mgfv_vcycle(mgfv_ctx* c, const double* f, double* u)
{
  if (!c) return fv_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return fv_fail(c, MG_EINVAL, "f and u must be non-NULL");
  return vcycle_impl(c, f, u);
}

mg_status mgfv_solve(mgfv_ctx* c, const double* f, double* u, double tol, int* cycles,
                     double* resnorm)
{
  if (!c) return fv_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return fv_fail(c, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol >= 0) || !std::isfinite(tol)) return fv_fail(c, MG_EINVAL, "tol must be finite and >= 0");
  double rn2 = 0;
  norm2(c, f, u);
  mg_status st = fv_launch_check(c, "norm");
  if (!st) st = read_norm(c, &rn2);
  double rn = std::sqrt(rn2);
  int k = 0;
  while (!st && std::isfinite(rn) && rn > tol && k < c->g.max_cycles) {
    if ((st = vcycle_impl(c, f, u))) break;
    ++k;
    norm2(c, f, u);
    if ((st = fv_launch_check(c, "norm"))) break;
    if ((st = read_norm(c, &rn2))) break;
    rn = std::sqrt(rn2);
  }
  if (cycles) *cycles = k;
  if (resnorm) *resnorm = rn;
  if (st) return st;
  if (!std::isfinite(rn)) return fv_fail(c, MG_ENAN, "residual norm is not finite after %d cycles", k);
  if (rn > tol)
    return fv_fail(c, MG_ENOCONV, "residual norm %.3e > tol %.3e after %d cycles", rn, tol, k);
  return MG_OK;
}

}  // extern "C"
