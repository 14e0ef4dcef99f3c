// Galerkin coarsening of the variable-coefficient operator behind the C ABI of
// include/mg_galerkin.h.  Level 0 runs the 7-point kernels of mg_kernels.hip (red-black
// Gauss-Seidel with face coefficients, residual + full weighting, trilinear prolongation,
// norms); the coarse levels hold 27-point stencils built on the GPU by probing R A P with
// combs of coarse nodes, and run the kernels below: eight-colour Gauss-Seidel, residual with
// full weighting, and the exact solve of the one-node coarsest level.  A coarse level stores
// its stencil colour-major: for each of the eight parity colours, 27 arrays over that colour's
// nodes in C order, so that a colour pass of the smoother reads its coefficients contiguously.
#include "../../include/mg_galerkin.h"
#include "mg_kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>
#include <vector>

namespace {

constexpr size_t kGalAlign = 256;
constexpr int kGalThreads = 256;
constexpr int kCentre = 13;  // stencil array of the node itself: 9 + 3 + 1

thread_local char g_gal_err[512] = "no error";

__device__ __forceinline__ size_t gidx(int n, int z, int y, int x)
{
  return ((size_t)z * n + y) * (size_t)n + x;
}

// Colour-major stencil storage of a level with n nodes per side: half = (n-1)/2 slots per axis
// and colour; interior index v of parity p sits in slot (v - 2 + p) / 2; the coefficient of
// offset o at a node of colour c and slot t is S[(c * 27 + o) * half^3 + t].
__device__ __forceinline__ int colour_of(int z, int y, int x) { return 4 * (z & 1) + 2 * (y & 1) + (x & 1); }

__device__ __forceinline__ size_t slot_of(int half, int z, int y, int x)
{
  const int jz = (z - 2 + (z & 1)) / 2, jy = (y - 2 + (y & 1)) / 2, jx = (x - 2 + (x & 1)) / 2;
  return ((size_t)jz * half + jy) * half + jx;
}

// first coefficient (offset 0) of interior node (z, y, x); offset o at + o * half^3
template <typename TS>
__device__ __forceinline__ const TS* node_coeffs(const TS* S, int half, int z, int y, int x)
{
  const size_t h3 = (size_t)half * half * half;
  return S + (size_t)colour_of(z, y, x) * 27 * h3 + slot_of(half, z, y, x);
}

// (A u)_i - a_ii u_i: the off-diagonal part of the 27-point stencil at interior node i
template <typename TS>
__device__ __forceinline__ double offdiag(const TS* __restrict__ Sn, size_t h3,
                                          const double* __restrict__ u, int n, int z, int y, int x)
{
  double s = 0.0;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    if (o == kCentre) continue;
    const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
    s += (double)Sn[o * h3] * u[gidx(n, z + dz, y + dy, x + dx)];
  }
  return s;
}

// one colour of eight-colour Gauss-Seidel: nodes with parities (pz, py, px) of colour c
template <typename TS>
__global__ void __launch_bounds__(kGalThreads)
    k_gal_gs(int n, const TS* __restrict__ S, const double* __restrict__ f, double* u, int c)
{
  const int half = (n - 1) / 2;
  const int t = blockIdx.x * kGalThreads + threadIdx.x;
  if (t >= half * half * half) return;
  const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
  // interior index with parity p: 2 j + 2 - p  (p = 1: 1, 3, ..; p = 0: 2, 4, ..)
  const int x = 2 * (t % half) + 2 - px, y = 2 * ((t / half) % half) + 2 - py, z = 2 * (t / (half * half)) + 2 - pz;
  if (x > n - 2 || y > n - 2 || z > n - 2) return;
  const size_t h3 = (size_t)half * half * half;
  const TS* Sn = S + (size_t)c * 27 * h3 + t;
  const size_t i = gidx(n, z, y, x);
  u[i] = (f[i] - offdiag(Sn, h3, u, n, z, y, x)) / (double)Sn[kCentre * h3];
}

// r = f - A u at interior nodes (f == nullptr reads 0); the boundary of r is not written
template <typename TS>
__global__ void __launch_bounds__(kGalThreads)
    k_gal_residual(int n, const TS* __restrict__ S, const double* __restrict__ f,
                   const double* __restrict__ u, double* __restrict__ r)
{
  const int m = n - 2;
  const int t = blockIdx.x * kGalThreads + threadIdx.x;
  if (t >= m * m * m) return;
  const int x = 1 + t % m, y = 1 + (t / m) % m, z = 1 + t / (m * m);
  const int half = (n - 1) / 2;
  const size_t h3 = (size_t)half * half * half;
  const TS* Sn = node_coeffs(S, half, z, y, x);
  const size_t i = gidx(n, z, y, x);
  const double au = (double)Sn[kCentre * h3] * u[i] + offdiag(Sn, h3, u, n, z, y, x);
  r[i] = (f ? f[i] : 0.0) - au;
}

// fc = full weighting of r at coarse interior nodes (nf: fine nodes per side)
__global__ void __launch_bounds__(kGalThreads)
    k_gal_fw(int nf, const double* __restrict__ r, double* __restrict__ fc)
{
  const int nc = (nf - 1) / 2 + 1, m = nc - 2;
  const int t = blockIdx.x * kGalThreads + threadIdx.x;
  if (t >= m * m * m) return;
  const int X = 1 + t % m, Y = 1 + (t / m) % m, Z = 1 + t / (m * m);
  double s = 0.0;
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const double w = (oz ? 0.25 : 0.5) * (oy ? 0.25 : 0.5) * (ox ? 0.25 : 0.5);
        s += w * r[gidx(nf, 2 * Z + oz, 2 * Y + oy, 2 * X + ox)];
      }
  fc[gidx(nc, Z, Y, X)] = s;
}

// e = the comb of residue class (cz, cy, cx): 1 at interior nodes J with J_a = c_a mod 3
__global__ void __launch_bounds__(kGalThreads)
    k_gal_comb(int n, int cz, int cy, int cx, double* __restrict__ e)
{
  const size_t t = (size_t)blockIdx.x * kGalThreads + threadIdx.x;
  const size_t cnt = (size_t)n * n * n;
  if (t >= cnt) return;
  const int x = (int)(t % n), y = (int)((t / n) % n), z = (int)(t / ((size_t)n * n));
  const bool in = x > 0 && y > 0 && z > 0 && x < n - 1 && y < n - 1 && z < n - 1;
  e[t] = in && x % 3 == cx && y % 3 == cy && z % 3 == cz ? 1.0 : 0.0;
}

// S[o][I] = -fc[I] at coarse interior nodes, o the offset to I's neighbour of class c
__global__ void __launch_bounds__(kGalThreads)
    k_gal_scatter(int nc, int cz, int cy, int cx, const double* __restrict__ fc,
                  double* __restrict__ S)
{
  const int m = nc - 2;
  const int t = blockIdx.x * kGalThreads + threadIdx.x;
  if (t >= m * m * m) return;
  const int X = 1 + t % m, Y = 1 + (t / m) % m, Z = 1 + t / (m * m);
  auto off = [](int c, int I) { const int r = ((c - I) % 3 + 3) % 3; return r == 2 ? -1 : r; };
  const int o = 9 * (off(cz, Z) + 1) + 3 * (off(cy, Y) + 1) + (off(cx, X) + 1);
  const int half = (nc - 1) / 2;
  const size_t h3 = (size_t)half * half * half;
  const_cast<double*>(node_coeffs(S, half, Z, Y, X))[o * h3] = -fc[gidx(nc, Z, Y, X)];
}

__global__ void __launch_bounds__(kGalThreads)
    k_gal_to_f32(const double* __restrict__ S, float* __restrict__ S32, size_t count)
{
  const size_t t = (size_t)blockIdx.x * kGalThreads + threadIdx.x;
  if (t < count) S32[t] = (float)S[t];
}

// the coarsest level (3^3 nodes): its one interior node (colour 7, slot 0 of one)
__global__ void k_gal_coarsest(const double* __restrict__ S, const double* __restrict__ f,
                               double* __restrict__ u)
{
  const size_t i = gidx(3, 1, 1, 1);
  u[i] = f[i] / node_coeffs(S, 1, 1, 1, 1)[kCentre];
}

// out[o][i] = the stencil in natural layout (27 arrays of n^3 values, 0 off the interior)
__global__ void __launch_bounds__(kGalThreads)
    k_gal_export(int n, const double* __restrict__ S, double* __restrict__ out)
{
  const size_t t = (size_t)blockIdx.x * kGalThreads + threadIdx.x;
  const size_t cnt = (size_t)n * n * n;
  if (t >= cnt) return;
  const int x = (int)(t % n), y = (int)((t / n) % n), z = (int)(t / ((size_t)n * n));
  const bool in = x > 0 && y > 0 && z > 0 && x < n - 1 && y < n - 1 && z < n - 1;
  const int half = (n - 1) / 2;
  const size_t h3 = (size_t)half * half * half;
  const double* Sn = in ? node_coeffs(S, half, z, y, x) : nullptr;
  for (int o = 0; o < 27; ++o) out[o * cnt + t] = in ? Sn[o * h3] : 0.0;
}

unsigned blocks_for(size_t count) { return (unsigned)((count + kGalThreads - 1) / kGalThreads); }

}  // namespace

struct GalLevel {
  int n = 0;
  size_t cnt = 0;
  size_t scnt = 0;      // doubles of the colour-major stencil: 8 colours x 27 x ((n-1)/2)^3
  double* u = nullptr;  // correction (levels >= 1)
  double* f = nullptr;  // right-hand side (levels >= 1)
  double* r = nullptr;  // residual (levels >= 1)
  double* S = nullptr;  // colour-major stencil (levels >= 1)
  float* S32 = nullptr; // its FP32 copy for the cycle (coarse_f32)
};

struct mggal_ctx {
  mggal_grid g{};
  hipStream_t s = nullptr;
  double h = 0;
  double* k = nullptr;      // copy of the coefficient
  double* probe = nullptr;  // level-0 probe vector; the sweeps' second buffer after setup
  double* zero = nullptr;   // level-0 zero right-hand side (probing)
  double* partial = nullptr;
  double* scal = nullptr;
  std::vector<GalLevel> lv;
  char err[512] = "no error";
};

namespace {

mg_status gal_fail(mggal_ctx* c, mg_status st, const char* fmt, ...)
{
  char* buf = c ? c->err : g_gal_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
  return st;
}

mg_status gal_hip(mggal_ctx* c, hipError_t e, const char* what)
{
  if (e == hipSuccess) return MG_OK;
  return gal_fail(c, MG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

mg_status gal_validate(const mggal_grid* g)
{
  if (!g) return gal_fail(nullptr, MG_EINVAL, "grid description is NULL");
  const int n = g->n;
  if (n < 5 || n > 1025 || ((n - 1) & (n - 2)) != 0)
    return gal_fail(nullptr, MG_EINVAL, "n must be 2^m + 1 in [5, 1025] (got %d)", n);
  int nl = n;
  for (int l = 1; l < g->levels; ++l) nl = (nl - 1) / 2 + 1;
  if (g->levels < 2 || nl != 3)
    return gal_fail(nullptr, MG_EINVAL, "levels must reach 3 nodes per side (n=%d, levels=%d)", n, g->levels);
  if (g->nu1 < 0 || g->nu2 < 0) return gal_fail(nullptr, MG_EINVAL, "nu1, nu2 must be >= 0");
  if (g->max_cycles < 1) return gal_fail(nullptr, MG_EINVAL, "max_cycles must be >= 1");
  if (g->coarse_f32 != 0 && g->coarse_f32 != 1) return gal_fail(nullptr, MG_EINVAL, "coarse_f32 must be 0 or 1");
  return MG_OK;
}

struct GalCarver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count)
  {
    off = (off + kGalAlign - 1) / kGalAlign * kGalAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

void gal_layout(const mggal_grid* g, GalCarver& cv, mggal_ctx* c)
{
  const size_t cnt0 = (size_t)g->n * g->n * g->n;
  double* k = cv.take<double>(cnt0);
  double* probe = cv.take<double>(cnt0);
  double* zero = cv.take<double>(cnt0);
  double* partial = cv.take<double>(mgk::kStreamPartials);
  double* scal = cv.take<double>(8);
  std::vector<GalLevel> lv;
  int n = g->n;
  for (int l = 0; l < g->levels; ++l) {
    GalLevel L;
    L.n = n;
    L.cnt = (size_t)n * n * n;
    const size_t half = (size_t)(n - 1) / 2;
    L.scnt = 8 * 27 * half * half * half;
    if (l > 0) {
      L.u = cv.take<double>(L.cnt);
      L.f = cv.take<double>(L.cnt);
      L.r = cv.take<double>(L.cnt);
      L.S = cv.take<double>(L.scnt);
      if (g->coarse_f32) L.S32 = cv.take<float>(L.scnt);
    }
    lv.push_back(L);
    n = (n - 1) / 2 + 1;
  }
  if (c) {
    c->k = k;
    c->probe = probe;
    c->zero = zero;
    c->partial = partial;
    c->scal = scal;
    c->lv = lv;
  }
}

// level 0 on a large grid: the streaming kernels of the rediscretised path
bool fine_tiled(const mggal_ctx* c) { return mgk::rbgs_tiled_supported(3, c->g.n); }

void smooth(mggal_ctx* c, int l, const double* f, double* u, int sweeps)
{
  const GalLevel& L = c->lv[l];
  if (l == 0 && fine_tiled(c)) {
    // one red-black sweep per out-of-place pass, alternating with the second buffer (same
    // boundary values)
    mgk::copy_boundary(c->s, 3, L.n, u, c->probe);
    double *cur = u, *oth = c->probe;
    for (int s = 0; s < sweeps; ++s) {
      mgk::rbgs_tiled<double>(c->s, L.n, c->h, c->k, f, cur, oth, 1, false);
      double* x = cur;
      cur = oth;
      oth = x;
    }
    if (cur != u) mgk::copy<double>(c->s, L.cnt, cur, u);
    return;
  }
  for (int s = 0; s < sweeps; ++s) {
    if (l == 0) {
      mgk::rbgs_colour<double>(c->s, 3, L.n, c->h, c->k, f, u, 0);
      mgk::rbgs_colour<double>(c->s, 3, L.n, c->h, c->k, f, u, 1);
    } else {
      const int half = (L.n - 1) / 2;
      for (int col = 0; col < 8; ++col) {
        const unsigned gb = blocks_for((size_t)half * half * half);
        if (L.S32) k_gal_gs<float><<<gb, kGalThreads, 0, c->s>>>(L.n, L.S32, f, u, col);
        else k_gal_gs<double><<<gb, kGalThreads, 0, c->s>>>(L.n, L.S, f, u, col);
      }
    }
  }
}

// fc (level l+1) = FW(f - A_l u); f == nullptr reads 0
void restrict_to(mggal_ctx* c, int l, const double* f, const double* u, double* fc)
{
  const GalLevel& L = c->lv[l];
  if (l == 0) {
    if (fine_tiled(c)) mgk::restrict_residual_tiled<double>(c->s, L.n, c->h, c->k, f ? f : c->zero, u, fc);
    else mgk::restrict_residual<double>(c->s, 3, L.n, c->h, c->k, f ? f : c->zero, u, fc);
  } else {
    const size_t mf = (size_t)L.n - 2, mc = (size_t)c->lv[l + 1].n - 2;
    // the probes that build the hierarchy always run with the FP64 stencil
    if (L.S32 && f) k_gal_residual<float><<<blocks_for(mf * mf * mf), kGalThreads, 0, c->s>>>(L.n, L.S32, f, u, L.r);
    else k_gal_residual<double><<<blocks_for(mf * mf * mf), kGalThreads, 0, c->s>>>(L.n, L.S, f, u, L.r);
    k_gal_fw<<<blocks_for(mc * mc * mc), kGalThreads, 0, c->s>>>(L.n, L.r, fc);
  }
}

void vcycle_rec(mggal_ctx* c, int l, const double* f, double* u)
{
  const int last = (int)c->lv.size() - 1;
  if (l == last) {
    k_gal_coarsest<<<1, 1, 0, c->s>>>(c->lv[l].S, f, u);
    return;
  }
  smooth(c, l, f, u, c->g.nu1);
  GalLevel& C = c->lv[l + 1];
  restrict_to(c, l, f, u, C.f);
  mgk::fill<double>(c->s, C.cnt, 0.0, C.u);
  vcycle_rec(c, l + 1, C.f, C.u);
  mgk::prolong_add<double>(c->s, 3, C.n, C.u, u);
  smooth(c, l, f, u, c->g.nu2);
}

// Galerkin operator of level l+1 by probing with the 27 combs of coarse nodes
void build_level(mggal_ctx* c, int l)
{
  GalLevel& F = c->lv[l];
  GalLevel& C = c->lv[l + 1];
  double* w = l == 0 ? c->probe : F.u;  // fine probe vector (zero boundary)
  mgk::fill<double>(c->s, C.scnt, 0.0, C.S);
  const size_t m = (size_t)C.n - 2;
  for (int cz = 0; cz < 3; ++cz)
    for (int cy = 0; cy < 3; ++cy)
      for (int cx = 0; cx < 3; ++cx) {
        k_gal_comb<<<blocks_for(C.cnt), kGalThreads, 0, c->s>>>(C.n, cz, cy, cx, C.u);
        mgk::fill<double>(c->s, F.cnt, 0.0, w);
        mgk::prolong_add<double>(c->s, 3, C.n, C.u, w);
        restrict_to(c, l, nullptr, w, C.f);
        k_gal_scatter<<<blocks_for(m * m * m), kGalThreads, 0, c->s>>>(C.n, cz, cy, cx, C.f, C.S);
      }
}

mg_status read_norm2(mggal_ctx* c, const double* f, const double* u, int mode, double* out)
{
  if (fine_tiled(c)) mgk::resid_norm2_tiled(c->s, c->g.n, c->h, c->k, f, u, mode, c->partial, c->scal);
  else mgk::resid_norm2(c->s, 3, c->g.n, c->h, c->k, f, u, mode, c->partial, c->scal);
  if (mg_status st = gal_hip(c, hipGetLastError(), "norm")) return st;
  if (mg_status st = gal_hip(c, hipMemcpyAsync(out, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s),
                             "reading the norm"))
    return st;
  return gal_hip(c, hipStreamSynchronize(c->s), "stream synchronisation");
}

}  // namespace

// ================================================================== C ABI
extern "C" {

size_t mggal_workspace_bytes(const mggal_grid* grid)
{
  if (gal_validate(grid) != MG_OK) return 0;
  GalCarver cv{nullptr};
  gal_layout(grid, cv, nullptr);
  return cv.off + kGalAlign;
}

mg_status mggal_setup(const mggal_grid* grid, const double* k, void* workspace, size_t bytes,
                      void* stream, mggal_ctx** out)
{
  if (!out) return gal_fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (mg_status st = gal_validate(grid)) return st;
  if (!k) return gal_fail(nullptr, MG_EINVAL, "k is NULL");
  if (!workspace) return gal_fail(nullptr, MG_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kGalAlign != 0)
    return gal_fail(nullptr, MG_EINVAL, "workspace must be %zu-byte aligned", kGalAlign);
  const size_t need = mggal_workspace_bytes(grid);
  if (bytes < need) return gal_fail(nullptr, MG_ENOMEM, "workspace of %zu bytes < %zu required", bytes, need);
  mggal_ctx* c = new (std::nothrow) mggal_ctx;
  if (!c) return gal_fail(nullptr, MG_ENOMEM, "host allocation of the context failed");
  c->g = *grid;
  c->s = static_cast<hipStream_t>(stream);
  c->h = 1.0 / (grid->n - 1);
  GalCarver cv{static_cast<char*>(workspace)};
  gal_layout(grid, cv, c);
  mgk::copy<double>(c->s, c->lv[0].cnt, k, c->k);
  mgk::fill<double>(c->s, c->lv[0].cnt, 0.0, c->zero);
  for (size_t l = 1; l < c->lv.size(); ++l) {  // zero boundaries of every coarse array
    mgk::fill<double>(c->s, c->lv[l].cnt, 0.0, c->lv[l].u);
    mgk::fill<double>(c->s, c->lv[l].cnt, 0.0, c->lv[l].f);
    mgk::fill<double>(c->s, c->lv[l].cnt, 0.0, c->lv[l].r);
  }
  for (size_t l = 0; l + 1 < c->lv.size(); ++l) build_level(c, (int)l);
  for (size_t l = 1; l < c->lv.size(); ++l)
    if (c->lv[l].S32)
      k_gal_to_f32<<<blocks_for(c->lv[l].scnt), kGalThreads, 0, c->s>>>(c->lv[l].S, c->lv[l].S32, c->lv[l].scnt);
  mg_status st = gal_hip(c, hipGetLastError(), "building the Galerkin hierarchy");
  if (!st) st = gal_hip(c, hipStreamSynchronize(c->s), "setup");
  if (st) {
    snprintf(g_gal_err, sizeof g_gal_err, "%s", c->err);
    delete c;
    return st;
  }
  *out = c;
  return MG_OK;
}

void mggal_destroy(mggal_ctx* c) { delete c; }

const char* mggal_last_error(const mggal_ctx* c) { return c ? c->err : g_gal_err; }

mg_status mggal_stencil(mggal_ctx* c, int level, double* out)
{
  if (!c) return gal_fail(nullptr, MG_EINVAL, "context is NULL");
  if (level < 1 || level >= (int)c->lv.size()) return gal_fail(c, MG_EINVAL, "level %d has no stencil", level);
  if (!out) return gal_fail(c, MG_EINVAL, "out is NULL");
  const GalLevel& L = c->lv[level];
  k_gal_export<<<blocks_for(L.cnt), kGalThreads, 0, c->s>>>(L.n, L.S, out);
  return gal_hip(c, hipGetLastError(), "exporting the stencil");
}

mg_status mggal_vcycle(mggal_ctx* c, const double* f, double* u)
{
  if (!c) return gal_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return gal_fail(c, MG_EINVAL, "f and u must be non-NULL");
  vcycle_rec(c, 0, f, u);
  return gal_hip(c, hipGetLastError(), "V-cycle");
}

mg_status mggal_solve(mggal_ctx* c, const double* f, double* u, double tol, int* cycles,
                      double* relres)
{
  if (!c) return gal_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return gal_fail(c, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol > 0)) return gal_fail(c, MG_EINVAL, "tol must be > 0");
  double b2 = 0, r2 = 0;
  mg_status st = read_norm2(c, f, u, 1, &b2);
  const double bn = std::sqrt(b2);
  if (!st && !(bn > 0 && std::isfinite(bn))) st = gal_fail(c, MG_EINVAL, "right-hand side norm %.3e", bn);
  int kcyc = 0;
  double rel = 1.0;
  if (!st) st = read_norm2(c, f, u, 0, &r2);
  if (!st) rel = std::sqrt(r2) / bn;
  while (!st && std::isfinite(rel) && rel > tol && kcyc < c->g.max_cycles) {
    vcycle_rec(c, 0, f, u);
    ++kcyc;
    st = read_norm2(c, f, u, 0, &r2);
    rel = std::sqrt(r2) / bn;
  }
  if (cycles) *cycles = kcyc;
  if (relres) *relres = rel;
  if (st) return st;
  if (!std::isfinite(rel)) return gal_fail(c, MG_ENAN, "residual norm is not finite after %d cycles", kcyc);
  if (rel > tol) return gal_fail(c, MG_ENOCONV, "relative residual %.3e > tol %.3e after %d cycles", rel, tol, kcyc);
  return MG_OK;
}

}  // extern "C"
