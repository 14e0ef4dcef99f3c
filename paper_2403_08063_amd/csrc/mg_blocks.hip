// The 2:1 refined block layout of Sect. 5 and its ghost-layer exchange (Sect. 3: same-level
// copies, F2C linear interpolation, C2F extrapolation of order 0, 1 or 2 with the remapping
// at block edges), behind the C ABI of include/mg_blocks.h, with a damped-Jacobi solver of
// the composite cell-centred system.
//
// The host builds the layout's face table once (per block and face: the kind of neighbour,
// the neighbouring block or blocks and, for C2F, the quadrant of the coarse face); the fill
// kernel runs one thread per ghost cell of every block face and evaluates its rule on the
// fly: the C2F value is the tensor product of three 1D Lagrange weight sets (normal,
// first and second tangential axis), the bases chosen per cell as the rule prescribes.  The
// Jacobi kernel runs one thread per inner cell of all blocks, each block with its own h.
#include "../../include/mg_blocks.h"
#include "mg_kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <new>
#include <tuple>
#include <vector>

namespace {

constexpr int kBlocks = 120;
constexpr int kFaceInts = 8;  // kind, neighbour blocks[4], quadrant s1, s2, pad
constexpr size_t kBlkAlign = 256;
constexpr int kBlkNormBlocks = 1024;
enum { kFaceBoundary = 0, kFaceSame = 1, kFaceF2C = 2, kFaceC2F = 3 };

thread_local char g_blk_err[512] = "no error";

struct BlockDesc {
  int level;  // 2 or 3
  int idx[3];
  double width;
};

std::vector<BlockDesc> build_layout()
{
  std::vector<BlockDesc> out;
  auto refined = [](int i) { return i == 1 || i == 2; };
  for (int bz = 0; bz < 4; ++bz)
    for (int by = 0; by < 4; ++by)
      for (int bx = 0; bx < 4; ++bx)
        if (!(refined(bx) && refined(by) && refined(bz))) out.push_back({2, {bx, by, bz}, 0.25});
  for (int fz = 0; fz < 8; ++fz)
    for (int fy = 0; fy < 8; ++fy)
      for (int fx = 0; fx < 8; ++fx)
        if (refined(fx / 2) && refined(fy / 2) && refined(fz / 2)) out.push_back({3, {fx, fy, fz}, 0.125});
  return out;
}

// face f = 2 * axis + side (axis 0 = x, 1 = y, 2 = z; side 0 = low, 1 = high)
std::vector<int> build_faces(const std::vector<BlockDesc>& blocks)
{
  std::map<std::tuple<int, int, int, int>, int> find;
  for (int b = 0; b < (int)blocks.size(); ++b)
    find[{blocks[b].level, blocks[b].idx[0], blocks[b].idx[1], blocks[b].idx[2]}] = b;
  auto refined2 = [](const int* i) {
    for (int a = 0; a < 3; ++a)
      if (!(i[a] == 1 || i[a] == 2)) return false;
    return true;
  };
  std::vector<int> t(blocks.size() * 6 * kFaceInts, 0);
  for (int b = 0; b < (int)blocks.size(); ++b) {
    const BlockDesc& d = blocks[b];
    for (int ax = 0; ax < 3; ++ax) {
      const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;  // tangential axes, increasing
      for (int side = 0; side < 2; ++side) {
        int* e = &t[((size_t)b * 6 + 2 * ax + side) * kFaceInts];
        int n[3] = {d.idx[0], d.idx[1], d.idx[2]};
        n[ax] += side ? 1 : -1;
        const int per = d.level == 2 ? 4 : 8;
        if (n[ax] < 0 || n[ax] >= per) {
          e[0] = kFaceBoundary;
          continue;
        }
        if (d.level == 2) {
          if (refined2(n)) {
            e[0] = kFaceF2C;
            for (int s1 = 0; s1 < 2; ++s1)
              for (int s2 = 0; s2 < 2; ++s2) {
                int f[3] = {2 * n[0], 2 * n[1], 2 * n[2]};
                f[ax] += side ? 0 : 1;
                f[t0] += s1;
                f[t1] += s2;
                e[1 + 2 * s1 + s2] = find.at({3, f[0], f[1], f[2]});
              }
          } else {
            e[0] = kFaceSame;
            e[1] = find.at({2, n[0], n[1], n[2]});
          }
        } else {
          const int p[3] = {n[0] / 2, n[1] / 2, n[2] / 2};
          if (refined2(p)) {
            e[0] = kFaceSame;
            e[1] = find.at({3, n[0], n[1], n[2]});
          } else {
            e[0] = kFaceC2F;
            e[1] = find.at({2, p[0], p[1], p[2]});
            e[5] = n[t0] % 2;
            e[6] = n[t1] % 2;
          }
        }
      }
    }
  }
  return t;
}

// Lagrange weights of `cnt` bases at `nodes` for target x (host: the C2F weight table)
void lagrange(int cnt, const double* nodes, double x, double* w)
{
  for (int i = 0; i < cnt; ++i) {
    double v = 1.0;
    for (int j = 0; j < cnt; ++j)
      if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    w[i] = v;
  }
}

// C2F weights: along the normal (bases 0, -1, -2 away from the face, target +1/4) and along
// a tangential axis for each choice of the first base (-2, -1, 0) and target (-1/4, +1/4)
struct C2FWeights {
  double wn[3];
  double wt[3][2][3];  // [first base + 2][target: 0 = -1/4, 1 = +1/4][base]
};

C2FWeights c2f_weights(int order)
{
  C2FWeights W{};
  const int cnt = order + 1;
  double nodes[3];
  for (int a = 0; a < cnt; ++a) nodes[a] = -(double)a;
  lagrange(cnt, nodes, 0.25, W.wn);
  for (int first = -2; first <= 0; ++first)
    for (int t = 0; t < 2; ++t) {
      for (int a = 0; a < cnt; ++a) nodes[a] = first + a;
      lagrange(cnt, nodes, t ? 0.25 : -0.25, W.wt[first + 2][t]);
    }
  return W;
}

}  // namespace

struct mgblk_ctx {
  mgblk_grid g{};
  hipStream_t s = nullptr;
  int* faces = nullptr;   // device face table
  double* hs = nullptr;   // device: h of every block
  double* t = nullptr;    // second buffer of the blocks
  double* partial = nullptr;
  double* scal = nullptr;
  size_t cnt = 0;         // doubles of all blocks
  std::vector<double> hhost;
  C2FWeights w{};
  char err[512] = "no error";
};

namespace {

mg_status blk_fail(mgblk_ctx* c, mg_status st, const char* fmt, ...)
{
  char* buf = c ? c->err : g_blk_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
  return st;
}

mg_status blk_validate(const mgblk_grid* g)
{
  if (!g) return blk_fail(nullptr, MG_EINVAL, "grid description is NULL");
  if (g->B < 4 || g->B > 256 || (g->B & 1))
    return blk_fail(nullptr, MG_EINVAL, "B must be even in [4, 256] (got %d)", g->B);
  if (g->order < 0 || g->order > 2) return blk_fail(nullptr, MG_EINVAL, "order must be 0, 1 or 2");
  if (!(g->omega > 0.0 && g->omega < 2.0)) return blk_fail(nullptr, MG_EINVAL, "omega must be in (0, 2)");
  return MG_OK;
}

struct BlkCarver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count)
  {
    off = (off + kBlkAlign - 1) / kBlkAlign * kBlkAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

void blk_layout(const mgblk_grid* g, BlkCarver& cv, mgblk_ctx* c)
{
  const size_t m = (size_t)g->B + 2;
  const size_t cnt = (size_t)kBlocks * m * m * m;
  int* faces = cv.take<int>((size_t)kBlocks * 6 * kFaceInts);
  double* hs = cv.take<double>(kBlocks);
  double* t = cv.take<double>(cnt);
  double* partial = cv.take<double>(kBlkNormBlocks);
  double* scal = cv.take<double>(8);
  if (c) {
    c->faces = faces;
    c->hs = hs;
    c->t = t;
    c->partial = partial;
    c->scal = scal;
    c->cnt = cnt;
  }
}

mg_status blk_hip(mgblk_ctx* c, hipError_t e, const char* what)
{
  if (e == hipSuccess) return MG_OK;
  return blk_fail(c, MG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ size_t bidx(int m, int b, int z, int y, int x)
{
  return (((size_t)b * m + z) * (size_t)m + y) * (size_t)m + x;
}

// (x, y, z) from the index along axis ax and the two tangential indices (increasing axes)
__device__ __forceinline__ void face_coords(int ax, int n, int t1, int t2, int& x, int& y, int& z)
{
  if (ax == 0) { x = n; y = t1; z = t2; }
  else if (ax == 1) { y = n; x = t1; z = t2; }
  else { z = n; x = t1; y = t2; }
}

// first tangential base (offset from coarse index T, 0-based in [0, B)) for the fine position
// on side t (0: -1/4, 1: +1/4)
__device__ __forceinline__ int tangential_first(int order, int T, int B, int t)
{
  if (order == 0) return 0;
  if (order == 1) {
    int a = t ? 0 : -1;
    if (T + a < 0) a = 0;
    if (T + a + 1 >= B) a = -1;
    return a;
  }
  if (T - 1 < 0) return 0;       // the downwind base would be a ghost: remap by -2 o
  if (T + 1 >= B) return -2;     // the upwind one
  return -1;
}

constexpr int kFillThreads = 256;

__global__ void __launch_bounds__(kFillThreads)
    k_blk_fill(int B, int order, C2FWeights W, const int* __restrict__ faces, double* __restrict__ u)
{
  const int m = B + 2;
  const int q = blockIdx.x * kFillThreads + threadIdx.x;  // ghost cell of the face
  if (q >= B * B) return;
  const int f = blockIdx.y, b = blockIdx.z;
  const int ax = f >> 1, side = f & 1;
  const int* e = faces + ((size_t)b * 6 + f) * kFaceInts;
  const int kind = e[0];
  if (kind == kFaceBoundary) return;
  const int t1 = 1 + q % B, t2 = 1 + q / B;
  int gx, gy, gz;
  face_coords(ax, side ? B + 1 : 0, t1, t2, gx, gy, gz);
  const size_t gi = bidx(m, b, gz, gy, gx);
  if (kind == kFaceSame) {
    int x, y, z;
    face_coords(ax, side ? 1 : B, t1, t2, x, y, z);
    u[gi] = u[bidx(m, e[1], z, y, x)];
    return;
  }
  const int half = B / 2;
  if (kind == kFaceF2C) {
    const int s1 = (t1 - 1) / half, s2 = (t2 - 1) / half;
    const int fb = e[1 + 2 * s1 + s2];
    const int f1 = 2 * ((t1 - 1) % half) + 1, f2 = 2 * ((t2 - 1) % half) + 1;
    const int l0 = side ? 1 : B, l1 = side ? 2 : B - 1;
    double s = 0.0;
    for (int li = 0; li < 2; ++li)
      for (int d2 = 0; d2 < 2; ++d2)
        for (int d1 = 0; d1 < 2; ++d1) {
          int x, y, z;
          face_coords(ax, li ? l1 : l0, f1 + d1, f2 + d2, x, y, z);
          s += 0.125 * u[bidx(m, fb, z, y, x)];
        }
    u[gi] = s;
    return;
  }
  // C2F: coarse cell (T1, T2) of the quadrant and the fine position in it
  const int cb = e[1];
  const int T1 = e[5] * half + (t1 - 1) / 2, T2 = e[6] * half + (t2 - 1) / 2;
  const int p1 = (t1 - 1) % 2, p2 = (t2 - 1) % 2;  // 0: -1/4, 1: +1/4
  const int a1 = tangential_first(order, T1, B, p1), a2 = tangential_first(order, T2, B, p2);
  const double* w1 = W.wt[a1 + 2][p1];
  const double* w2 = W.wt[a2 + 2][p2];
  const int cn = order + 1;
  const int ci = side ? 1 : B, away = side ? 1 : -1;
  double s = 0.0;
  for (int a = 0; a < cn; ++a)  // normal bases 0, -1, -2: away from the interface
    for (int j2 = 0; j2 < cn; ++j2)
      for (int j1 = 0; j1 < cn; ++j1) {
        int x, y, z;
        face_coords(ax, ci + away * a, T1 + 1 + a1 + j1, T2 + 1 + a2 + j2, x, y, z);
        s += W.wn[a] * w2[j2] * w1[j1] * u[bidx(m, cb, z, y, x)];
      }
  u[gi] = s;
}

// (A u) at inner cell (z, y, x) of block b: ghost neighbours on the domain boundary as
// 2 g - u_i, the others as stored (filled from the neighbours)
__device__ __forceinline__ double blk_apply_at(int B, const int* __restrict__ fb, double ih2,
                                               const double* __restrict__ u, size_t i, int z,
                                               int y, int x)
{
  const int m = B + 2;
  const size_t sy = (size_t)m, sz = (size_t)m * m;
  const double c = u[i];
  auto v = [&](double nb, bool bnd) { return bnd ? 2.0 * nb - c : nb; };
  const double v0 = v(u[i - 1], x == 1 && fb[0 * kFaceInts] == kFaceBoundary);
  const double v1 = v(u[i + 1], x == B && fb[1 * kFaceInts] == kFaceBoundary);
  const double v2 = v(u[i - sy], y == 1 && fb[2 * kFaceInts] == kFaceBoundary);
  const double v3 = v(u[i + sy], y == B && fb[3 * kFaceInts] == kFaceBoundary);
  const double v4 = v(u[i - sz], z == 1 && fb[4 * kFaceInts] == kFaceBoundary);
  const double v5 = v(u[i + sz], z == B && fb[5 * kFaceInts] == kFaceBoundary);
  double s = c - v0;
  s = s + (c - v1);
  s = s + (c - v2);
  s = s + (c - v3);
  s = s + (c - v4);
  s = s + (c - v5);
  return s * ih2;
}

constexpr int kJacThreads = 64;

__global__ void __launch_bounds__(kJacThreads)
    k_blk_jacobi(int B, double omega, const int* __restrict__ faces, const double* __restrict__ hs,
                 const double* __restrict__ f, const double* __restrict__ u, double* __restrict__ uout)
{
  const int x = 1 + blockIdx.x * kJacThreads + threadIdx.x, y = 1 + blockIdx.y;
  const int b = blockIdx.z / B, z = 1 + blockIdx.z % B;
  if (x > B) return;
  const int m = B + 2;
  const double h = hs[b];
  const size_t i = bidx(m, b, z, y, x);
  const double au = blk_apply_at(B, faces + (size_t)b * 6 * kFaceInts, 1.0 / (h * h), u, i, z, y, x);
  uout[i] = u[i] + omega * (h * h / 6.0) * (f[i] - au);
}

__global__ void __launch_bounds__(256)
    k_blk_norm2(int B, const int* __restrict__ faces, const double* __restrict__ hs,
                const double* __restrict__ f, const double* __restrict__ u,
                double* __restrict__ partial)
{
  __shared__ double part[4];
  const int m = B + 2;
  const size_t total = (size_t)kBlocks * B * B * B;
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int x = 1 + (int)(t % B), y = 1 + (int)((t / B) % B), z = 1 + (int)((t / ((size_t)B * B)) % B);
    const int b = (int)(t / ((size_t)B * B * B));
    const double h = hs[b];
    const size_t i = bidx(m, b, z, y, x);
    const double r = f[i] - blk_apply_at(B, faces + (size_t)b * 6 * kFaceInts, 1.0 / (h * h), u, i, z, y, x);
    acc += r * r;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ void __launch_bounds__(256)
    k_blk_sum(const double* __restrict__ partial, int count, double* __restrict__ out)
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

void fill(mgblk_ctx* c, double* u)
{
  const int B = c->g.B;
  const dim3 grid((unsigned)((B * B + kFillThreads - 1) / kFillThreads), 6, kBlocks);
  k_blk_fill<<<grid, kFillThreads, 0, c->s>>>(B, c->g.order, c->w, c->faces, u);
}

// sweeps with a fill before each, alternating u and the second buffer; returns the result
double* sweeps(mgblk_ctx* c, const double* f, double* u, int count)
{
  const int B = c->g.B;
  const dim3 grid((unsigned)((B + kJacThreads - 1) / kJacThreads), B, kBlocks * B);
  double *cur = u, *oth = c->t;
  for (int s = 0; s < count; ++s) {
    fill(c, cur);
    k_blk_jacobi<<<grid, kJacThreads, 0, c->s>>>(B, c->g.omega, c->faces, c->hs, f, cur, oth);
    double* x = cur;
    cur = oth;
    oth = x;
  }
  return cur;
}

mg_status norm2(mgblk_ctx* c, const double* f, double* u, double* out)
{
  fill(c, u);
  k_blk_norm2<<<kBlkNormBlocks, 256, 0, c->s>>>(c->g.B, c->faces, c->hs, f, u, c->partial);
  k_blk_sum<<<1, 256, 0, c->s>>>(c->partial, kBlkNormBlocks, c->scal);
  if (mg_status st = blk_hip(c, hipGetLastError(), "norm")) return st;
  if (mg_status st = blk_hip(c, hipMemcpyAsync(out, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s),
                             "reading the norm"))
    return st;
  return blk_hip(c, hipStreamSynchronize(c->s), "stream synchronisation");
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int mgblk_block_count(void) { return kBlocks; }

size_t mgblk_workspace_bytes(const mgblk_grid* grid)
{
  if (blk_validate(grid) != MG_OK) return 0;
  BlkCarver cv{nullptr};
  blk_layout(grid, cv, nullptr);
  return cv.off + kBlkAlign;
}

mg_status mgblk_setup(const mgblk_grid* grid, void* workspace, size_t bytes, void* stream,
                      mgblk_ctx** out)
{
  if (!out) return blk_fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (mg_status st = blk_validate(grid)) return st;
  if (!workspace) return blk_fail(nullptr, MG_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kBlkAlign != 0)
    return blk_fail(nullptr, MG_EINVAL, "workspace must be %zu-byte aligned", kBlkAlign);
  const size_t need = mgblk_workspace_bytes(grid);
  if (bytes < need) return blk_fail(nullptr, MG_ENOMEM, "workspace of %zu bytes < %zu required", bytes, need);
  mgblk_ctx* c = new (std::nothrow) mgblk_ctx;
  if (!c) return blk_fail(nullptr, MG_ENOMEM, "host allocation of the context failed");
  c->g = *grid;
  c->s = static_cast<hipStream_t>(stream);
  c->w = c2f_weights(grid->order);
  BlkCarver cv{static_cast<char*>(workspace)};
  blk_layout(grid, cv, c);
  const std::vector<BlockDesc> blocks = build_layout();
  if ((int)blocks.size() != kBlocks) {
    delete c;
    return blk_fail(nullptr, MG_EINVAL, "layout has %zu blocks", blocks.size());
  }
  const std::vector<int> faces = build_faces(blocks);
  c->hhost.resize(kBlocks);
  for (int b = 0; b < kBlocks; ++b) c->hhost[b] = blocks[b].width / grid->B;
  mg_status st = blk_hip(c, hipMemcpyAsync(c->faces, faces.data(), faces.size() * sizeof(int),
                                           hipMemcpyHostToDevice, c->s), "uploading the face table");
  if (!st)
    st = blk_hip(c, hipMemcpyAsync(c->hs, c->hhost.data(), kBlocks * sizeof(double),
                                   hipMemcpyHostToDevice, c->s), "uploading the block widths");
  // the host tables are pageable: finish the copies before they go out of scope
  if (!st) st = blk_hip(c, hipStreamSynchronize(c->s), "setup");
  if (st) {
    snprintf(g_blk_err, sizeof g_blk_err, "%s", c->err);
    delete c;
    return st;
  }
  *out = c;
  return MG_OK;
}

void mgblk_destroy(mgblk_ctx* c) { delete c; }

const char* mgblk_last_error(const mgblk_ctx* c) { return c ? c->err : g_blk_err; }

mg_status mgblk_fill(mgblk_ctx* c, double* u)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!u) return blk_fail(c, MG_EINVAL, "u is NULL");
  fill(c, u);
  return blk_hip(c, hipGetLastError(), "ghost fill");
}

mg_status mgblk_jacobi(mgblk_ctx* c, const double* f, double* u, int count)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u || count < 0) return blk_fail(c, MG_EINVAL, "bad Jacobi arguments");
  mgk::copy<double>(c->s, c->cnt, u, c->t);  // the second buffer's boundary ghosts
  double* r = sweeps(c, f, u, count);
  if (r != u) mgk::copy<double>(c->s, c->cnt, r, u);
  return blk_hip(c, hipGetLastError(), "Jacobi");
}

mg_status mgblk_residual_norm2(mgblk_ctx* c, const double* f, double* u, double* out)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u || !out) return blk_fail(c, MG_EINVAL, "f, u and out must be non-NULL");
  return norm2(c, f, u, out);
}

mg_status mgblk_solve(mgblk_ctx* c, const double* f, double* u, double tol, int max_sweeps,
                      int check_every, int* nsweeps, double* resnorm)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return blk_fail(c, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol >= 0) || max_sweeps < 0 || check_every < 2 || (check_every & 1))
    return blk_fail(c, MG_EINVAL, "tol >= 0, max_sweeps >= 0, check_every even and >= 2");
  mgk::copy<double>(c->s, c->cnt, u, c->t);
  double rn2 = 0;
  mg_status st = norm2(c, f, u, &rn2);
  double rn = std::sqrt(rn2);
  int k = 0;
  while (!st && std::isfinite(rn) && rn > tol && k < max_sweeps) {
    const int n = check_every < max_sweeps - k ? check_every : max_sweeps - k;
    double* r = sweeps(c, f, u, n);
    if (r != u) mgk::copy<double>(c->s, c->cnt, r, u);
    k += n;
    st = norm2(c, f, u, &rn2);
    rn = std::sqrt(rn2);
  }
  if (nsweeps) *nsweeps = k;
  if (resnorm) *resnorm = rn;
  if (st) return st;
  if (!std::isfinite(rn)) return blk_fail(c, MG_ENAN, "residual norm is not finite after %d sweeps", k);
  if (rn > tol) return blk_fail(c, MG_ENOCONV, "residual norm %.3e > tol %.3e after %d sweeps", rn, tol, k);
  return MG_OK;
}

}  // extern "C"
