// The 2:1 refined block layout of Sect. 5 and its ghost-layer exchange (Sect. 3: same-level
// copies, F2C linear interpolation, C2F extrapolation of order 0, 1 or 2 with the remapping
// at block edges), behind the C ABI of include/mg_blocks.h, with a damped-Jacobi solver of
// the composite cell-centred system: plain sweeps, or V-cycles over levels of the same layout
// with B/2^l cells per block (Sect. 5's solver: damped Jacobi as smoother and coarsest solver).
//
// The host builds the layout's face table once (per block and face: the kind of neighbour,
// the neighbouring block or blocks and, for C2F, the quadrant of the coarse face); the fill
// kernel runs one thread per ghost cell of every block face and evaluates its rule on the
// fly: the C2F value is the tensor product of three 1D Lagrange weight sets (normal,
// first and second tangential axis), the bases chosen per cell as the rule prescribes.  The
// Jacobi kernel runs one thread per inner cell of all blocks, each block with its own h; the
// restriction one thread per coarse cell (its 8 children's residuals, mean), the
// prolongation one thread per fine cell (parent and three face neighbours, weight 1/4 each).
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

// one level of the hierarchy: B cells per block; u, f only below the finest level (the
// caller owns the finest level's arrays), t the second buffer of the Jacobi sweeps
struct BlkLevel {
  int B = 0;
  size_t cnt = 0;         // doubles of all blocks
  double* hs = nullptr;   // device: h of every block
  double* u = nullptr;
  double* t = nullptr;
  double* f = nullptr;
};

struct mgblk_ctx {
  mgblk_grid g{};
  hipStream_t s = nullptr;
  int* faces = nullptr;   // device face table
  double* partial = nullptr;
  double* scal = nullptr;
  std::vector<BlkLevel> lv;
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
  if (g->levels < 0 || g->levels > 8) return blk_fail(nullptr, MG_EINVAL, "levels must be in [0, 8]");
  for (int l = 1, b = g->B; l < g->levels; ++l, b /= 2)
    if (b % 4 || b / 2 < 4)
      return blk_fail(nullptr, MG_EINVAL, "B=%d has no %d levels of even block sizes >= 4", g->B, g->levels);
  if (g->nu1 < 0 || g->nu2 < 0 || g->coarse_iters < 0)
    return blk_fail(nullptr, MG_EINVAL, "nu1, nu2 and coarse_iters must be >= 0");
  if (g->max_cycles < 1) return blk_fail(nullptr, MG_EINVAL, "max_cycles must be >= 1");
  return MG_OK;
}

// block sizes of the levels: `levels` of them, or (0) halving while the half is even and >= 4
std::vector<int> level_sizes(const mgblk_grid* g)
{
  std::vector<int> out{g->B};
  if (g->levels == 0) {
    while (out.back() % 4 == 0 && out.back() / 2 >= 4) out.push_back(out.back() / 2);
  } else {
    while ((int)out.size() < g->levels) out.push_back(out.back() / 2);
  }
  return out;
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
  int* faces = cv.take<int>((size_t)kBlocks * 6 * kFaceInts);
  double* partial = cv.take<double>(kBlkNormBlocks);
  double* scal = cv.take<double>(8);
  std::vector<BlkLevel> lv;
  for (int B : level_sizes(g)) {
    BlkLevel L;
    const size_t m = (size_t)B + 2;
    L.B = B;
    L.cnt = (size_t)kBlocks * m * m * m;
    L.hs = cv.take<double>(kBlocks);
    L.t = cv.take<double>(L.cnt);
    if (!lv.empty()) {
      L.u = cv.take<double>(L.cnt);
      L.f = cv.take<double>(L.cnt);
    }
    lv.push_back(L);
  }
  if (c) {
    c->faces = faces;
    c->partial = partial;
    c->scal = scal;
    c->lv = lv;
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
// (selects, not stores through a reference chosen by ax: those end up in per-lane scratch)
__device__ __forceinline__ void face_coords(int ax, int n, int t1, int t2, int& x, int& y, int& z)
{
  x = ax == 0 ? n : t1;
  y = ax == 1 ? n : (ax == 0 ? t1 : t2);
  z = ax == 2 ? n : t2;
}

// first tangential base (offset from coarse index T, 0-based in [0, B)) for the fine position
// on side t (0: -1/4, 1: +1/4)
__device__ __forceinline__ int tangential_first(int order, int T, int B, int t)
{
  if (order == 0) return 0;
  if (order == 1) return T - 1 < 0 ? 0 : -1;  // the cell and its downwind neighbour, remapped
                                              // to the upwind one at the block's lower edge
  if (T - 1 < 0) return 0;       // the downwind base would be a ghost: remap by -2 o
  if (T + 1 >= B) return -2;     // the upwind one
  return -1;
}

// value of the interface ghost cell (t1, t2) of face (ax, side) with face-table entry e (kind
// same, F2C or C2F), from the neighbouring blocks' inner cells read through rd(b, z, y, x).
// The C2F order is a compile-time constant, so that the (order+1)^3 terms unroll and their
// loads are issued together instead of one round trip after another.
template <int ORDER, class Rd>
__device__ __forceinline__ double interface_ghost(const Rd& rd, int B, const C2FWeights& W,
                                                  const int* e, int ax, int side, int t1, int t2)
{
  constexpr int order = ORDER;
  const int kind = e[0];
  if (kind == kFaceSame) {
    int x, y, z;
    face_coords(ax, side ? 1 : B, t1, t2, x, y, z);
    return rd(e[1], z, y, x);
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
          s += 0.125 * rd(fb, z, y, x);
        }
    return s;
  }
  // C2F: coarse cell (T1, T2) of the quadrant and the fine position in it
  const int cb = e[1];
  const int T1 = e[5] * half + (t1 - 1) / 2, T2 = e[6] * half + (t2 - 1) / 2;
  const int p1 = (t1 - 1) % 2, p2 = (t2 - 1) % 2;  // 0: -1/4, 1: +1/4
  const int a1 = tangential_first(order, T1, B, p1), a2 = tangential_first(order, T2, B, p2);
  const double* w1 = W.wt[a1 + 2][p1];
  const double* w2 = W.wt[a2 + 2][p2];
  constexpr int cn = order + 1;
  const int ci = side ? 1 : B, away = side ? 1 : -1;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < cn; ++a)  // normal bases 0, -1, -2: away from the interface
#pragma unroll
    for (int j2 = 0; j2 < cn; ++j2)
#pragma unroll
      for (int j1 = 0; j1 < cn; ++j1) {
        int x, y, z;
        face_coords(ax, ci + away * a, T1 + 1 + a1 + j1, T2 + 1 + a2 + j2, x, y, z);
        s += W.wn[a] * w2[j2] * w1[j1] * rd(cb, z, y, x);
      }
  return s;
}

constexpr int kFillThreads = 256;

// ghost cell q (0 .. B^2-1) of face f of block b: filled by its rule unless the face lies on
// the domain boundary
template <int ORDER>
__device__ __forceinline__ void fill_ghost(int B, const C2FWeights& W,
                                           const int* __restrict__ faces, double* __restrict__ u,
                                           int q, int f, int b)
{
  const int m = B + 2;
  const int* e = faces + ((size_t)b * 6 + f) * kFaceInts;
  if (e[0] == kFaceBoundary) return;
  const int t1 = 1 + q % B, t2 = 1 + q / B;
  int gx, gy, gz;
  face_coords(f >> 1, (f & 1) ? B + 1 : 0, t1, t2, gx, gy, gz);
  auto rd = [&](int bb, int z, int y, int x) { return u[bidx(m, bb, z, y, x)]; };
  u[bidx(m, b, gz, gy, gx)] = interface_ghost<ORDER>(rd, B, W, e, f >> 1, f & 1, t1, t2);
}

template <int ORDER>
__global__ void __launch_bounds__(kFillThreads)
    k_blk_fill(int B, C2FWeights W, const int* __restrict__ faces, double* __restrict__ u)
{
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // ghost cell of the face
  if (q >= B * B) return;
  fill_ghost<ORDER>(B, W, faces, u, q, blockIdx.y, blockIdx.z);
}

// (A u) at inner cell (z, y, x) of block b from the six stored neighbours: interface ghosts
// filled from the neighbouring blocks; on the solution level the domain-boundary ghosts hold
// the Dirichlet data at their own centres and are read as stored (Sect. 5; the reading under
// which Table 1's errors are reproduced), on the correction levels (coarse) the correction
// vanishes on the boundary face: such a ghost enters as 2 g - u_i with its stored g = 0
__device__ __forceinline__ double blk_apply_at(int B, const int* __restrict__ fb, double ih2,
                                               const double* __restrict__ u, size_t i, int z,
                                               int y, int x, bool coarse)
{
  const int m = B + 2;
  const size_t sy = (size_t)m, sz = (size_t)m * m;
  const double c = u[i];
  auto v = [&](double nb, bool bnd) { return (coarse && bnd) ? 2.0 * nb - c : nb; };
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

// (A u) at a cell from its value c and its six neighbours' values v (-x, +x, -y, +y, -z, +z),
// as blk_apply_at forms it; bnd bit a: neighbour a is a domain-boundary ghost
__device__ __forceinline__ double blk_apply_vals(double ih2, double c, const double (&v)[6],
                                                 unsigned bnd, bool coarse)
{
  double w[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) w[a] = (coarse && ((bnd >> a) & 1u)) ? 2.0 * v[a] - c : v[a];
  double s = c - w[0];
  s = s + (c - w[1]);
  s = s + (c - w[2]);
  s = s + (c - w[3]);
  s = s + (c - w[4]);
  s = s + (c - w[5]);
  return s * ih2;
}

// One thread per inner cell of all blocks of size B, 256 threads per workgroup: for B >= 64
// a workgroup covers 64 x 4 cells of an (x, y) plane (grid: x tiles, y tiles, blocks x B
// planes); for smaller blocks a flat index over the blocks' cells (B^3 >= 64 cells a block).
constexpr int kCellThreads = 256;
constexpr int kCellRowsMin = 64;

dim3 cell_grid(int B)
{
  if (B >= kCellRowsMin) return dim3((unsigned)((B + 63) / 64), (unsigned)((B + 3) / 4), (unsigned)(kBlocks * B));
  const size_t cells = (size_t)kBlocks * B * B * B;
  return dim3((unsigned)((cells + kCellThreads - 1) / kCellThreads), 1, 1);
}

// 1-based inner coordinates of this thread's cell; false past the end
__device__ __forceinline__ bool cell_of(int B, int& b, int& z, int& y, int& x)
{
  if (B >= kCellRowsMin) {
    x = 1 + blockIdx.x * 64 + (threadIdx.x & 63);
    y = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
    b = blockIdx.z / B;
    z = 1 + blockIdx.z % B;
    return x <= B && y <= B;
  }
  const int n2 = B * B, n3 = n2 * B;
  const int t = blockIdx.x * kCellThreads + threadIdx.x;
  if (t >= kBlocks * n3) return false;
  b = t / n3;
  int r = t - b * n3;
  const int zz = r / n2;
  r -= zz * n2;
  const int yy = r / B;
  z = 1 + zz;
  y = 1 + yy;
  x = 1 + r - yy * B;
  return true;
}

// the damped Jacobi update of inner cell (z, y, x) of block b, u -> uout
__device__ __forceinline__ void jacobi_cell(int B, double omega, const int* __restrict__ faces,
                                            const double* __restrict__ hs,
                                            const double* __restrict__ f,
                                            const double* __restrict__ u,
                                            double* __restrict__ uout, bool coarse, int b, int z,
                                            int y, int x)
{
  const int m = B + 2;
  const double h = hs[b];
  const size_t i = bidx(m, b, z, y, x);
  const double au = blk_apply_at(B, faces + (size_t)b * 6 * kFaceInts, 1.0 / (h * h), u, i, z, y, x,
                                 coarse);
  uout[i] = u[i] + omega * (h * h / 6.0) * (f[i] - au);
}

// jacobi_cell of an identically zero u: the same operations on literal zeros (the ghost
// values of a zero u are 0 too: linear rules, and a zero Dirichlet g on a coarse level)
__device__ __forceinline__ void jacobi_cell_zero(int B, double omega,
                                                 const double* __restrict__ hs,
                                                 const double* __restrict__ f,
                                                 double* __restrict__ uout, bool coarse, int b,
                                                 int z, int y, int x)
{
  const int m = B + 2;
  const double h = hs[b];
  const size_t i = bidx(m, b, z, y, x);
  const double zero[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double au = blk_apply_vals(1.0 / (h * h), 0.0, zero, 0u, coarse);
  uout[i] = 0.0 + omega * (h * h / 6.0) * (f[i] - au);
}

__global__ void __launch_bounds__(kCellThreads)
    k_blk_jacobi(int B, double omega, const int* __restrict__ faces, const double* __restrict__ hs,
                 const double* __restrict__ f, const double* __restrict__ u, double* __restrict__ uout,
                 int coarse, int zero)
{
  int b, z, y, x;
  if (!cell_of(B, b, z, y, x)) return;
  if (zero) jacobi_cell_zero(B, omega, hs, f, uout, coarse != 0, b, z, y, x);
  else jacobi_cell(B, omega, faces, hs, f, u, uout, coarse != 0, b, z, y, x);
}

// Damped-Jacobi sweep of a level of small blocks (B <= kSmallB) in one launch, one workgroup
// per block: workgroup b fills block b's interface ghosts of u from the neighbouring blocks'
// inner cells (which no workgroup writes in this launch), then, after a barrier, sweeps
// block b's inner cells into uout.  Same values as k_blk_fill followed by k_blk_jacobi, in
// one launch instead of two: on the coarsest level, whose 256 iterations are launch-bound,
// that halves the launches.
constexpr int kSmallB = 16;
constexpr int kSmallThreadsMax = 1024;
int small_threads(int B)
{
  const int work = 6 * B * B > B * B * B ? 6 * B * B : B * B * B;
  const int t = (work + 63) / 64 * 64;
  return t < kSmallThreadsMax ? t : kSmallThreadsMax;
}

// ZERO: u is identically 0 (a coarse level's initial correction; not read, its ghosts not
// filled): each cell takes jacobi_cell's formula on literal zeros.
template <int ORDER, bool ZERO>
__global__ void __launch_bounds__(kSmallThreadsMax)
    k_blk_sweep_small(int B, C2FWeights W, double omega, const int* __restrict__ faces,
                      const double* __restrict__ hs, const double* __restrict__ f, double* u,
                      double* __restrict__ uout, int coarse)
{
  const int b = blockIdx.x;
  const int nf = B * B, n3 = nf * B;
  if (!ZERO) {
    for (int g = threadIdx.x; g < 6 * nf; g += blockDim.x) fill_ghost<ORDER>(B, W, faces, u, g % nf, g / nf, b);
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n3; t += blockDim.x) {
    const int zz = t / nf, r = t - zz * nf, yy = r / B;
    if (ZERO) jacobi_cell_zero(B, omega, hs, f, uout, coarse != 0, b, 1 + zz, 1 + yy, 1 + r - yy * B);
    else jacobi_cell(B, omega, faces, hs, f, u, uout, coarse != 0, b, 1 + zz, 1 + yy, 1 + r - yy * B);
  }
}

// Damped-Jacobi sweep of blocks of >= 64 cells a side, marching along z: a thread owns
// column (x, y) of a 64 x 4-cell tile of one block for kZRun consecutive planes and keeps
// u of the planes z-1, z, z+1 in registers, so each u value is loaded once by its column
// instead of once per z-neighbour; x and y neighbours come from the caches.  Per cell the
// operations of jacobi_cell.  Grid: (B/64, B/4, blocks x B/kZRun).
#ifndef MG_BLK_ZRUN
#define MG_BLK_ZRUN 8
#endif
constexpr int kZRun = MG_BLK_ZRUN;
__global__ void __launch_bounds__(kCellThreads)
    k_blk_jacobi_z(int B, double omega, const int* __restrict__ faces, const double* __restrict__ hs,
                   const double* __restrict__ f, const double* __restrict__ u,
                   double* __restrict__ uout, int coarse, int zero)
{
  const int x = 1 + blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x > B || y > B) return;
  const int runs = B / kZRun;
  const int b = blockIdx.z / runs;
  const int z0 = 1 + (blockIdx.z % runs) * kZRun;
  const int m = B + 2;
  const size_t sy = (size_t)m, sz = (size_t)m * m;
  const double h = hs[b];
  const double ih2 = 1.0 / (h * h), coef = omega * (h * h / 6.0);
  const int* fb = faces + (size_t)b * 6 * kFaceInts;
  const unsigned bxy = (x == 1 && fb[0 * kFaceInts] == kFaceBoundary ? 1u : 0u) |
                       (x == B && fb[1 * kFaceInts] == kFaceBoundary ? 2u : 0u) |
                       (y == 1 && fb[2 * kFaceInts] == kFaceBoundary ? 4u : 0u) |
                       (y == B && fb[3 * kFaceInts] == kFaceBoundary ? 8u : 0u);
  const bool zlo = fb[4 * kFaceInts] == kFaceBoundary, zhi = fb[5 * kFaceInts] == kFaceBoundary;
  size_t i = bidx(m, b, z0, y, x);
  if (zero) {
    // u identically 0 (a coarse level's initial correction): the formula on literal zeros
    for (int k = 0; k < kZRun; ++k, i += sz) {
      const int z = z0 + k;
      const double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      const unsigned bnd = bxy | (z == 1 && zlo ? 16u : 0u) | (z == B && zhi ? 32u : 0u);
      const double au = blk_apply_vals(ih2, 0.0, v, bnd, coarse != 0);
      uout[i] = 0.0 + coef * (f[i] - au);
    }
    return;
  }
  double zm = u[i - sz], c = u[i];
  for (int k = 0; k < kZRun; ++k, i += sz) {
    const int z = z0 + k;
    const double zp = u[i + sz];
    const double v[6] = {u[i - 1], u[i + 1], u[i - sy], u[i + sy], zm, zp};
    const unsigned bnd = bxy | (z == 1 && zlo ? 16u : 0u) | (z == B && zhi ? 32u : 0u);
    const double au = blk_apply_vals(ih2, c, v, bnd, coarse != 0);
    uout[i] = c + coef * (f[i] - au);
    zm = c;
    c = zp;
  }
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
    const double r = f[i] - blk_apply_at(B, faces + (size_t)b * 6 * kFaceInts, 1.0 / (h * h), u, i, z, y, x,
                                         false);
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

// ---------------------------------------------------------------- multigrid transfers
// fc = mean of the 8 children's residuals f - A u (children in z, y, x order) for every coarse
// inner cell; uc (optional) = 0 there.  B: fine block size, u's ghosts filled; one thread per
// coarse cell (cell_grid(B / 2)).
__global__ void __launch_bounds__(kCellThreads)
    k_blk_restrict(int B, const int* __restrict__ faces, const double* __restrict__ hs,
                   const double* __restrict__ f, const double* __restrict__ u,
                   double* __restrict__ fc, double* __restrict__ uc, int coarse)
{
  const int Bc = B / 2;
  int b, Z, Y, X;
  if (!cell_of(Bc, b, Z, Y, X)) return;
  --Z;
  --Y;
  --X;  // 0-based coarse indices
  const int m = B + 2;
  const double h = hs[b];
  const double ih2 = 1.0 / (h * h);
  const int* fb = faces + (size_t)b * 6 * kFaceInts;
  double s = 0.0;
  bool first = true;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int z = 1 + 2 * Z + dz, y = 1 + 2 * Y + dy, x = 1 + 2 * X + dx;
        const size_t i = bidx(m, b, z, y, x);
        const double r = f[i] - blk_apply_at(B, fb, ih2, u, i, z, y, x, coarse != 0);
        s = first ? r : s + r;
        first = false;
      }
  const size_t ci = bidx(Bc + 2, b, Z + 1, Y + 1, X + 1);
  fc[ci] = 0.125 * s;
  if (uc) uc[ci] = 0.0;
}

// u += P e on the inner cells (B: fine block size; e: B/2 cells per block, interface ghosts
// filled).  A fine cell lies towards +1 along an axis where its 0-based index is odd, -1
// where even; its correction is (e_P + e_x + e_y + e_z) / 4 with e_a the parent's neighbour on
// that side along axis a, -e_P where that neighbour lies across the domain boundary.
__global__ void __launch_bounds__(kCellThreads)
    k_blk_prolong(int B, const int* __restrict__ faces, const double* __restrict__ e,
                  double* __restrict__ u)
{
  int b, z1, y1, x1;
  if (!cell_of(B, b, z1, y1, x1)) return;
  const int x0 = x1 - 1, y0 = y1 - 1, z0 = z1 - 1;  // 0-based fine inner indices
  const int Bc = B / 2, mc = Bc + 2;
  const int* fb = faces + (size_t)b * 6 * kFaceInts;
  const int X = 1 + x0 / 2, Y = 1 + y0 / 2, Z = 1 + z0 / 2;
  const int dx = (x0 & 1) ? 1 : -1, dy = (y0 & 1) ? 1 : -1, dz = (z0 & 1) ? 1 : -1;
  const double eP = e[bidx(mc, b, Z, Y, X)];
  auto across = [&](int n, int face) {  // neighbour index n along an axis in the ghost layer?
    return (n == 0 || n == Bc + 1) && fb[face * kFaceInts] == kFaceBoundary;
  };
  const double ex = across(X + dx, (x0 & 1)) ? -eP : e[bidx(mc, b, Z, Y, X + dx)];
  const double ey = across(Y + dy, 2 + (y0 & 1)) ? -eP : e[bidx(mc, b, Z, Y + dy, X)];
  const double ez = across(Z + dz, 4 + (z0 & 1)) ? -eP : e[bidx(mc, b, Z + dz, Y, X)];
  const size_t i = bidx(B + 2, b, z0 + 1, y0 + 1, x0 + 1);
  u[i] = u[i] + 0.25 * (((eP + ex) + ey) + ez);
}

#ifndef MG_BLK_RESTRICT_Z_MIN
#define MG_BLK_RESTRICT_Z_MIN 32
#endif
constexpr int kRestrictZMin = MG_BLK_RESTRICT_Z_MIN;
// Residual restriction for fine blocks of >= 2 kRestrictZMin cells a side, marching along
// z: a thread owns coarse column (X, Y) of a 64 x 4 coarse tile for kZRun coarse planes and
// keeps the 2 x 2 fine columns of the planes 2Z .. 2Z+3 it needs in registers (the upper two
// are the next coarse plane's lower two).  Per child the operations of k_blk_restrict, summed
// in the same order.  Grid: (Bc/64, Bc/4, blocks x Bc/kZRun).
__global__ void __launch_bounds__(kCellThreads)
    k_blk_restrict_z(int B, const int* __restrict__ faces, const double* __restrict__ hs,
                     const double* __restrict__ f, const double* __restrict__ u,
                     double* __restrict__ fc, double* __restrict__ uc, int coarse)
{
  const int Bc = B / 2;
  const int X = blockIdx.x * 64 + (threadIdx.x & 63), Y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (X >= Bc || Y >= Bc) return;  // 0-based coarse indices
  const int runs = Bc / kZRun;
  const int b = blockIdx.z / runs;
  const int Z0 = (blockIdx.z % runs) * kZRun;
  const int m = B + 2, mc = Bc + 2;
  const size_t sy = (size_t)m;
  const double h = hs[b];
  const double ih2 = 1.0 / (h * h);
  const int* fb = faces + (size_t)b * 6 * kFaceInts;
  const int x0 = 1 + 2 * X, y0 = 1 + 2 * Y;  // first child column and row
  unsigned bxy[2][2];  // per child (dy, dx): x/y neighbours on the domain boundary
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const int x = x0 + dx, y = y0 + dy;
      bxy[dy][dx] = (x == 1 && fb[0 * kFaceInts] == kFaceBoundary ? 1u : 0u) |
                    (x == B && fb[1 * kFaceInts] == kFaceBoundary ? 2u : 0u) |
                    (y == 1 && fb[2 * kFaceInts] == kFaceBoundary ? 4u : 0u) |
                    (y == B && fb[3 * kFaceInts] == kFaceBoundary ? 8u : 0u);
    }
  const bool zlo = fb[4 * kFaceInts] == kFaceBoundary, zhi = fb[5 * kFaceInts] == kFaceBoundary;
  // P[q][dy][dx]: u of fine plane 2Z + q (q = 0..3) at the child column (dy, dx)
  double P[4][2][2];
  auto load_plane = [&](int q, int z) {
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) P[q][dy][dx] = u[bidx(m, b, z, y0 + dy, x0 + dx)];
  };
  load_plane(0, 2 * Z0);
  load_plane(1, 2 * Z0 + 1);
  for (int k = 0; k < kZRun; ++k) {
    const int Z = Z0 + k;
    load_plane(2, 2 * Z + 2);
    load_plane(3, 2 * Z + 3);
    double s = 0.0;
    bool first = true;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int z = 1 + 2 * Z + dz, y = y0 + dy, x = x0 + dx;
          const size_t i = bidx(m, b, z, y, x);
          const double c = P[1 + dz][dy][dx];
          const double v[6] = {dx ? P[1 + dz][dy][0] : u[i - 1], dx ? u[i + 1] : P[1 + dz][dy][1],
                               dy ? P[1 + dz][0][dx] : u[i - sy], dy ? u[i + sy] : P[1 + dz][1][dx],
                               P[dz][dy][dx], P[2 + dz][dy][dx]};
          const unsigned bnd = bxy[dy][dx] | (z == 1 && zlo ? 16u : 0u) | (z == B && zhi ? 32u : 0u);
          const double r = f[i] - blk_apply_vals(ih2, c, v, bnd, coarse != 0);
          s = first ? r : s + r;
          first = false;
        }
    const size_t ci = bidx(mc, b, Z + 1, Y + 1, X + 1);
    fc[ci] = 0.125 * s;
    if (uc) uc[ci] = 0.0;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        P[0][dy][dx] = P[2][dy][dx];
        P[1][dy][dx] = P[3][dy][dx];
      }
  }
}

// u += P e for fine blocks of >= 64 cells a side, marching along z: a thread owns fine column
// (x, y) of a 64 x 4 tile for kZRun fine planes; the parent and its x and y neighbours are
// the same for the two fine planes of a coarse plane.  Per cell the operations of
// k_blk_prolong.  Grid: (B/64, B/4, blocks x B/kZRun).
__global__ void __launch_bounds__(kCellThreads)
    k_blk_prolong_z(int B, const int* __restrict__ faces, const double* __restrict__ e,
                    double* __restrict__ u)
{
  const int x1 = 1 + blockIdx.x * 64 + (threadIdx.x & 63), y1 = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x1 > B || y1 > B) return;
  const int runs = B / kZRun;
  const int b = blockIdx.z / runs;
  const int zs = (blockIdx.z % runs) * kZRun;  // first 0-based fine plane (even)
  const int x0 = x1 - 1, y0 = y1 - 1;
  const int Bc = B / 2, mc = Bc + 2;
  const int* fb = faces + (size_t)b * 6 * kFaceInts;
  const int X = 1 + x0 / 2, Y = 1 + y0 / 2;
  const int dx = (x0 & 1) ? 1 : -1, dy = (y0 & 1) ? 1 : -1;
  auto across = [&](int n, int face) {
    return (n == 0 || n == Bc + 1) && fb[face * kFaceInts] == kFaceBoundary;
  };
  const bool ax = across(X + dx, (x0 & 1)), ay = across(Y + dy, 2 + (y0 & 1));
  size_t i = bidx(B + 2, b, zs + 1, y1, x1);
  const size_t sz = (size_t)(B + 2) * (B + 2);
  for (int k = 0; k < kZRun; k += 2) {
    const int Z = 1 + (zs + k) / 2;
    const double eP = e[bidx(mc, b, Z, Y, X)];
    const double ex = ax ? -eP : e[bidx(mc, b, Z, Y, X + dx)];
    const double ey = ay ? -eP : e[bidx(mc, b, Z, Y + dy, X)];
#pragma unroll
    for (int j = 0; j < 2; ++j, i += sz) {
      const int dz = j ? 1 : -1;  // 0-based fine plane zs + k + j: even -> -1, odd -> +1
      const double ez = across(Z + dz, 4 + j) ? -eP : e[bidx(mc, b, Z + dz, Y, X)];
      u[i] = u[i] + 0.25 * (((eP + ex) + ey) + ez);
    }
  }
}

// dst = src on the domain-boundary ghost cells (the Dirichlet data of the second buffer)
__global__ void __launch_bounds__(kFillThreads)
    k_blk_copy_boundary(int B, const int* __restrict__ faces, const double* __restrict__ src,
                        double* __restrict__ dst)
{
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B * B) return;
  const int f = blockIdx.y, b = blockIdx.z;
  if (faces[((size_t)b * 6 + f) * kFaceInts] != kFaceBoundary) return;
  int x, y, z;
  face_coords(f >> 1, (f & 1) ? B + 1 : 0, 1 + q % B, 1 + q / B, x, y, z);
  const size_t i = bidx(B + 2, b, z, y, x);
  dst[i] = src[i];
}

// ---------------------------------------------------------------- host drivers
// one workgroup per (face, block) and up to kFillThreads ghost cells of the face; faces of
// at most 64 cells (B <= 8) take one wave, not a workgroup of mostly idle waves
int face_threads(int B) { return B * B <= 64 ? 64 : kFillThreads; }
dim3 face_grid(int B)
{
  const int t = face_threads(B);
  return dim3((unsigned)((B * B + t - 1) / t), 6, kBlocks);
}

void fill(mgblk_ctx* c, int l, double* u)
{
  const int B = c->lv[l].B;
  const dim3 g = face_grid(B);
  const int t = face_threads(B);
  if (c->g.order == 0) k_blk_fill<0><<<g, t, 0, c->s>>>(B, c->w, c->faces, u);
  else if (c->g.order == 1) k_blk_fill<1><<<g, t, 0, c->s>>>(B, c->w, c->faces, u);
  else k_blk_fill<2><<<g, t, 0, c->s>>>(B, c->w, c->faces, u);
}

void copy_boundary(mgblk_ctx* c, int l, const double* src, double* dst)
{
  const int B = c->lv[l].B;
  k_blk_copy_boundary<<<face_grid(B), face_threads(B), 0, c->s>>>(B, c->faces, src, dst);
}

// `count` sweeps on level l with a fill before each, alternating between cur and oth (which
// holds the same domain-boundary ghosts); returns the buffer holding the result.  zero: cur is
// identically 0 (a coarse level's initial correction, l > 0): the first sweep reads neither
// it nor its ghosts, and needs no fill (same values).
double* sweeps(mgblk_ctx* c, int l, const double* f, double* cur, double* oth, int count,
               bool zero = false)
{
  const BlkLevel& L = c->lv[l];
  const int B = L.B;
  const dim3 grid = cell_grid(B);
  const bool zrun = B >= kCellRowsMin && B % kZRun == 0;
  const dim3 zgrid((unsigned)((B + 63) / 64), (unsigned)((B + 3) / 4), (unsigned)(kBlocks * (B / kZRun)));
  for (int s = 0; s < count; ++s) {
    const bool z0 = zero && s == 0 && l > 0;
    if (B <= kSmallB) {
      auto k = c->g.order == 0 ? (z0 ? k_blk_sweep_small<0, true> : k_blk_sweep_small<0, false>)
               : c->g.order == 1 ? (z0 ? k_blk_sweep_small<1, true> : k_blk_sweep_small<1, false>)
                                 : (z0 ? k_blk_sweep_small<2, true> : k_blk_sweep_small<2, false>);
      k<<<kBlocks, small_threads(B), 0, c->s>>>(B, c->w, c->g.omega, c->faces, L.hs, f, cur, oth,
                                                l > 0);
      double* x = cur;
      cur = oth;
      oth = x;
      continue;
    }
    if (!z0) fill(c, l, cur);
    if (zrun)
      k_blk_jacobi_z<<<zgrid, kCellThreads, 0, c->s>>>(B, c->g.omega, c->faces, L.hs, f, cur, oth, l > 0,
                                                       z0);
    else
      k_blk_jacobi<<<grid, kCellThreads, 0, c->s>>>(B, c->g.omega, c->faces, L.hs, f, cur, oth, l > 0,
                                                    z0);
    double* x = cur;
    cur = oth;
    oth = x;
  }
  return cur;
}

// fills u's ghosts on level l, fc (level l+1) = restricted residual, uc inner = 0 if given
void restrict_residual(mgblk_ctx* c, int l, const double* f, double* u, double* fc, double* uc)
{
  const BlkLevel& L = c->lv[l];
  const int Bc = L.B / 2;
  fill(c, l, u);
  // the plane-marching kernel from 32 coarse cells a side on (its 64 x 4 tile then leaves
  // half the lanes idle, but marching in z still beats one thread per coarse cell: 64^3 ->
  // 32^3 in about 0.15 ms instead of 0.24)
  if (Bc >= kRestrictZMin && Bc % kZRun == 0)
    k_blk_restrict_z<<<dim3((unsigned)((Bc + 63) / 64), (unsigned)((Bc + 3) / 4),
                            (unsigned)(kBlocks * (Bc / kZRun))),
                       kCellThreads, 0, c->s>>>(L.B, c->faces, L.hs, f, u, fc, uc, l > 0);
  else
    k_blk_restrict<<<cell_grid(Bc), kCellThreads, 0, c->s>>>(L.B, c->faces, L.hs, f, u, fc, uc, l > 0);
}

// fills ec's interface ghosts (level l+1), then u (level l) += P ec
void prolong_correct(mgblk_ctx* c, int l, double* ec, double* u)
{
  const int B = c->lv[l].B;
  fill(c, l + 1, ec);
  if (B >= kCellRowsMin && B % kZRun == 0)
    k_blk_prolong_z<<<dim3((unsigned)((B + 63) / 64), (unsigned)((B + 3) / 4),
                           (unsigned)(kBlocks * (B / kZRun))),
                      kCellThreads, 0, c->s>>>(B, c->faces, ec, u);
  else
    k_blk_prolong<<<cell_grid(B), kCellThreads, 0, c->s>>>(B, c->faces, ec, u);
}

// V(nu1, nu2) on level l from the iterate in x (y: the level's second buffer); returns the
// buffer holding the result.  Coarse problems start from 0 in the level's u.
double* vcycle_rec(mgblk_ctx* c, int l, const double* f, double* x, double* y, bool zero = false)
{
  const int last = (int)c->lv.size() - 1;
  if (l == last) return sweeps(c, l, f, x, y, c->g.coarse_iters, zero);
  double* cur = sweeps(c, l, f, x, y, c->g.nu1, zero);
  double* oth = cur == x ? y : x;
  BlkLevel& C = c->lv[l + 1];
  // the coarse level starts from a zero correction: read as 0 by its first sweep, or, when
  // its first step is not a sweep, written by the restriction
  const bool czero = (l + 1 == last ? c->g.coarse_iters : c->g.nu1) > 0;
  restrict_residual(c, l, f, cur, C.f, czero ? nullptr : C.u);
  double* ec = vcycle_rec(c, l + 1, C.f, C.u, C.t, czero);
  prolong_correct(c, l, ec, cur);
  return sweeps(c, l, f, cur, oth, c->g.nu2);
}

mg_status norm2(mgblk_ctx* c, const double* f, double* u, double* out)
{
  fill(c, 0, u);
  k_blk_norm2<<<kBlkNormBlocks, 256, 0, c->s>>>(c->lv[0].B, c->faces, c->lv[0].hs, f, u, c->partial);
  k_blk_sum<<<1, 256, 0, c->s>>>(c->partial, kBlkNormBlocks, c->scal);
  if (mg_status st = blk_hip(c, hipGetLastError(), "norm")) return st;
  if (mg_status st = blk_hip(c, hipMemcpyAsync(out, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s),
                             "reading the norm"))
    return st;
  return blk_hip(c, hipStreamSynchronize(c->s), "stream synchronisation");
}

// one V-cycle on the finest level, the result in u
void vcycle_top(mgblk_ctx* c, const double* f, double* u)
{
  BlkLevel& F = c->lv[0];
  copy_boundary(c, 0, u, F.t);
  double* r = vcycle_rec(c, 0, f, u, F.t);
  if (r != u) mgk::copy<double>(c->s, F.cnt, r, u);
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
  const int nlev = (int)c->lv.size();
  c->hhost.resize((size_t)kBlocks * nlev);
  for (int l = 0; l < nlev; ++l)
    for (int b = 0; b < kBlocks; ++b) c->hhost[(size_t)l * kBlocks + b] = blocks[b].width / c->lv[l].B;
  mg_status st = blk_hip(c, hipMemcpyAsync(c->faces, faces.data(), faces.size() * sizeof(int),
                                           hipMemcpyHostToDevice, c->s), "uploading the face table");
  for (int l = 0; l < nlev && !st; ++l)
    st = blk_hip(c, hipMemcpyAsync(c->lv[l].hs, &c->hhost[(size_t)l * kBlocks], kBlocks * sizeof(double),
                                   hipMemcpyHostToDevice, c->s), "uploading the block widths");
  // coarse levels: zero Dirichlet data in the ghost layers of both buffers, never rewritten
  for (int l = 1; l < nlev && !st; ++l) {
    st = blk_hip(c, hipMemsetAsync(c->lv[l].u, 0, c->lv[l].cnt * sizeof(double), c->s), "clearing a level");
    if (!st) st = blk_hip(c, hipMemsetAsync(c->lv[l].t, 0, c->lv[l].cnt * sizeof(double), c->s), "clearing a level");
  }
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
  fill(c, 0, u);
  return blk_hip(c, hipGetLastError(), "ghost fill");
}

mg_status mgblk_jacobi(mgblk_ctx* c, const double* f, double* u, int count)
{
  return mgblk_smooth(c, 0, f, u, count);
}

int mgblk_levels(const mgblk_ctx* c) { return c ? (int)c->lv.size() : 0; }

mg_status mgblk_smooth(mgblk_ctx* c, int level, const double* f, double* u, int count)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (level < 0 || level >= (int)c->lv.size()) return blk_fail(c, MG_EINVAL, "level %d out of range", level);
  if (!f || !u || count < 0) return blk_fail(c, MG_EINVAL, "bad Jacobi arguments");
  BlkLevel& L = c->lv[level];
  if (u == L.t) return blk_fail(c, MG_EINVAL, "u is the level's internal buffer");
  copy_boundary(c, level, u, L.t);
  double* r = sweeps(c, level, f, u, L.t, count);
  if (r != u) mgk::copy<double>(c->s, L.cnt, r, u);
  return blk_hip(c, hipGetLastError(), "Jacobi");
}

mg_status mgblk_restrict_residual(mgblk_ctx* c, int level, const double* f, double* u, double* fc)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (level < 0 || level + 1 >= (int)c->lv.size())
    return blk_fail(c, MG_EINVAL, "level %d has no coarser level", level);
  if (!f || !u || !fc) return blk_fail(c, MG_EINVAL, "f, u and fc must be non-NULL");
  restrict_residual(c, level, f, u, fc, nullptr);
  return blk_hip(c, hipGetLastError(), "restriction");
}

mg_status mgblk_prolong_correct(mgblk_ctx* c, int level, double* ec, double* u)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (level < 0 || level + 1 >= (int)c->lv.size())
    return blk_fail(c, MG_EINVAL, "level %d has no coarser level", level);
  if (!ec || !u) return blk_fail(c, MG_EINVAL, "ec and u must be non-NULL");
  prolong_correct(c, level, ec, u);
  return blk_hip(c, hipGetLastError(), "prolongation");
}

mg_status mgblk_vcycle(mgblk_ctx* c, const double* f, double* u)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return blk_fail(c, MG_EINVAL, "f and u must be non-NULL");
  vcycle_top(c, f, u);
  return blk_hip(c, hipGetLastError(), "V-cycle");
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
  BlkLevel& F = c->lv[0];
  copy_boundary(c, 0, u, F.t);
  double rn2 = 0;
  mg_status st = norm2(c, f, u, &rn2);
  double rn = std::sqrt(rn2);
  int k = 0;
  while (!st && std::isfinite(rn) && rn > tol && k < max_sweeps) {
    const int n = check_every < max_sweeps - k ? check_every : max_sweeps - k;
    double* r = sweeps(c, 0, f, u, F.t, n);
    if (r != u) mgk::copy<double>(c->s, F.cnt, r, u);
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

mg_status mgblk_mg_solve(mgblk_ctx* c, const double* f, double* u, double tol, int* cycles,
                         double* resnorm)
{
  if (!c) return blk_fail(nullptr, MG_EINVAL, "context is NULL");
  if (!f || !u) return blk_fail(c, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol >= 0)) return blk_fail(c, MG_EINVAL, "tol must be >= 0");
  double rn2 = 0;
  mg_status st = norm2(c, f, u, &rn2);
  double rn = std::sqrt(rn2);
  int k = 0;
  while (!st && std::isfinite(rn) && rn > tol && k < c->g.max_cycles) {
    vcycle_top(c, f, u);
    ++k;
    st = norm2(c, f, u, &rn2);
    rn = std::sqrt(rn2);
  }
  if (cycles) *cycles = k;
  if (resnorm) *resnorm = rn;
  if (st) return st;
  if (!std::isfinite(rn)) return blk_fail(c, MG_ENAN, "residual norm is not finite after %d cycles", k);
  if (rn > tol) return blk_fail(c, MG_ENOCONV, "residual norm %.3e > tol %.3e after %d cycles", rn, tol, k);
  return MG_OK;
}

}  // extern "C"
