// Temporally blocked red-black Gauss-Seidel for large 3D levels on gfx950.
//
// One launch performs S (1 or 2) complete red-black sweeps, out of place:
// uout = RBGS^S(uin), bitwise equal to S sweeps of the per-colour kernel (the same point
// formulas, mg_stencil.h).  The smoother is the hot loop of the V-cycle (the paper's
// light-speed model, Sect. 6, prices one lattice update of the finest-level smoother at
// 24 bytes: load u, load f, store u); fusing S sweeps divides that traffic by S.
//
// Decomposition
//  - A workgroup owns a 2D tile of BX = 128 columns x BY = W*RPW rows of one z-chunk and
//    streams through its planes in increasing z.  Lane l of wave w holds columns 2l and
//    2l+1 of rows w*RPW .. w*RPW+RPW-1: in every row exactly one of the two columns has a
//    given colour, so each half-sweep updates one node per lane per row and no lane idles
//    on the colour test.
//  - S sweeps are 2S half-sweeps ("stages").  Stage j (colour j mod 2, red first) updates
//    plane p = zl-1-j when plane zl has just been loaded: plane p's stage j needs planes
//    p-1 and p+1 after stage j-1, and stage j-1 reached p+1 earlier in the same step and
//    p-1 one step earlier.  Plane zl-H, H = 2S, is final and is stored.
//  - Stage j is applied only to nodes at least j+1 positions inside the loaded tile (and
//    the z-chunk's loaded range): its neighbours then have completed stage j-1.  After 2S
//    stages the final nodes are those at least H = 2S positions inside: the loaded tile
//    overlaps its neighbours by 2H columns / rows / planes (redundant halo), so tiles are
//    independent and the result does not depend on the schedule.
//  - Values live in registers: per lane a queue of H+2 planes (z-neighbours are own
//    registers), x-neighbours come from the adjacent lane by a cross-lane shuffle,
//    y-neighbours are own registers except across wave boundaries, where the first and
//    last row of each wave are exchanged through LDS (only the colour the next stage reads,
//    double-buffered by step parity so that one barrier per plane suffices).
//  - blockIdx -> tile is XCD-aware: a workgroup b runs on XCD b mod 8, so every XCD is given
//    a contiguous range of tiles, whose shared halo columns and rows then meet in the same L2.
#include "mg_kernels.h"
#include "mg_stencil.h"

#include <utility>

namespace mgk {
namespace {

template <int V>
using IC = std::integral_constant<int, V>;

constexpr int imod(int a, int m) { return ((a % m) + m) % m; }

template <typename T, bool VAR, int S, int W, int RPW>
struct Tiled {
  static constexpr int H = 2 * S;        // halo = number of stages
  static constexpr int BX = 128;         // columns per tile (2 per lane)
  static constexpr int BY = W * RPW;     // rows per tile
  static constexpr int TXO = BX - 2 * H; // output columns per tile
  static constexpr int TYO = BY - 2 * H; // output rows per tile
  static constexpr int Q = H + 2;        // planes held per lane
  static_assert(RPW % 2 == 0, "row parity must be uniform across the waves of a tile");
  static_assert(TYO > 0, "tile too short for the halo");

  struct Shared {
    T eu[2][H][W][2][64];                    // wave-boundary rows of u
    T ek[VAR ? 2 : 1][VAR ? H : 1][W][2][64]; // and of k
  };

  // B0 = parity of (global x of column 0) + (global y of row 0) + z0 - 1 (see below).
  template <int B0, bool ZERO_IN>
  __device__ __forceinline__ static void run(const T* __restrict__ uin, T* __restrict__ uout,
                                             const T* __restrict__ f, const T* __restrict__ k,
                                             int n, T h2, int ox, int oy, int z0, int z1,
                                             Shared& sh)
  {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int gx0 = ox - H;           // global x of tile column 0
    const int gxa = gx0 + 2 * lane;   // global x of this lane's first column
    const int gyw = oy - H + w * RPW; // global y of this wave's first row
    const size_t nn = (size_t)n;

    // validity of this lane's columns and rows (inside the grid) and interior-ness
    bool colok[2], colin[2], rowok[RPW], rowin[RPW];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const int gx = gxa + o;
      colok[o] = gx >= 0 && gx <= n - 1;
      colin[o] = gx >= 1 && gx <= n - 2;
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int gy = gyw + i;
      rowok[i] = gy >= 0 && gy <= n - 1;
      rowin[i] = gy >= 1 && gy <= n - 2;
    }

    T U[Q][RPW][2], F[Q][RPW][2], K[Q][RPW][2];
    T PU[RPW][2], PF[RPW][2], PK[RPW][2];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          U[q][i][o] = T(0);
          F[q][i][o] = T(0);
          if (VAR) K[q][i][o] = T(0);
        }

    auto load = [&](int zl) {
      const bool zok = zl >= 0 && zl <= n - 1;
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const bool ok = zok && rowok[i] && colok[o];
          const size_t idx = ((size_t)zl * nn + (size_t)(gyw + i)) * nn + (size_t)(gxa + o);
          T vu = T(0), vf = T(0), vk = T(0);
          if (ok) {
            if (!ZERO_IN) vu = uin[idx];
            vf = f[idx];
            if (VAR) vk = k[idx];
          }
          PU[i][o] = vu;
          PF[i][o] = vf;
          if (VAR) PK[i][o] = vk;
        }
    };

    const int zbeg = z0 - H, zend = z1 + H;  // planes loaded: [zbeg, zend)
    int zl = zbeg;
    int step = 0;
    load(zl);

    // One step for phase P = step mod Q: the plane zl - d sits in queue slot (P - d) mod Q.
    // The update column of row i in this step is o_i = (B0 + i + P) & 1, because the
    // colour of (x, y, p) is (x + y + p) & 1 and, at stage j, colour j&1 and p = zl-1-j
    // make x's parity depend on zl only.
    auto body = [&](auto PC) -> bool {
      constexpr int P = decltype(PC)::value;
      constexpr int s0 = imod(P, Q);
      // the prefetched plane zl enters the queue
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          U[s0][i][o] = PU[i][o];
          F[s0][i][o] = PF[i][o];
          if (VAR) K[s0][i][o] = PK[i][o];
        }
      __syncthreads();
      if (zl + 1 < zend) load(zl + 1);
      const int rb = (step + 1) & 1;  // LDS buffer written in the previous step
      const int wb = step & 1;        // LDS buffer written in this step

#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int p = zl - 1 - j;
        const int plo = max(1, z0 - (H - 1 - j)), phi = min(n - 2, z1 - 1 + (H - 1 - j));
        if (p < plo || p > phi) continue;  // uniform across the workgroup
        const int cs = imod(P - 1 - j, Q);  // centre plane p
        const int cm = imod(P - 2 - j, Q);  // plane p - 1
        const int cp = imod(P - j, Q);      // plane p + 1
        const int pslot = imod(p, H);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int o = (B0 + i + P) & 1;
          const int pr = w * RPW + i;  // tile row
          const int px = 2 * lane + o; // tile column
          const bool act = rowin[i] && colin[o] && pr >= j + 1 && pr <= BY - 2 - j &&
                           px >= j + 1 && px <= BX - 2 - j;
          // x-neighbours: own other column, or the neighbouring lane's
          T xm, xp, kxm = T(0), kxp = T(0);
          if (o == 0) {
            xm = __shfl_up(U[cs][i][1], 1, 64);
            xp = U[cs][i][1];
            if (VAR) { kxm = __shfl_up(K[cs][i][1], 1, 64); kxp = K[cs][i][1]; }
          } else {
            xm = U[cs][i][0];
            xp = __shfl_down(U[cs][i][0], 1, 64);
            if (VAR) { kxm = K[cs][i][0]; kxp = __shfl_down(K[cs][i][0], 1, 64); }
          }
          // y-neighbours in column o: own rows, or the adjacent wave's edge row
          T ym = T(0), yp = T(0), kym = T(0), kyp = T(0);
          if (i > 0) {
            ym = U[cs][i - 1][o];
            if (VAR) kym = K[cs][i - 1][o];
          } else if (w > 0) {
            ym = sh.eu[rb][pslot][w - 1][1][lane];
            if (VAR) kym = sh.ek[rb][pslot][w - 1][1][lane];
          }
          if (i < RPW - 1) {
            yp = U[cs][i + 1][o];
            if (VAR) kyp = K[cs][i + 1][o];
          } else if (w < W - 1) {
            yp = sh.eu[rb][pslot][w + 1][0][lane];
            if (VAR) kyp = sh.ek[rb][pslot][w + 1][0][lane];
          }
          const T zm = U[cm][i][o], zp = U[cp][i][o];
          const T h2f = h2 * F[cs][i][o];
          T v;
          if (!VAR) {
            v = gs_const<T, 3>(h2f, xm, xp, ym, yp, zm, zp);
          } else {
            v = gs_var<T, 3>(h2f, K[cs][i][o], xm, kxm, xp, kxp, ym, kym, yp, kyp, zm,
                             K[cm][i][o], zp, K[cp][i][o]);
          }
          if (act) U[cs][i][o] = v;
        }
      }

      // Edge rows for the next step: planes zl - d, d = 0..H-1.  The next step's stage d
      // reads plane zl - d in colour (d + 1) & 1, which in row i is column
      // (B0 + i + P) & 1 -- the same column as this step's update column.
#pragma unroll
      for (int d = 0; d < H; ++d) {
        const int sl = imod(P - d, Q);
        const int pslot = imod(zl - d, H);
        {
          constexpr int i = 0;
          const int o = (B0 + i + P) & 1;
          sh.eu[wb][pslot][w][0][lane] = U[sl][i][o];
          if (VAR) sh.ek[wb][pslot][w][0][lane] = K[sl][i][o];
        }
        {
          constexpr int i = RPW - 1;
          const int o = (B0 + i + P) & 1;
          sh.eu[wb][pslot][w][1][lane] = U[sl][i][o];
          if (VAR) sh.ek[wb][pslot][w][1][lane] = K[sl][i][o];
        }
      }

      // store the finished plane zl - H
      const int pout = zl - H;
      if (pout >= z0 && pout < z1) {
        constexpr int so = imod(P - H, Q);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int pr = w * RPW + i;
          if (!rowin[i] || pr < H || pr > BY - 1 - H) continue;
          const size_t base = ((size_t)pout * nn + (size_t)(gyw + i)) * nn + (size_t)gxa;
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const int px = 2 * lane + o;
            if (colin[o] && px >= H && px <= BX - 1 - H) uout[base + o] = U[so][i][o];
          }
        }
      }
      ++step;
      ++zl;
      return zl < zend;
    };

    auto unrolled = [&](auto... PCs) {
      bool go = true;
      ((go = go && body(PCs)), ...);
      return go;
    };
    auto round = [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
      return unrolled(IC<Ps>{}...);
    };
    while (round(std::make_integer_sequence<int, Q>{})) {
    }
  }
};

template <typename T, bool VAR, int S, int W, int RPW, bool ZERO_IN>
__global__ void __launch_bounds__(64 * W)
    k_rbgs_tiled(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ f,
                 const T* __restrict__ k, int n, T h2, int tiles_x, int tiles_y, int zlen)
{
  using C = Tiled<T, VAR, S, W, RPW>;
  __shared__ typename C::Shared sh;
  // XCD-aware tile index: workgroup b runs on XCD b % 8; XCD x gets tiles
  // [start_x, start_x + count_x) in order.
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b & 7, jb = b >> 3, q = nb >> 3, rem = nb & 7;
  const int t = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + jb;
  const int tx = t % tiles_x;
  const int ty = (t / tiles_x) % tiles_y;
  const int tz = t / (tiles_x * tiles_y);
  const int ox = 1 + tx * C::TXO, oy = 1 + ty * C::TYO;
  const int z0 = 1 + tz * zlen;
  const int z1 = min(z0 + zlen, n - 1);
  // parity of (x of column 0) + (y of row 0) + z0 - 1; RPW is even, so it is the same
  // for every wave's first row
  const int b0 = ((ox - C::H) + (oy - C::H) + z0 - 1) & 1;
  if (b0) C::template run<1, ZERO_IN>(uin, uout, f, k, n, h2, ox, oy, z0, z1, sh);
  else C::template run<0, ZERO_IN>(uin, uout, f, k, n, h2, ox, oy, z0, z1, sh);
}

struct LaunchShape {
  int tiles_x, tiles_y, nchunks, zlen, blocks;
};

template <typename C>
LaunchShape shape_for(int n, int target_blocks)
{
  LaunchShape L;
  const int m = n - 2;
  L.tiles_x = (m + C::TXO - 1) / C::TXO;
  L.tiles_y = (m + C::TYO - 1) / C::TYO;
  const int per = L.tiles_x * L.tiles_y;
  int chunks = (target_blocks + per - 1) / per;
  if (chunks < 1) chunks = 1;
  // keep chunks at least 4H planes deep so the z-halo stays a small overhead
  const int maxchunks = m / (4 * C::H) > 0 ? m / (4 * C::H) : 1;
  if (chunks > maxchunks) chunks = maxchunks;
  L.zlen = (m + chunks - 1) / chunks;
  L.nchunks = (m + L.zlen - 1) / L.zlen;
  L.blocks = per * L.nchunks;
  return L;
}

template <typename T, bool VAR, int S, int W, int RPW>
void launch_cfg(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin, T* uout,
                bool zero_in, int target_blocks)
{
  using C = Tiled<T, VAR, S, W, RPW>;
  const LaunchShape L = shape_for<C>(n, target_blocks);
  const T h2 = (T)(h * h);
  if (zero_in)
    k_rbgs_tiled<T, VAR, S, W, RPW, true><<<L.blocks, 64 * W, 0, s>>>(
        uin, uout, f, k, n, h2, L.tiles_x, L.tiles_y, L.zlen);
  else
    k_rbgs_tiled<T, VAR, S, W, RPW, false><<<L.blocks, 64 * W, 0, s>>>(
        uin, uout, f, k, n, h2, L.tiles_x, L.tiles_y, L.zlen);
}

}  // namespace

bool rbgs_tiled_supported(int dim, int n) { return dim == 3 && n >= 33; }

int rbgs_tiled_max_sweeps(bool var, size_t value_bytes)
{
  // the FP64 variable-coefficient pass keeps k in registers too: one sweep per pass keeps
  // it free of register spills
  return (var && value_bytes == 8) ? 1 : 2;
}

template <typename T>
void rbgs_tiled(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin, T* uout,
                int sweeps, bool zero_in)
{
  constexpr int kTarget = 512;  // workgroups per launch before z-chunking stops
  // the host asks for 2 sweeps with k only in FP32 (rbgs_tiled_max_sweeps)
  if (sweeps == 2) {
    if (k) {
      if constexpr (sizeof(T) == 4) launch_cfg<T, true, 2, 8, 4>(s, n, h, k, f, uin, uout, zero_in, kTarget);
    } else {
      launch_cfg<T, false, 2, 8, 4>(s, n, h, k, f, uin, uout, zero_in, kTarget);
    }
  } else {
    if (k) launch_cfg<T, true, 1, 8, 4>(s, n, h, k, f, uin, uout, zero_in, kTarget);
    else launch_cfg<T, false, 1, 8, 4>(s, n, h, k, f, uin, uout, zero_in, kTarget);
  }
}

template void rbgs_tiled<double>(hipStream_t, int, double, const double*, const double*,
                                 const double*, double*, int, bool);
template void rbgs_tiled<float>(hipStream_t, int, double, const float*, const float*,
                                const float*, float*, int, bool);

}  // namespace mgk
