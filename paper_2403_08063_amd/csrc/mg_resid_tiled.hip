// Streaming residual kernels for large 3D levels on gfx950: one pass over u and f per call.
//
//  - restriction (Stream): fc = FW(f - A u) on the coarse interior (full weighting, the
//    tensor product of (1/4, 1/2, 1/4));
//  - norm (Pass, below): sum over interior nodes of (f - A u)^2, per-workgroup partial sums
//    reduced afterwards in a fixed order; optionally with the interior of u read as 0 (the
//    norm of the full right-hand side);
//  - refinement pass (Pass): u_out = u + s e (e in float), r = f - A u_out,
//    r32 = r * inv_scale (float), sum of r^2 -- the FP64 update, residual, norm and down-cast
//    of one step of iterative refinement fused in one pass;
//  - the cell-centred finite-volume sweep, norm and restriction (Pass).
//
// Restriction decomposition (as in the fused smoother): a workgroup owns a tile of 128 columns x
// W*RPW rows of a z-chunk and streams through its planes; lane l of wave w holds columns
// 2l, 2l+1 of rows w*RPW .. w*RPW+RPW-1.  A lane keeps u on the planes s-1, s, s+1 in
// registers (the residual's z-neighbours), takes x-neighbours from adjacent lanes by DPP
// and y-neighbours from its own rows or, across wave boundaries, from edge rows exchanged
// through LDS one step ahead (double-buffered: one barrier per plane).  Tiles overlap by
// the one-node halo the residual needs; each output node belongs to exactly one tile.
//
// Restriction: lane l's first column is the fine node 2X of coarse column X, so
// FW_x = r(2X-1)/4 + r(2X)/2 + r(2X+1)/4 needs one DPP; a wave's even rows are fine rows
// 2Y and FW_y combines rows 2Y-1, 2Y, 2Y+1 one step later (the row above a wave comes from
// the previous wave through LDS); FW_z accumulates over the fine planes 2Z-1, 2Z, 2Z+1.
// Paper: the residual-norm stopping test of Sect. 5; the operators of Sect. 5, Eq. 1.
#include "mg_buffer.h"
#include "mg_kernels.h"
#include "mg_lanes.h"
#include "mg_stencil.h"

#include <type_traits>

namespace mgk {
namespace {

template <int V>
using IC = std::integral_constant<int, V>;

enum { kRestrict = 0, kNorm = 1, kRefine = 2, kFvNorm = 3, kFvJacobi = 4, kFvRestrict = 5,
       kRefineRhs = 6, kFvJacobiProlong = 7, kNormRhs = 8 };

// Shape of the finite-volume sweep with the prolongation from N = 256 on (waves, rows per
// wave, column pairs per lane), from timing sweeps on MI355X at 512^3 cells: 128 x 32-cell
// tiles (two row pairs per lane; the interpolation needs the registers a second column pair
// would take).
#ifndef MG_FV_PROLONG_CP
#define MG_FV_PROLONG_CP 1
#endif
#ifndef MG_FV_PROLONG_W
#define MG_FV_PROLONG_W 8
#endif
#ifndef MG_FV_PROLONG_RPW
#define MG_FV_PROLONG_RPW 4
#endif

// (A u)_i of the cell-centred finite-volume operator from the six neighbour values (ghost
// neighbours already replaced by 2 g - u_i), in the order -x, +x, -y, +y, -z, +z.
__device__ __forceinline__ double fv_au(double ih2, double ui, double v0, double v1, double v2,
                                        double v3, double v4, double v5)
{
  double s = ui - v0;
  s = s + (ui - v1);
  s = s + (ui - v2);
  s = s + (ui - v3);
  s = s + (ui - v4);
  s = s + (ui - v5);
  return s * ih2;
}

template <typename T, bool VAR, int MODE, int W, int RPW, int PD>
struct Stream {
  static_assert(MODE == kRestrict, "the streaming restriction (norms and refinement: Pass)");
  static_assert(PD == 1 || PD == 2, "prefetch depth");
  static constexpr int BX = 128;
  static constexpr int BY = W * RPW;
  static constexpr int CX = 62, CY = BY / 2 - 2;  // coarse columns / rows per tile
  static_assert(RPW % 2 == 0, "fine row parity must be uniform across waves");

  struct Shared {
    T eu[2][W][2][2][64];  // edge rows of u: [buffer][wave][first/last row][column][lane]
    T ek[VAR ? 2 : 1][VAR ? W : 1][2][2][64];
    T erx[2][W][64];  // x-filtered residual of a wave's last row
  };

  struct Args {
    const T* f;
    const T* u;
    const T* k;
    T* out;  // fc
    int n;
    T ih2;
    int tiles_x, tiles_y, zlen;
  };

  __device__ __forceinline__ static void run(const Args& a, Shared& sh)
  {
    const int n = a.n;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware tile index (workgroup b runs on XCD b % 8)
    const int b = blockIdx.x, nb = gridDim.x;
    const int xcd = b & 7, jb = b >> 3, q = nb >> 3, rem = nb & 7;
    const int t = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + jb;
    const int tx = t % a.tiles_x, ty = (t / a.tiles_x) % a.tiles_y, tz = t / (a.tiles_x * a.tiles_y);

    // fine tile origin and residual planes [sbeg, send] of the coarse planes [Z0, Z1)
    const int nc = (n - 1) / 2 + 1;
    const int X0 = 1 + tx * CX, Y0 = 1 + ty * CY;
    const int Z0 = 1 + tz * a.zlen;
    const int Z1 = min(Z0 + a.zlen, nc - 1);
    const int gx0 = 2 * X0 - 2, gy0 = 2 * Y0 - 2;
    const int sbeg = 2 * Z0 - 1, send = 2 * Z1 - 1;
    const int gxa = gx0 + 2 * lane;
    const int gyw = gy0 + w * RPW;

    // Addresses: per-plane buffer resources, a uniform row byte offset and a per-lane
    // column byte offset.  Clamped coordinates keep every load in bounds.
    uint32_t cxb[2];
    bool colin[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const int gx = gxa + o;
      const uint32_t c = (uint32_t)min(max(gx, 0), n - 1);
      colin[o] = gx >= 1 && gx <= n - 2;
      cxb[o] = c * (uint32_t)sizeof(T);
    }
    uint32_t rowb[RPW];
    bool rowin[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int gy = gyw + i;
      const uint32_t r = (uint32_t)(min(max(gy, 0), n - 1) * n);
      rowb[i] = r * (uint32_t)sizeof(T);
      rowin[i] = gy >= 1 && gy <= n - 2;
    }
    const uint32_t planeb = (uint32_t)((size_t)n * (size_t)n * sizeof(T));
    const int wm = w > 0 ? w - 1 : 0, wp = w < W - 1 ? w + 1 : W - 1;  // adjacent waves

    // Queue of the planes s-1, s, s+1 and PD prefetch buffers.  PD = 2: at step s the
    // loads of plane s+3 are issued into one buffer while plane s+2 (issued a step earlier)
    // waits in the other, so each load has two steps' work to arrive in.  PD = 1 (fewer
    // registers): plane s+2 is loaded and consumed in step s.
    T U[3][RPW][2], F[3][RPW][2], K[3][RPW][2];
    T PU[PD][RPW][2], PF[PD][RPW][2], PK[PD][RPW][2];
    auto load = [&](auto BC, int z) {
      constexpr int bb = decltype(BC)::value;
      const size_t zc = (size_t)min(max(z, 0), n - 1);
      const PlaneBuf bu = plane_buf(a.u, zc * planeb, planeb);
      const PlaneBuf bf = plane_buf(a.f, zc * planeb, planeb);
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          PU[bb][i][o] = buf_load<T>(bu, cxb[o], rowb[i]);
          PF[bb][i][o] = buf_load<T>(bf, cxb[o], rowb[i]);
        }
      if constexpr (VAR) {
        const PlaneBuf bk = plane_buf(a.k, zc * planeb, planeb);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int o = 0; o < 2; ++o) PK[bb][i][o] = buf_load<T>(bk, cxb[o], rowb[i]);
      }
    };
    // plane z enters the queue from buffer BB
    auto shift_in = [&](auto BC, int) {
      constexpr int bb = decltype(BC)::value;
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const T v = PU[bb][i][o];
          U[0][i][o] = U[1][i][o]; U[1][i][o] = U[2][i][o]; U[2][i][o] = v;
          F[0][i][o] = F[1][i][o]; F[1][i][o] = F[2][i][o]; F[2][i][o] = PF[bb][i][o];
          if constexpr (VAR) {
            K[0][i][o] = K[1][i][o]; K[1][i][o] = K[2][i][o]; K[2][i][o] = PK[bb][i][o];
          }
        }
    };
    auto write_edges = [&](int buf, int slot) {  // first and last row of a queued plane
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        sh.eu[buf][w][0][o][lane] = U[slot][0][o];
        sh.eu[buf][w][1][o][lane] = U[slot][RPW - 1][o];
        if constexpr (VAR) {
          sh.ek[buf][w][0][o][lane] = K[slot][0][o];
          sh.ek[buf][w][1][o][lane] = K[slot][RPW - 1][o];
        }
      }
    };

    // prologue: planes sbeg-1, sbeg, sbeg+1 in the queue, edges of plane sbeg written,
    // plane sbeg+2 on its way into buffer 0
    load(IC<0>{}, sbeg - 1);
    shift_in(IC<0>{}, sbeg - 1);
    load(IC<0>{}, sbeg);
    shift_in(IC<0>{}, sbeg);
    load(IC<0>{}, sbeg + 1);
    shift_in(IC<0>{}, sbeg + 1);
    write_edges(1, 1);  // edges of plane sbeg, read at the first step from buffer 1
    const int lastload = send + 1;  // the last plane any step reads
    if (PD == 2 && sbeg + 2 <= lastload) load(IC<0>{}, sbeg + 2);

    T rxprev[RPW];
    T acc[RPW / 2];
#pragma unroll
    for (int i = 0; i < RPW; ++i) rxprev[i] = T(0);
#pragma unroll
    for (int i = 0; i < RPW / 2; ++i) acc[i] = T(0);

    // One step at plane s; the step's parity BB (step count from sbeg) selects the
    // prefetch buffer and the LDS edge buffers.
    auto stepfn = [&](auto BC, int s) {
      constexpr int bb = decltype(BC)::value;
      constexpr int rb = 1 - bb, wb = bb;  // LDS buffer written in the previous / this step
      __syncthreads();
      constexpr int lb = PD == 2 ? 1 - bb : 0;  // buffer of this step's loads
      constexpr int cb = PD == 2 ? bb : 0;      // buffer of the plane entering the queue
      if (s + PD + 1 <= lastload) load(IC<lb>{}, s + PD + 1);

      if (s > sbeg) {
        // FW_y of plane s-1 for the coarse rows at even fine rows, then FW_z over the fine
        // planes 2Z-1 (1/4), 2Z (1/2), 2Z+1 (1/4)
        const int sp = s - 1;
        T ry[RPW / 2];
#pragma unroll
        for (int i = 0; i < RPW; i += 2) {
          const T above = i > 0 ? rxprev[i - 1] : (w > 0 ? sh.erx[rb][w - 1][lane] : T(0));
          ry[i / 2] = (T(0.25) * above + T(0.5) * rxprev[i]) + T(0.25) * rxprev[i + 1];
        }
        if (sp & 1) {
          // plane sp = 2Z+1 completes coarse plane Z and starts plane Z+1
          const int Z = (sp - 1) / 2;
          const int nc = (n - 1) / 2 + 1;
          const bool store = Z >= Z0 && Z < Z1;
          const size_t zo = (size_t)Z * nc * nc;
#pragma unroll
          for (int i = 0; i < RPW; i += 2) {
            const T done = acc[i / 2] + T(0.25) * ry[i / 2];
            const int crow = (w * RPW + i) / 2;  // coarse Y = Y0 - 1 + crow
            const int Y = gy0 / 2 + crow;
            const int X = gx0 / 2 + lane;
            if (store && crow >= 1 && crow <= CY && lane >= 1 && lane <= CX && Y <= nc - 2 &&
                X <= nc - 2)
              a.out[zo + (size_t)Y * nc + X] = done;
            acc[i / 2] = T(0.25) * ry[i / 2];
          }
        } else {
#pragma unroll
          for (int i = 0; i < RPW; i += 2) acc[i / 2] = acc[i / 2] + T(0.5) * ry[i / 2];
        }
      }

      if (s <= send) {
        // residual at plane s (queue slot 1), every node; the first and the last wave read
        // their own edge rows at the tile edge, where no residual is used
        T r[RPW][2];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const T l1 = from_lane_below(U[1][i][1]);
          const T r0 = from_lane_above(U[1][i][0]);
          T kl1 = T(0), kr0 = T(0);
          if constexpr (VAR) { kl1 = from_lane_below(K[1][i][1]); kr0 = from_lane_above(K[1][i][0]); }
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const T ui = U[1][i][o];
            const T xm = o == 0 ? l1 : U[1][i][0];
            const T xp = o == 0 ? U[1][i][1] : r0;
            T ym, yp, kym = T(0), kyp = T(0);
            if (i > 0) {
              ym = U[1][i - 1][o];
              if constexpr (VAR) kym = K[1][i - 1][o];
            } else {
              ym = sh.eu[rb][wm][1][o][lane];
              if constexpr (VAR) kym = sh.ek[rb][wm][1][o][lane];
            }
            if (i < RPW - 1) {
              yp = U[1][i + 1][o];
              if constexpr (VAR) kyp = K[1][i + 1][o];
            } else {
              yp = sh.eu[rb][wp][0][o][lane];
              if constexpr (VAR) kyp = sh.ek[rb][wp][0][o][lane];
            }
            const T zm = U[0][i][o], zp = U[2][i][o];
            T au;
            if constexpr (!VAR) {
              au = au_const<T, 3>(a.ih2, ui, xm, xp, ym, yp, zm, zp);
            } else {
              const T kxm = o == 0 ? kl1 : K[1][i][0];
              const T kxp = o == 0 ? K[1][i][1] : kr0;
              au = au_var<T, 3>(a.ih2, ui, K[1][i][o], xm, kxm, xp, kxp, ym, kym, yp, kyp, zm,
                                K[0][i][o], zp, K[2][i][o]);
            }
            r[i][o] = F[1][i][o] - au;
          }
        }
        // fine nodes outside the interior carry no residual
        const bool zin = s >= 1 && s <= n - 2;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
#pragma unroll
          for (int o = 0; o < 2; ++o)
            r[i][o] = (zin && rowin[i] && colin[o]) ? r[i][o] : T(0);
          const T left = from_lane_below(r[i][1]);
          rxprev[i] = (T(0.25) * left + T(0.5) * r[i][0]) + T(0.25) * r[i][1];
        }
        sh.erx[wb][w][lane] = rxprev[RPW - 1];
      }
      // next step: planes s, s+1, s+2; edges of plane s+1 (slot 2 before the shift)
      write_edges(wb, 2);
      shift_in(IC<cb>{}, s + 2);
    };

    // one step past the last residual plane: its FW_y and FW_z complete the last coarse plane
    const int last = send + 1;
    for (int s = sbeg; s <= last;) {
      stepfn(IC<0>{}, s);
      if (++s > last) break;
      stepfn(IC<1>{}, s);
      ++s;
    }
  }
};

// Norm and refinement passes with an exact partition of the interior (no tile overlap).
//
// A workgroup of W waves owns the interior nodes of a tile of BX = 128*CP columns x
// BY = W*RPW rows of a z-chunk.  Lane l of wave w holds the column pairs (c, c+1) with
// c = ox + 128p + 2l, p < CP, of the rows oy + w*RPW + i; the tile origin ox is odd, so
// each pair is one 16-byte access (8 bytes in the FP32 arrays), and the last interior
// column n-2 (odd, n = 2^m + 1) opens the pair whose second column is the boundary n-1.
// The one-node halo is loaded, not recomputed: the column left and right of the tile by
// lanes 0 and 63 of one extra load per row, the row below / above the tile by the first /
// last wave.  x-neighbours come from adjacent lanes by DPP (the lane without a source lane
// takes the halo column or the adjacent pair's edge lane instead of 0), y-neighbours from
// the lane's own rows or the adjacent wave's edge rows through LDS (double-buffered, one
// barrier per plane), z-neighbours from a queue of three planes.  Compared with
// overlapping 128-column tiles this drops the tiles that own a few columns at the end of
// a row and halves the memory instructions.
//
// The same decomposition serves the cell-centred finite-volume scheme (MODE kFvNorm,
// kFvJacobi): N^3 cells with a ghost layer, n = N + 2 values per side.  The ghost layer
// holds the Dirichlet value at the face centre, and a ghost neighbour enters the operator
// as 2 g - u_i; kFvJacobi writes the damped Jacobi update u + coef (f - A u) out of place.
// kFvRestrict writes the mean of the 8 children's residuals to the coarse level: a lane's
// column pair, a wave's row pair and a pair of consecutive planes (z-chunks of even length
// starting on odd planes) are the children of one coarse cell, summed in the order z, y, x.
// kFvJacobiProlong is the Jacobi sweep of u + P e: the coarse-grid correction e (N/2 cells
// per side) is interpolated onto every fine value the sweep reads -- the lane's own cells,
// the halo column and the halo row -- once they are in registers, so the corrected iterate
// is never stored.  The tile's coarse region (the parents of its cells, the halo's parents
// and one coarse cell around them) is staged plane by plane in LDS: a ring of three coarse
// planes, one new plane every second fine plane.  Each fine value sums its 8 weighted
// coarse terms in the order z, y, x, parent first (the stand-alone prolongation's order).
template <bool VAR, int MODE, int W, int RPW, int CP>
struct Pass {
  static constexpr bool PRO = MODE == kFvJacobiProlong;
  static constexpr bool JAC = MODE == kFvJacobi || PRO;  // writes a Jacobi update
  static constexpr bool FV = MODE == kFvNorm || JAC || MODE == kFvRestrict;
  // refinement pass; kRefineRhs (the first pass of a solve, no correction) also sums the
  // squares of the full right-hand side b = f - A u_B (u_B: the Dirichlet data of u with a
  // zero interior), with the operations of the norm pass reading the interior of u as 0
  static constexpr bool REFINE = MODE == kRefine || MODE == kRefineRhs;
  static constexpr bool RHS = MODE == kRefineRhs || MODE == kNormRhs;  // kNormRhs: both norms
  static_assert(MODE != kFvRestrict || RPW % 2 == 0, "row pairs of the restriction");
  static_assert(!PRO || RPW % 2 == 0, "row pairs share their coarse parents");
  static_assert(!(FV && VAR), "the finite-volume scheme has a constant coefficient");
  static_assert(W >= 2, "the first and the last wave load the tile's halo rows");
  static constexpr int BX = 128 * CP, BY = W * RPW;
  static constexpr int NE = RPW > 1 ? 2 : 1;  // edge rows of a wave: first, last
  // prolongation: coarse rows and columns staged per coarse plane (parents of the tile's
  // BY rows and BX columns and one more on each side), values loaded per thread
  static constexpr int CRY = PRO ? BY / 2 + 2 : 1, CRX = PRO ? 64 * CP + 2 : 1;
  static constexpr int CLD = PRO ? (CRY * CRX + 64 * W - 1) / (64 * W) : 1;

  struct Shared {
    double eu[2][W][NE][CP][2][64];  // [buffer][wave][first/last row][pair][column][lane]
    double ek[VAR ? 2 : 1][VAR ? W : 1][VAR ? NE : 1][VAR ? CP : 1][2][64];
    double cz[PRO ? 3 : 1][CRY * CRX];  // prolongation: coarse plane Z in slot Z mod 3
    double red[W];
    double redb[W];
  };

  struct Args {
    const double* f;
    const double* u;
    const double* k;
    double* out;         // refinement: u_out
    const float* e;      // refinement: correction (nullptr: none)
    float* r32;          // refinement: scaled residual
    double* partial;
    double scale;        // refinement: u_out = u + scale * e
    double inv_scale;    // refinement: r32 = r * inv_scale
    double coef;         // finite-volume Jacobi: u_out = u + coef * (f - A u)
    const double* ec;    // finite-volume prolongation: coarse correction, (N/2 + 2)^3
    int zero_interior;   // norm: read the interior of u as 0; FV Jacobi: u is 0 (not read)
    int n;
    double ih2;
    int tiles_x, tiles_y, zlen;
    double* partial_b;   // kRefineRhs: per-workgroup sums of b^2
  };

  __device__ __forceinline__ static void run(const Args& a, Shared& sh)
  {
    const int n = a.n;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware tile index (workgroup b runs on XCD b % 8): the y-adjacent tiles of a
    // z-chunk, which share their halo rows, run on one XCD and its L2
    const int b = blockIdx.x, nb = gridDim.x;
    const int xcd = b & 7, jb = b >> 3, q = nb >> 3, rem = nb & 7;
    const int t = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + jb;
    const int tx = t % a.tiles_x, ty = (t / a.tiles_x) % a.tiles_y, tz = t / (a.tiles_x * a.tiles_y);
    const int ox = 1 + tx * BX, oy = 1 + ty * BY;
    const int z0 = 1 + tz * a.zlen, z1 = min(z0 + a.zlen, n - 1);  // owned planes [z0, z1)

    // Column pairs: byte offsets (double and float arrays); store offsets outside the
    // plane's range for lanes that own no column of the pair (those stores are dropped).
    uint32_t cb[CP], cf[CP], sb[CP], sf[CP];
    bool in0[CP], in1[CP];
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const int c = ox + 128 * p + 2 * lane;
      const uint32_t lc = (uint32_t)min(c, n - 2);
      in0[p] = c <= n - 2;
      in1[p] = c + 1 <= n - 2;
      cb[p] = lc * 8u;
      cf[p] = lc * 4u;
      sb[p] = in0[p] ? cb[p] : 0x80000000u;
      sf[p] = in0[p] ? cf[p] : 0x80000000u;
    }
    const int hc = lane == 63 ? min(ox + BX, n - 1) : ox - 1;  // halo column (lanes 0, 63)
    const bool hcin = hc >= 1 && hc <= n - 2;
    const uint32_t hcb = (uint32_t)hc * 8u, hcf = (uint32_t)hc * 4u;
    uint32_t rb8[RPW], rb4[RPW];
    bool rin[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int gy = oy + w * RPW + i;
      const uint32_t r = (uint32_t)(min(gy, n - 1) * n);
      rb8[i] = r * 8u;
      rb4[i] = r * 4u;
      rin[i] = gy <= n - 2;
    }
    const bool hw = w == 0 || w == W - 1;  // loads a halo row
    const int hy = w == 0 ? oy - 1 : min(oy + BY, n - 1);
    const bool hyin = hy >= 1 && hy <= n - 2;
    const uint32_t hrb8 = (uint32_t)(hy * n) * 8u, hrb4 = (uint32_t)(hy * n) * 4u;
    const uint32_t planeb = (uint32_t)((size_t)n * (size_t)n * 8u);
    const uint32_t planef = (uint32_t)((size_t)n * (size_t)n * 4u);
    const int wm = w > 0 ? w - 1 : 0, wp = w < W - 1 ? w + 1 : W - 1;
    const bool corr = REFINE && a.e != nullptr;
    // finite volumes: which neighbours of a lane's cells are ghost cells (x per pair and
    // column, y per row; z per plane in the step)
    bool gx0[CP], gxp0[CP], gxp1[CP], gym[RPW], gyp[RPW];
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const int c = ox + 128 * p + 2 * lane;
      gx0[p] = c == 1;
      gxp0[p] = c + 1 == n - 1;
      gxp1[p] = c + 2 == n - 1;
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int gy = oy + w * RPW + i;
      gym[i] = gy == 1;
      gyp[i] = gy + 1 == n - 1;
    }

    // Prolongation (u + P e): the coarse region's origin is the parent of the tile's first
    // cell minus one; a lane's rows 2i', 2i'+1 (global rows odd, even) share the parent row
    // wave*RPW/2 + i' + 1 of the region and take the row below / above as the neighbour; its
    // column pair shares the parent column 64 p + lane + 1 (neighbour left / right).  The
    // halo column is the parent's right half (lane 0: parent 0, neighbour 1) or left half
    // (lane 63: parent 64 CP + 1, neighbour 64 CP); likewise the halo rows.
    const int cxo = (ox + 1) / 2 - 1, cyo = (oy + 1) / 2 - 1;
    const int ncs = (n - 2) / 2;  // coarse cells per side
    auto cload = [&](int Zc, double (&R)[CLD]) {
#pragma unroll
      for (int k = 0; k < CLD; ++k) {
        const int t = (int)threadIdx.x + k * 64 * W;
        double v = 0.0;
        if (t < CRY * CRX) {
          const int ly = t / CRX, lx = t - ly * CRX;
          int Z = Zc, Y = cyo + ly, X = cxo + lx;
          if (Z >= 0 && Z <= ncs + 1 && Y <= ncs + 1 && X <= ncs + 1) {
            // the ghost layer holds the homogeneous extension: minus the adjacent cell
            double sg = 1.0;
            if (Z == 0) { Z = 1; sg = -sg; }
            if (Z == ncs + 1) { Z = ncs; sg = -sg; }
            if (Y == 0) { Y = 1; sg = -sg; }
            if (Y == ncs + 1) { Y = ncs; sg = -sg; }
            if (X == 0) { X = 1; sg = -sg; }
            if (X == ncs + 1) { X = ncs; sg = -sg; }
            const size_t mc = (size_t)ncs + 2;
            v = sg * a.ec[((size_t)Z * mc + (size_t)Y) * mc + (size_t)X];
          }
        }
        R[k] = v;
      }
    };
    auto cstore = [&](int Zc, const double (&R)[CLD]) {
      double* d = sh.cz[PRO ? Zc % 3 : 0];
#pragma unroll
      for (int k = 0; k < CLD; ++k) {
        const int t = (int)threadIdx.x + k * 64 * W;
        if (t < CRY * CRX) d[t] = R[k];
      }
    };
    // P e of a fine cell sums 8 terms in the order z, y, x, parent first: on the parent
    // plane the parent row (parent column, then the neighbour column) and the neighbour row,
    // then the same on the neighbour plane, with the weights kWp (parent column) and kWq
    // (neighbour column) of those four rows: products of 3/4 and 1/4, exact.
    constexpr double kWp[4] = {0.421875, 0.140625, 0.140625, 0.046875};
    constexpr double kWq[4] = {0.140625, 0.046875, 0.046875, 0.015625};
    auto planes_of = [&](int z, const double*& cp, const double*& cq) {
      const int pz = (z + 1) >> 1, qz = (z & 1) ? pz - 1 : pz + 1;
      cp = sh.cz[PRO ? pz % 3 : 0];
      cq = sh.cz[PRO ? qz % 3 : 0];
    };
    // P e at region rows yp (parent), yq (neighbour) and columns xp, xq of the two planes
    auto pe = [&](const double* cp, const double* cq, int yp, int yq, int xp, int xq) {
      double e = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double* row = (k < 2 ? cp : cq) + (k % 2 ? yq : yp) * CRX;
        const double e1 = e + kWp[k] * row[xp];
        e = e1 + kWq[k] * row[xq];
      }
      return e;
    };
    const int lyw = w * (RPW / 2) + 1;  // parent row (region) of the wave's first row pair
    const int hyp = w == 0 ? 0 : BY / 2 + 1, hyq = w == 0 ? 1 : BY / 2;
    double CR[CLD];                        // the coarse plane to be staged next
    double EXn[PRO ? RPW : 1], EXo[PRO ? RPW : 1];  // halo column's P e: last plane, the one before
#pragma unroll
    for (int i = 0; i < (PRO ? RPW : 1); ++i) EXn[i] = EXo[i] = 0.0;

    // Norm with zero_interior reads interior values of u as 0; the refinement pass adds
    // scale * e to them.
    auto adjust = [&](double v, float ev, bool in) -> double {
      if constexpr (FV) return v;
      else if constexpr (MODE == kNorm) return (a.zero_interior && in) ? 0.0 : v;
      else return (corr && in) ? v + a.scale * (double)ev : v;
    };

    // Queue of the planes s-1, s, s+1 (u adjusted; k); plane s+2 in flight.  f, the halo
    // column and the halo row are needed on plane s only: plane s+1 in flight.
    double U[3][RPW][CP][2], K[VAR ? 3 : 1][RPW][CP][2];
    double PU[RPW][CP][2], PK[RPW][CP][2];
    float PE[RPW][CP][2];
    double F[RPW][CP][2], PF[RPW][CP][2];
    double X[RPW], PX[RPW], XK[RPW], PXK[RPW];
    float PXE[RPW];
    double H[CP][2], PH[CP][2], HK[CP][2], PHK[CP][2];
    float PHE[CP][2];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      PXE[i] = 0.0f;
#pragma unroll
      for (int p = 0; p < CP; ++p) PE[i][p][0] = PE[i][p][1] = 0.0f;
    }
#pragma unroll
    for (int p = 0; p < CP; ++p) PHE[p][0] = PHE[p][1] = 0.0f;

    // finite-volume sweep from a zero iterate (a coarse level's first sweep: the correction
    // and its ghost layer are 0): u is not read
    const bool uzero = MODE == kFvJacobi && a.zero_interior;
    auto load_q = [&](int z) {
      const size_t zc = (size_t)min(max(z, 0), n - 1);
      const PlaneBuf bu = plane_buf(a.u, zc * planeb, planeb);
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int p = 0; p < CP; ++p) {
          if (uzero) PU[i][p][0] = PU[i][p][1] = 0.0;
          else buf_load2(bu, cb[p], rb8[i], PU[i][p][0], PU[i][p][1]);
        }
      if constexpr (VAR) {
        const PlaneBuf bk = plane_buf(a.k, zc * planeb, planeb);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int p = 0; p < CP; ++p) buf_load2(bk, cb[p], rb8[i], PK[i][p][0], PK[i][p][1]);
      }
      if (corr) {
        const PlaneBuf be = plane_buf(a.e, zc * planef, planef);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int p = 0; p < CP; ++p) buf_load2(be, cf[p], rb4[i], PE[i][p][0], PE[i][p][1]);
      }
    };
    // u + P e on plane z, the last plane of the queue (U[2]), for the lane's cells; the
    // halo column's values of plane z are kept until plane z is computed
    auto prolong_in = [&](int z) {
      const bool zin = z >= 1 && z <= n - 2;
#pragma unroll
      for (int i = 0; i < RPW; ++i) EXo[i] = EXn[i];
      if (!zin) return;
      const double *cp, *cq;
      planes_of(z, cp, cq);
#pragma unroll
      for (int i2 = 0; i2 < RPW / 2; ++i2) {
        const int yp = lyw + i2;
        // rows 2 i2 (odd: neighbour row below) and 2 i2 + 1 (even: above)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int i = 2 * i2 + j;
          if (!rin[i]) continue;
          const int yq = j ? yp + 1 : yp - 1;
#pragma unroll
          for (int p = 0; p < CP; ++p)
#pragma unroll
            for (int o = 0; o < 2; ++o) {
              const int xp = 64 * p + lane + 1;
              const double e = pe(cp, cq, yp, yq, xp, o ? xp + 1 : xp - 1);
              if (o ? in1[p] : in0[p]) U[2][i][p][o] = U[2][i][p][o] + e;
            }
          EXn[i] = pe(cp, cq, yp, yq, lane == 63 ? 64 * CP + 1 : 0, lane == 63 ? 64 * CP : 1);
        }
      }
    };
    // u + P e on plane s's halo column (kept from prolong_in) and halo row
    auto prolong_halo = [&](int s) {
#pragma unroll
      for (int i = 0; i < RPW; ++i)
        if (rin[i] && hcin) X[i] = X[i] + EXo[i];
      if (!(hw && hyin)) return;
      const double *cp, *cq;
      planes_of(s, cp, cq);
      double E[CP][2];
#pragma unroll
      for (int p = 0; p < CP; ++p)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const int xp = 64 * p + lane + 1;
          E[p][o] = pe(cp, cq, hyp, hyq, xp, o ? xp + 1 : xp - 1);
        }
#pragma unroll
      for (int p = 0; p < CP; ++p)
#pragma unroll
        for (int o = 0; o < 2; ++o)
          if (o ? in1[p] : in0[p]) H[p][o] = H[p][o] + E[p][o];
    };
    auto shift_in = [&](int z) {
      const bool zin = z >= 1 && z <= n - 2;
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int p = 0; p < CP; ++p)
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const double v = adjust(PU[i][p][o], PE[i][p][o], zin && rin[i] && (o ? in1[p] : in0[p]));
            U[0][i][p][o] = U[1][i][p][o]; U[1][i][p][o] = U[2][i][p][o]; U[2][i][p][o] = v;
            if constexpr (VAR) {
              K[0][i][p][o] = K[1][i][p][o]; K[1][i][p][o] = K[2][i][p][o]; K[2][i][p][o] = PK[i][p][o];
            }
          }
    };
    auto load_c = [&](int z) {
      const size_t zc = (size_t)min(max(z, 0), n - 1);
      const PlaneBuf bu = plane_buf(a.u, zc * planeb, planeb);
      const PlaneBuf bf = plane_buf(a.f, zc * planeb, planeb);
      const PlaneBuf bk = plane_buf(a.k, zc * planeb, planeb);
      const PlaneBuf be = plane_buf(a.e, zc * planef, planef);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
#pragma unroll
        for (int p = 0; p < CP; ++p) buf_load2(bf, cb[p], rb8[i], PF[i][p][0], PF[i][p][1]);
        PX[i] = uzero ? 0.0 : buf_load<double>(bu, hcb, rb8[i]);
        if constexpr (VAR) PXK[i] = buf_load<double>(bk, hcb, rb8[i]);
        if (corr) PXE[i] = buf_load<float>(be, hcf, rb4[i]);
      }
      if (hw) {
#pragma unroll
        for (int p = 0; p < CP; ++p) {
          if (uzero) PH[p][0] = PH[p][1] = 0.0;
          else buf_load2(bu, cb[p], hrb8, PH[p][0], PH[p][1]);
          if constexpr (VAR) buf_load2(bk, cb[p], hrb8, PHK[p][0], PHK[p][1]);
          if (corr) buf_load2(be, cf[p], hrb4, PHE[p][0], PHE[p][1]);
        }
      }
    };
    auto take_c = [&](int z) {
      const bool zin = z >= 1 && z <= n - 2;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
#pragma unroll
        for (int p = 0; p < CP; ++p) {
          F[i][p][0] = PF[i][p][0];
          F[i][p][1] = PF[i][p][1];
        }
        X[i] = adjust(PX[i], PXE[i], zin && rin[i] && hcin);
        if constexpr (VAR) XK[i] = PXK[i];
      }
#pragma unroll
      for (int p = 0; p < CP; ++p)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          H[p][o] = adjust(PH[p][o], PHE[p][o], zin && hyin && (o ? in1[p] : in0[p]));
          if constexpr (VAR) HK[p][o] = PHK[p][o];
        }
    };
    auto write_edges = [&](int buf, int slot) {
#pragma unroll
      for (int p = 0; p < CP; ++p)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          sh.eu[buf][w][0][p][o][lane] = U[slot][0][p][o];
          if constexpr (NE == 2) sh.eu[buf][w][1][p][o][lane] = U[slot][RPW - 1][p][o];
          if constexpr (VAR) {
            sh.ek[buf][w][0][p][o][lane] = K[slot][0][p][o];
            if constexpr (NE == 2) sh.ek[buf][w][1][p][o][lane] = K[slot][RPW - 1][p][o];
          }
        }
    };

    float RK[RPW][CP][2];
    double JV[JAC ? RPW : 1][CP][2];
    double RA[MODE == kFvRestrict ? RPW / 2 : 1][CP];  // coarse sums of the plane pair
    // coarse level (restriction): column byte offsets, dropped where the pair is not owned
    uint32_t cco[CP];
    const int mc = (n - 2) / 2 + 2;
    const uint32_t cplane = (uint32_t)((size_t)mc * (size_t)mc * 8u);
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const int c = ox + 128 * p + 2 * lane;
      cco[p] = in0[p] ? (uint32_t)((c + 1) / 2) * 8u : 0x80000000u;
    }
    double sumsq = 0.0, sumsq_b = 0.0;
    auto store = [&](int sp) {  // u_out from queue slot 0, r32 from RK
      const PlaneBuf bo = plane_buf(a.out, (size_t)sp * planeb, planeb);
      if constexpr (JAC) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          if (!rin[i]) continue;
#pragma unroll
          for (int p = 0; p < CP; ++p) buf_store2(JV[i][p][0], JV[i][p][1], bo, sb[p], rb8[i]);
        }
        return;
      }
      const PlaneBuf br = plane_buf(a.r32, (size_t)sp * planef, planef);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if (!rin[i]) continue;
#pragma unroll
        for (int p = 0; p < CP; ++p) {
          buf_store2(U[0][i][p][0], U[0][i][p][1], bo, sb[p], rb8[i]);
          buf_store2(RK[i][p][0], RK[i][p][1], br, sf[p], rb4[i]);
        }
      }
    };

    // prologue: planes z0-1, z0, z0+1 queued, the plane arrays of z0 taken, the edges of
    // plane z0 written for the first step.
    // Prolongation: the correction reaches plane q+1 of the queue at the start of step q
    // (after the loads of the step are issued, so that it overlaps their latency) and plane
    // q's halo column and row in step q.  Step q therefore reads the coarse planes
    // floor(q/2) .. floor((q+1)/2) + 1: coarse plane Z is first read in step 2Z-3 and last
    // in step 2Z+1, so it is staged in step 2Z-4 (even steps: one plane each) into the slot
    // of plane Z-3, last read in step 2Z-5.  With z0 = 2 Z0 - 1 (odd) the prologue stages
    // Z0-1 .. Z0+1 and loads Z0+2 (staged in step z0+1).
    if constexpr (PRO) {
      const int Z0 = (z0 + 1) / 2;
      cload(Z0 - 1, CR);
      cstore(Z0 - 1, CR);
      cload(Z0, CR);
      cstore(Z0, CR);
      cload(Z0 + 1, CR);
      cstore(Z0 + 1, CR);
      cload(Z0 + 2, CR);
      __syncthreads();
    }
    load_q(z0 - 1);
    shift_in(z0 - 1);
    if constexpr (PRO) prolong_in(z0 - 1);
    load_q(z0);
    shift_in(z0);
    if constexpr (PRO) prolong_in(z0);
    load_q(z0 + 1);
    shift_in(z0 + 1);
    load_c(z0);
    take_c(z0);
    write_edges(1, 1);

    auto stepfn = [&](auto BC, int s) {
      constexpr int bb = decltype(BC)::value;
      constexpr int rb = 1 - bb, wb = bb;  // LDS buffer written in the previous / this step
      __syncthreads();
      if constexpr (PRO) {
        if (bb == 1) {  // even step s: stage coarse plane s/2 + 2, load the next one
          cstore(s / 2 + 2, CR);
          cload(s / 2 + 3, CR);
        }
      }
      if ((REFINE || JAC) && s > z0) store(s - 1);
      const bool gzm = s == 1, gzp = s + 1 == n - 1;
      if (s + 2 <= z1) load_q(s + 2);
      if (s + 1 < z1) load_c(s + 1);
      if constexpr (PRO) {
        prolong_in(s + 1);  // the edges of plane s+1 are written at the end of this step
        prolong_halo(s);
      }
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
#pragma unroll
        for (int p = 0; p < CP; ++p) {
          // x-neighbours: the lane without a source lane takes the adjacent pair's edge lane
          // or, at the tile's edge, the halo column (lane 0 left, lane 63 right)
          const double fl = p == 0 ? X[i] : lane_value(U[1][i][p - 1][1], 63);
          const double fr = p == CP - 1 ? X[i] : lane_value(U[1][i][p + 1][0], 0);
          const double l1 = from_lane_below_or(U[1][i][p][1], fl);
          const double r0 = from_lane_above_or(U[1][i][p][0], fr);
          double kl1 = 0.0, kr0 = 0.0;
          if constexpr (VAR) {
            const double gl = p == 0 ? XK[i] : lane_value(K[1][i][p - 1][1], 63);
            const double gr = p == CP - 1 ? XK[i] : lane_value(K[1][i][p + 1][0], 0);
            kl1 = from_lane_below_or(K[1][i][p][1], gl);
            kr0 = from_lane_above_or(K[1][i][p][0], gr);
          }
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const double ui = U[1][i][p][o];
            const double xm = o == 0 ? l1 : U[1][i][p][0];
            const double xp = o == 0 ? U[1][i][p][1] : r0;
            double ym, yp, kym = 0.0, kyp = 0.0;
            if (i > 0) {
              ym = U[1][i - 1][p][o];
              if constexpr (VAR) kym = K[1][i - 1][p][o];
            } else {
              ym = w > 0 ? sh.eu[rb][wm][NE - 1][p][o][lane] : H[p][o];
              if constexpr (VAR) kym = w > 0 ? sh.ek[rb][wm][NE - 1][p][o][lane] : HK[p][o];
            }
            if (i < RPW - 1) {
              yp = U[1][i + 1][p][o];
              if constexpr (VAR) kyp = K[1][i + 1][p][o];
            } else {
              yp = w < W - 1 ? sh.eu[rb][wp][0][p][o][lane] : H[p][o];
              if constexpr (VAR) kyp = w < W - 1 ? sh.ek[rb][wp][0][p][o][lane] : HK[p][o];
            }
            const double zm = U[0][i][p][o], zp = U[2][i][p][o];
            double au;
            if constexpr (FV) {
              const bool gxm = o == 0 && gx0[p], gxp = o == 0 ? gxp0[p] : gxp1[p];
              au = fv_au(a.ih2, ui, gxm ? 2.0 * xm - ui : xm, gxp ? 2.0 * xp - ui : xp,
                         gym[i] ? 2.0 * ym - ui : ym, gyp[i] ? 2.0 * yp - ui : yp,
                         gzm ? 2.0 * zm - ui : zm, gzp ? 2.0 * zp - ui : zp);
            } else if constexpr (!VAR) {
              au = au_const<double, 3>(a.ih2, ui, xm, xp, ym, yp, zm, zp);
            } else {
              const double kxm = o == 0 ? kl1 : K[1][i][p][0];
              const double kxp = o == 0 ? K[1][i][p][1] : kr0;
              au = au_var<double, 3>(a.ih2, ui, K[1][i][p][o], xm, kxm, xp, kxp, ym, kym, yp,
                                     kyp, zm, K[0][i][p][o], zp, K[2][i][p][o]);
            }
            const double r = F[i][p][o] - au;
            const bool own = rin[i] && (o ? in1[p] : in0[p]);
            if (own) sumsq += r * r;
            if constexpr (RHS) {
              // interior neighbours (and the owned node itself) read as 0
              const int c = ox + 128 * p + 2 * lane + o, gy = oy + w * RPW + i;
              const bool ixm = c - 1 >= 1, ixp = c + 1 <= n - 2;
              const bool iym = gy - 1 >= 1, iyp = gy + 1 <= n - 2;
              const bool izm = s - 1 >= 1, izp = s + 1 <= n - 2;
              const double bau = au_const<double, 3>(a.ih2, 0.0, ixm ? 0.0 : xm, ixp ? 0.0 : xp,
                                                     iym ? 0.0 : ym, iyp ? 0.0 : yp,
                                                     izm ? 0.0 : zm, izp ? 0.0 : zp);
              const double bv = F[i][p][o] - bau;
              if (own) sumsq_b += bv * bv;
            }
            if constexpr (REFINE) RK[i][p][o] = own ? (float)(r * a.inv_scale) : 0.0f;
            if constexpr (JAC) JV[i][p][o] = ui + a.coef * r;
            if constexpr (MODE == kFvRestrict) {
              // steps of parity 0 are the odd (first) planes of a coarse cell's children
              if (bb == 0 && i % 2 == 0 && o == 0) RA[i / 2][p] = 0.0;
              RA[i / 2][p] = RA[i / 2][p] + r;
            }
          }
        }
      }
      if constexpr (MODE == kFvRestrict) {
        if (bb == 1) {  // second plane of the pair: the coarse values are complete
          const PlaneBuf bc = plane_buf(a.out, (size_t)(s / 2) * cplane, cplane);
#pragma unroll
          for (int i = 0; i < RPW; i += 2) {
            if (!rin[i]) continue;
            const int Y = (oy + w * RPW + i + 1) / 2;
            const uint32_t row = (uint32_t)(Y * mc) * 8u;
#pragma unroll
            for (int p = 0; p < CP; ++p) buf_store(RA[i / 2][p] / 8.0, bc, cco[p], row);
          }
        }
      }
      write_edges(wb, 2);  // edges of plane s+1
      shift_in(s + 2);
      if (s + 1 < z1) take_c(s + 1);
    };

    for (int s = z0; s < z1;) {
      stepfn(IC<0>{}, s);
      if (++s >= z1) break;
      stepfn(IC<1>{}, s);
      ++s;
    }
    if (REFINE || JAC) store(z1 - 1);  // queue slot 0 holds plane z1-1
    if constexpr (JAC || MODE == kFvRestrict) return;  // no norm

#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) sumsq += __shfl_xor(sumsq, o2, 64);
    if constexpr (RHS) {
#pragma unroll
      for (int o2 = 32; o2 >= 1; o2 >>= 1) sumsq_b += __shfl_xor(sumsq_b, o2, 64);
    }
    __syncthreads();
    if (lane == 0) sh.red[w] = sumsq;
    if (RHS && lane == 0) sh.redb[w] = sumsq_b;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int v = 0; v < W; ++v) tot += sh.red[v];
      a.partial[blockIdx.x] = tot;
      if constexpr (RHS) {
        double totb = 0.0;
        for (int v = 0; v < W; ++v) totb += sh.redb[v];
        a.partial_b[blockIdx.x] = totb;
      }
    }
  }
};

template <bool VAR, int MODE, int W, int RPW, int CP>
__global__ void __launch_bounds__(64 * W) k_pass(typename Pass<VAR, MODE, W, RPW, CP>::Args a)
{
  using C = Pass<VAR, MODE, W, RPW, CP>;
  __shared__ typename C::Shared sh;
  C::run(a, sh);
}

template <typename T, bool VAR, int MODE, int W, int RPW, int PD>
__global__ void __launch_bounds__(64 * W) k_stream(typename Stream<T, VAR, MODE, W, RPW, PD>::Args a)
{
  using C = Stream<T, VAR, MODE, W, RPW, PD>;
  __shared__ typename C::Shared sh;
  C::run(a, sh);
}

__global__ void __launch_bounds__(256)
    k_sum_fixed(const double* __restrict__ partial, int count, double* __restrict__ out)
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

template <typename Kernel>
int capacity_of(Kernel kernel, int block)
{
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
      per_cu = 1;
    cache[dev] = cus * per_cu;
  }
  return cache[dev];
}

// z-chunk length minimising (rounds of resident workgroups) x (planes per workgroup)
int best_zlen(int per_tile_plane_count, int zext, int halo, int capacity, int max_blocks)
{
  long long best = -1;
  int bestz = zext;
  for (int c = 1; c <= zext; ++c) {
    const int zlen = (zext + c - 1) / c;
    const int chunks = (zext + zlen - 1) / zlen;
    const long long blocks = (long long)per_tile_plane_count * chunks;
    if (blocks > max_blocks) break;
    const long long rounds = (blocks + capacity - 1) / capacity;
    const long long cost = rounds * (zlen + halo);
    if (best < 0 || cost < best) { best = cost; bestz = zlen; }
  }
  return bestz;
}

// Tile shapes (waves per workgroup x rows per wave), per pass, from timing sweeps on MI355X
// at 513^3: the restriction keeps 4 rows per wave (its coarse rows pair fine rows), the
// norm and the refinement pass favour more, lighter waves.
constexpr int kW = 8, kRPW = 4;          // restriction
constexpr int kNW = 8, kNRPW = 2;        // norm
constexpr int kRW = 16, kRRPW = 2;       // refinement pass
constexpr int kRVW = 8;                  // ... with variable k (16 waves would spill registers)
// Prefetch depth: 2 wherever the second buffer keeps the occupancy (the FP64
// variable-coefficient restriction would spill registers with it).
#ifndef MG_RESTRICT32_PD
#define MG_RESTRICT32_PD 2
#endif
template <typename T, bool VAR>
constexpr int restrict_pd()
{
  return (sizeof(T) == 4 && !VAR) ? MG_RESTRICT32_PD : (VAR && sizeof(T) == 8) ? 1 : 2;
}
// The FP64 variable-coefficient restriction holds k as well: 12 waves of 2 rows keep it
// within the register file.
#ifndef MG_RESTRICT32_W
#define MG_RESTRICT32_W 8
#endif
template <typename T, bool VAR>
constexpr int restrict_w()
{
  return (VAR && sizeof(T) == 8) ? 12 : (sizeof(T) == 4 && !VAR) ? MG_RESTRICT32_W : kW;
}
template <typename T, bool VAR>
constexpr int restrict_rpw()
{
  return (VAR && sizeof(T) == 8) ? 2 : kRPW;
}

}  // namespace

template <typename T>
void restrict_residual_tiled(hipStream_t s, int nf, double h, const T* k, const T* f,
                             const T* u, T* fc)
{
  const int nc = (nf - 1) / 2 + 1;
  const int m = nc - 2;
  auto launch = [&](auto kern, auto argsproto, int w, int rpw) {
    using A = decltype(argsproto);
    A a{};
    a.f = f; a.u = u; a.k = k; a.out = fc; a.n = nf; a.ih2 = (T)(1.0 / (h * h));
    a.tiles_x = (m + 61) / 62;
    const int cy = w * rpw / 2 - 2;
    a.tiles_y = (m + cy - 1) / cy;
    const int per = a.tiles_x * a.tiles_y;
    a.zlen = best_zlen(per, m, 1, capacity_of(kern, 64 * w), 1 << 30);
    const int blocks = per * ((m + a.zlen - 1) / a.zlen);
    kern<<<blocks, 64 * w, 0, s>>>(a);
  };
  constexpr int pv = restrict_pd<T, true>(), pc = restrict_pd<T, false>();
  constexpr int wv = restrict_w<T, true>(), rv = restrict_rpw<T, true>();
  constexpr int wc = restrict_w<T, false>();
  if (k)
    launch(k_stream<T, true, kRestrict, wv, rv, pv>,
           typename Stream<T, true, kRestrict, wv, rv, pv>::Args{}, wv, rv);
  else
    launch(k_stream<T, false, kRestrict, wc, kRPW, pc>,
           typename Stream<T, false, kRestrict, wc, kRPW, pc>::Args{}, wc, kRPW);
}

namespace {
// Shapes of the exact-partition passes (waves x rows per wave x column pairs per lane),
// from timing sweeps on MI355X at 513^3.
#ifndef MG_PASS_W
#define MG_PASS_W 8
#endif
#ifndef MG_PASS_RPW
#define MG_PASS_RPW 2
#endif
#ifndef MG_PASS_CP
#define MG_PASS_CP 2
#endif
#ifndef MG_PASS_VAR_W
#define MG_PASS_VAR_W 8
#endif
#ifndef MG_PASS_VAR_RPW
#define MG_PASS_VAR_RPW 1
#endif
#ifndef MG_PASS_VAR_CP
#define MG_PASS_VAR_CP 2
#endif

template <bool VAR, int MODE, int W, int RPW, int CP>
void launch_pass(hipStream_t s, typename Pass<VAR, MODE, W, RPW, CP>::Args a, double* partial,
                 double* out)
{
  using C = Pass<VAR, MODE, W, RPW, CP>;
  auto kern = k_pass<VAR, MODE, W, RPW, CP>;
  const int m = a.n - 2;
  a.tiles_x = (m + C::BX - 1) / C::BX;
  a.tiles_y = (m + C::BY - 1) / C::BY;
  const int per = a.tiles_x * a.tiles_y;
  // the first refinement pass takes the norm pass's z-chunks, so that its right-hand-side
  // norm is summed in the norm pass's order
  const int cap = (MODE == kRefineRhs || MODE == kNormRhs)
                      ? capacity_of(k_pass<VAR, kNorm, W, RPW, CP>, 64 * W)
                      : capacity_of(kern, 64 * W);
  a.zlen = best_zlen(per, m, 2, cap, kStreamPartials);
  const int blocks = per * ((m + a.zlen - 1) / a.zlen);
  a.partial = partial;
  kern<<<blocks, 64 * W, 0, s>>>(a);
  k_sum_fixed<<<1, 256, 0, s>>>(partial, blocks, out);
  if (MODE == kRefineRhs || MODE == kNormRhs)
    k_sum_fixed<<<1, 256, 0, s>>>(a.partial_b, blocks, out + 1);
}

template <bool VAR, int MODE>
void run_pass(hipStream_t s, typename Pass<VAR, MODE, 4, 2, 4>::Args a, double* partial,
              double* out)
{
  // Args does not depend on the shape
  constexpr int W = VAR ? MG_PASS_VAR_W : MG_PASS_W, RPW = VAR ? MG_PASS_VAR_RPW : MG_PASS_RPW;
  constexpr int CP = VAR ? MG_PASS_VAR_CP : MG_PASS_CP, CPS = CP < 2 ? CP : 2;
  using A = typename Pass<VAR, MODE, W, RPW, CP>::Args;
  using AS = typename Pass<VAR, MODE, W, RPW, CPS>::Args;
  static_assert(sizeof(A) == sizeof(a) && sizeof(AS) == sizeof(a), "argument layout");
  // a 256-column tile covers the interior row of n = 257
  if (a.n - 2 > 128 * CPS)
    launch_pass<VAR, MODE, W, RPW, CP>(s, __builtin_bit_cast(A, a), partial, out);
  else
    launch_pass<VAR, MODE, W, RPW, CPS>(s, __builtin_bit_cast(AS, a), partial, out);
}
}  // namespace

void resid_norm2_tiled(hipStream_t s, int n, double h, const double* k, const double* f,
                       const double* u, int mode, double* partial, double* out)
{
  auto fill = [&](auto& a) {
    a.f = f; a.u = u; a.k = k; a.n = n; a.ih2 = 1.0 / (h * h); a.zero_interior = mode;
  };
  if (k) {
    Pass<true, kNorm, 4, 2, 4>::Args a{};
    fill(a);
    run_pass<true, kNorm>(s, a, partial, out);
  } else {
    Pass<false, kNorm, 4, 2, 4>::Args a{};
    fill(a);
    run_pass<false, kNorm>(s, a, partial, out);
  }
}

void resid_norm2_both_tiled(hipStream_t s, int n, double h, const double* f, const double* u,
                            double* partial, double* partial_b, double* out)
{
  Pass<false, kNormRhs, 4, 2, 4>::Args a{};
  a.f = f; a.u = u; a.n = n; a.ih2 = 1.0 / (h * h); a.partial_b = partial_b;
  run_pass<false, kNormRhs>(s, a, partial, out);
}

void ir_pass_tiled(hipStream_t s, int n, double h, const double* k, const double* f,
                   const double* u, const float* e, double scale, double inv_scale, double* uout,
                   float* r32, double* partial, double* out, double* partial_b)
{
  auto fill = [&](auto& a) {
    a.f = f; a.u = u; a.k = k; a.n = n; a.ih2 = 1.0 / (h * h); a.e = e; a.scale = scale;
    a.inv_scale = inv_scale; a.out = uout; a.r32 = r32; a.partial_b = partial_b;
  };
  if (!k && partial_b && !e) {
    Pass<false, kRefineRhs, 4, 2, 4>::Args a{};
    fill(a);
    run_pass<false, kRefineRhs>(s, a, partial, out);
  } else if (k) {
    Pass<true, kRefine, 4, 2, 4>::Args a{};
    fill(a);
    run_pass<true, kRefine>(s, a, partial, out);
  } else {
    Pass<false, kRefine, 4, 2, 4>::Args a{};
    fill(a);
    run_pass<false, kRefine>(s, a, partial, out);
  }
}

namespace {
// Shape of the finite-volume passes: the norm and refinement shape, 256-column tiles from
// N = 256 on (two per row at N = 512), 128 columns below; the sweep with the prolongation
// has a shape of its own.
template <int MODE, typename Fill>
void launch_fv(hipStream_t s, int N, double* partial, double* out, Fill fill)
{
  constexpr bool PRO = MODE == kFvJacobiProlong;
  constexpr int W = PRO ? MG_FV_PROLONG_W : MG_PASS_W, RPW = PRO ? MG_FV_PROLONG_RPW : MG_PASS_RPW;
  auto go = [&](auto cpc) {
    constexpr int CP = decltype(cpc)::value;
    using C = Pass<false, MODE, W, RPW, CP>;
    auto kern = k_pass<false, MODE, W, RPW, CP>;
    typename C::Args a{};
    fill(a);
    a.n = N + 2;
    a.tiles_x = (N + C::BX - 1) / C::BX;
    a.tiles_y = (N + C::BY - 1) / C::BY;
    const int per = a.tiles_x * a.tiles_y;
    a.zlen = best_zlen(per, N, 2, capacity_of(kern, 64 * W), kStreamPartials);
    // chunks start on odd planes
    if (MODE == kFvRestrict || MODE == kFvJacobiProlong) a.zlen += a.zlen & 1;
    const int blocks = per * ((N + a.zlen - 1) / a.zlen);
    a.partial = partial;
    kern<<<blocks, 64 * W, 0, s>>>(a);
    if (MODE == kFvNorm) k_sum_fixed<<<1, 256, 0, s>>>(partial, blocks, out);
  };
  if (N > 128) go(IC<MODE == kFvJacobiProlong ? MG_FV_PROLONG_CP : 2>{});
  else go(IC<1>{});
}
}  // namespace

bool fv_tiled_supported(int N) { return N >= 128; }

void fv_jacobi_tiled(hipStream_t s, int N, double h, double omega, const double* f,
                     const double* u, double* uout, double* partial, bool zero_u)
{
  launch_fv<kFvJacobi>(s, N, partial, nullptr, [&](auto& a) {
    a.f = f; a.u = u; a.out = uout; a.ih2 = 1.0 / (h * h); a.coef = omega * (h * h / 6.0);
    a.zero_interior = zero_u ? 1 : 0;
  });
}

void fv_jacobi_prolong_tiled(hipStream_t s, int N, double h, double omega, const double* f,
                             const double* u, const double* ec, double* uout, double* partial)
{
  launch_fv<kFvJacobiProlong>(s, N, partial, nullptr, [&](auto& a) {
    a.f = f; a.u = u; a.ec = ec; a.out = uout; a.ih2 = 1.0 / (h * h);
    a.coef = omega * (h * h / 6.0);
  });
}

void fv_restrict_tiled(hipStream_t s, int N, double h, const double* f, const double* u,
                       double* fc, double* partial)
{
  launch_fv<kFvRestrict>(s, N, partial, nullptr, [&](auto& a) {
    a.f = f; a.u = u; a.out = fc; a.ih2 = 1.0 / (h * h);
  });
}

void fv_norm2_tiled(hipStream_t s, int N, double h, const double* f, const double* u,
                    double* partial, double* out)
{
  launch_fv<kFvNorm>(s, N, partial, out, [&](auto& a) {
    a.f = f; a.u = u; a.ih2 = 1.0 / (h * h);
  });
}

template void restrict_residual_tiled<double>(hipStream_t, int, double, const double*,
                                              const double*, const double*, double*);
template void restrict_residual_tiled<float>(hipStream_t, int, double, const float*,
                                             const float*, const float*, float*);

}  // namespace mgk
