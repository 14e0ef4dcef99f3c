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
//  - Stage j is exact on the nodes at least j+1 positions inside the loaded tile (and the
//    z-chunk's loaded range): their neighbours have completed stage j-1 exactly.  After 2S
//    stages the final nodes are those at least H = 2S positions inside: the loaded tile
//    overlaps its neighbours by 2H columns / rows / planes (redundant halo), so tiles are
//    independent and the result does not depend on the schedule.  Nodes nearer the edge
//    are updated too, from incomplete neighbours: such values are read only by other
//    nodes nearer the edge at later stages and are never stored, so every stage runs on
//    the whole tile without region tests.  Only nodes of the grid boundary (Dirichlet
//    values, read by interior neighbours) keep their values.
//  - Values live in registers: per lane a queue of H+2 planes (z-neighbours are own
//    registers), x-neighbours come from the adjacent lane by a cross-lane shuffle,
//    y-neighbours are own registers except across wave boundaries, where the first and
//    last row of each wave are exchanged through LDS (only the colour the next stage reads,
//    double-buffered by step parity so that one barrier per plane suffices).
//  - blockIdx -> tile is XCD-aware: a workgroup b runs on XCD b mod 8, so every XCD is given
//    a contiguous range of tiles, whose shared halo columns and rows then meet in the same L2.
#include "mg_buffer.h"
#include "mg_kernels.h"
#include "mg_lanes.h"
#include "mg_stencil.h"

#include <mutex>
#include <utility>
#include <vector>

namespace mgk {
namespace {

template <int V>
using IC = std::integral_constant<int, V>;

enum { kInRead = 0, kInZero = 1, kInProlong = 2 };

constexpr int imod(int a, int m) { return ((a % m) + m) % m; }

// Operands of the fused refinement (RES = 2); unused by the other passes.
struct RefineArgs {
  const double* u;        // FP64 iterate
  double* out;            // u + s_e e on interior nodes (boundary not written)
  const double* f;        // FP64 right-hand side
  float* r32;             // (f - A out) / s_r on interior nodes
  const double* scale_e;  // device scalar s_e (the scale of the cycle's right-hand side)
  const double* scale_r;  // device scalar s_r
  double ih2;             // 1 / h^2
  double* partial;        // per-workgroup sums of (f - A out)^2 over interior nodes
};

// RES = 1: the pass also computes the residual f - A u of the smoothed iterate and its
// full-weighting restriction onto the next coarser level (the smoother's output stays in
// registers instead of being read back by a separate restriction pass).  The residual of
// plane q needs the final planes q-1, q, q+1, so it runs one step after plane q+1 became
// final: two more queued planes, a 4-node wider tile overlap in x and y (the residual is
// exact one node, its full weighting two nodes further inside than the final values) and
// 2 more final planes at each end of the z-chunk.
//
// RES = 2 (FP32, constant coefficient, 2 sweeps, with the coarse-grid correction): the pass
// is the last post-smoothing of an FP32 correction cycle and also performs the iterative
// refinement step that follows it -- u_out = u + s_e e on interior nodes (u, u_out FP64),
// r = f - A u_out in FP64, r32 = (float)(r / s_r) and the sum of r^2 -- with the arithmetic of
// the separate refinement pass, so the smoothed correction is never stored.  The residual of
// plane q needs the corrected iterate on planes q-1, q, q+1, formed as each plane of the
// correction becomes final: a 2-node wider tile overlap in x and y (the residual is exact
// one node further inside than the correction) and one more final plane at each end of the
// z-chunk; the corrected planes wait in a ring of three per lane.
//
// LW = lanes per tile row: 64 (a wave's lanes span the tile's 128 columns), or 32 (the tile
// is 64 columns wide and each wave holds two row bands of RPW rows, lanes 0-31 the first and
// lanes 32-63 the second: a squarer tile of the same node count, with less halo per output
// node).  A band of 32 lanes is then a "row group" of its own: it exchanges edge rows with
// the neighbouring groups through LDS like a wave does, and its x-neighbours come from the
// adjacent lanes by the same wave-wide shift -- lane 32's left neighbour is lane 31 of the
// other band, a value of another row, but column 0 of a tile is never exact (nor is column
// 63, which receives lane 32's value), so no exact value reads it.
template <typename T, bool VAR, int S, int W, int RPW, int PD, int RES = 0, int LW = 64>
struct Tiled {
  static_assert(PD == 1 || PD == 2, "prefetch depth");
  static_assert(RES == 0 || (!VAR && S == 2), "the fused restriction serves the plain 2-sweep pass");
  static_assert(RES != 2 || sizeof(T) == 4, "the fused refinement follows an FP32 cycle");
  static constexpr bool REF = RES == 2;
  static_assert(LW == 64 || LW == 32, "lanes per tile row");
  static constexpr int G = 64 / LW;      // row groups per wave
  static constexpr int VW = W * G;       // row groups per tile
  static constexpr int H = 2 * S;        // halo = number of stages
  static constexpr int BX = 2 * LW;      // columns per tile (2 per lane)
  static constexpr int BY = VW * RPW;    // rows per tile
  static constexpr int XR = RES == 1 ? 4 : REF ? 2 : 0;  // extra overlap: restriction, refinement
  static constexpr int ZR = RES == 1 ? 2 : REF ? 1 : 0;  // extra final planes at each end of a z-chunk
  static constexpr int TXO = BX - 2 * H - XR; // output columns per tile (tile stride)
  static constexpr int TYO = BY - 2 * H - XR; // output rows per tile
  static constexpr int Q = H + 2 + (RES == 1 ? 2 : 0);  // planes held per lane (even)
  static_assert(!REF || Q % 3 == 0, "the ring of corrected planes follows the queue's phases");
  static_assert(RPW % 2 == 0, "row parity must be uniform across the waves of a tile");
  static_assert(TYO > 0, "tile too short for the halo");

  struct Shared {
    T eu[2][H][VW][2][LW];                     // row-group boundary rows of u
    T ek[VAR ? 2 : 1][VAR ? H : 1][VW][2][LW]; // and of k
    T er[RES == 1 ? 2 : 1][RES == 1 ? VW : 1][2][2][LW]; // RES 1: both columns of a final plane's edge rows
    T erx[RES == 1 ? 2 : 1][RES == 1 ? VW : 1][LW];      // RES 1: x-filtered residual of a group's first row
    double eun[REF ? 2 : 1][REF ? VW : 1][2][2][LW];     // REF: edge rows of a corrected plane
    double red[REF ? W : 1];                             // REF: per-wave sums of r^2
  };

  // The first column of every lane and the first row of every row group have odd global
  // indices (tile origins are odd, H and RPW even): the fused prolongation relies on it.
  static_assert(TXO % 2 == 0 && TYO % 2 == 0 && H % 2 == 0, "odd tile origins");

  // B0 = parity of (global x of column 0) + (global y of row 0) + z0 - 1 + ZR (see below).
  // IN: how the input is formed -- kInRead: uin; kInZero: 0 (uin not read);
  // kInProlong: uin + P ec, the coarse-grid correction ec (nc nodes per side) interpolated
  // with the same weights and summation order as the stand-alone prolongation kernel.
  template <int B0, int IN>
  __device__ __forceinline__ static void run(const T* __restrict__ uin, T* __restrict__ uout,
                                             const T* __restrict__ f, const T* __restrict__ k,
                                             const T* __restrict__ ec, int nc,
                                             int n, T h2, int ox, int oy, int z0, int z1,
                                             T ih2, T* __restrict__ fc, const RefineArgs& ra,
                                             Shared& sh)
  {
    static_assert(!REF || IN == kInProlong, "the fused refinement follows the post-smoothing");
    // lane within its row group, and the row group (wave-uniform for LW = 64, so that row
    // bookkeeping stays scalar there)
    const int lane = threadIdx.x & (LW - 1);
    const int w = LW == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)
                           : (int)(threadIdx.x >> 5);
    const int gxa = ox - H + 2 * lane;  // global x of this lane's first column
    const int gyw = oy - H + w * RPW;   // global y of this row group's first row
    const int wm = w > 0 ? w - 1 : 0, wp = w < VW - 1 ? w + 1 : VW - 1;  // adjacent groups

    // Addresses: a wave-uniform plane + row base (scalar registers; per lane for LW = 32)
    // plus a per-lane 32-bit column byte offset.  Coordinates outside the grid are clamped
    // onto it, so every load is in bounds; such positions are never updated and never read
    // by an exact value.  Bit 2i+o of `upd` (per lane): node (row i, column o) is interior
    // to the grid and may be updated.  Stores go to output rows (`rowout`) at the column
    // offset `sxb`, which is out of the plane's range -- the store is dropped -- for columns
    // that are not output columns of this tile.
    uint32_t cxb[2], sxb[2];
    unsigned upd = 0, rowout = 0;
    uint32_t rowb[RPW];  // clamped row start within a plane, in bytes
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const int gx = gxa + o, px = 2 * lane + o;
      const bool cin = gx >= 1 && gx <= n - 2;
      const bool cout = cin && px >= H && px < H + TXO;
      cxb[o] = (uint32_t)min(max(gx, 0), n - 1) * (uint32_t)sizeof(T);
      sxb[o] = cout ? cxb[o] : 0x80000000u;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int gy = gyw + i;
        upd |= (cin && gy >= 1 && gy <= n - 2) ? 1u << (2 * i + o) : 0u;
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int gy = gyw + i, pr = w * RPW + i;
      rowout |= (gy >= 1 && gy <= n - 2 && pr >= H && pr < H + TYO) ? 1u << i : 0u;
      rowb[i] = (uint32_t)(min(max(gy, 0), n - 1) * n) * (uint32_t)sizeof(T);
    }
    const uint32_t planeb = (uint32_t)((size_t)n * (size_t)n * sizeof(T));
    // Plane accesses at (row offset ro, column offset co): the row offset is the scalar
    // operand for LW = 64 and joins the per-lane offset for LW = 32.  Out-of-range column
    // offsets stay out of range.
    auto ld = [](PlaneBuf b, uint32_t co, uint32_t ro) -> T {
      if constexpr (LW == 64) return buf_load<T>(b, co, ro);
      else return buf_load<T>(b, co + ro, 0u);
    };

    T U[Q][RPW][2], F[Q][RPW][2], K[Q][RPW][2];
    // Prefetch buffers: plane zl+PD is loaded in the step that inserts plane zl, so each
    // load has PD steps' work to arrive in; with PD = 2 the buffer is chosen by the
    // plane's parity.
    T PU[PD][RPW][2], PF[PD][RPW][2], PK[PD][RPW][2];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          U[q][i][o] = T(0);
          F[q][i][o] = T(0);
          K[q][i][o] = T(0);
        }

    // Fused prolongation: coarse column cxa = (gxa - 1) / 2 and cxa + 1, coarse rows
    // cya .. cya + RPW/2 with cya = (gyw - 1) / 2, and the coarse planes floor(zl/2) (CA) and
    // floor(zl/2) + 1 (CB, odd zl only), all clamped into the coarse grid, loaded with the
    // fine plane into its prefetch buffer.
    // (Byte offsets: coarse rows uniform, coarse columns per lane.)
    constexpr int CR = RPW / 2 + 1;
    T CA[PD][CR][2], CB[PD][CR][2];
    uint32_t ccb[2] = {0, 0}, crb[CR];  // crb: uniform for LW = 64
    const uint32_t cplaneb = (uint32_t)((size_t)nc * (size_t)nc * sizeof(T));
    if (IN == kInProlong) {
      const int cxa = (gxa - 1) >> 1;
      ccb[0] = (uint32_t)min(max(cxa, 0), nc - 1) * (uint32_t)sizeof(T);
      ccb[1] = (uint32_t)min(max(cxa + 1, 0), nc - 1) * (uint32_t)sizeof(T);
      const int cya = (gyw - 1) >> 1;
#pragma unroll
      for (int r = 0; r < CR; ++r)
        crb[r] = (uint32_t)(min(max(cya + r, 0), nc - 1) * nc) * (uint32_t)sizeof(T);
    }
    auto load_coarse = [&](T (&E)[CR][2], int cz) {
      const PlaneBuf be = plane_buf(ec, (size_t)min(max(cz, 0), nc - 1) * cplaneb, cplaneb);
#pragma unroll
      for (int r = 0; r < CR; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) E[r][c] = ld(be, ccb[c], crb[r]);
    };

    // Loads of plane zl (parity ZP, known at compile time: see the step below) into
    // prefetch buffer BUF.
    auto load = [&](int zl, auto ZPC, auto BUFC) {
      constexpr int zp = decltype(ZPC)::value;
      constexpr int bf_ = decltype(BUFC)::value;
      const size_t zc = (size_t)min(max(zl, 0), n - 1);
      if constexpr (IN == kInProlong) {
        load_coarse(CA[bf_], zl >> 1);
        if constexpr (zp == 1) load_coarse(CB[bf_], (zl >> 1) + 1);
      }
      const size_t zb = zc * planeb;
      const PlaneBuf bu = plane_buf(uin, zb, planeb), bf = plane_buf(f, zb, planeb);
      const PlaneBuf bk = plane_buf(VAR ? k : f, zb, planeb);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          PU[bf_][i][o] = IN == kInZero ? T(0) : ld(bu, cxb[o], rowb[i]);
          PF[bf_][i][o] = ld(bf, cxb[o], rowb[i]);
          if constexpr (VAR) PK[bf_][i][o] = ld(bk, cxb[o], rowb[i]);
        }
      }
    };

    // Plane zl enters the queue one step after its loads were issued, so that no arithmetic
    // waits on them early; in kInProlong it gains the interpolated coarse-grid correction
    // P ec on interior nodes (coarse rows of a fine row
    // i: i/2, i/2+1 for even i (odd fine y), (i+1)/2 for odd i; coarse columns cxa, cxa+1 for
    // column 0 (odd fine x), cxa+1 for column 1; coarse planes CA (and CB for odd zl)).
    auto insert = [&](int zl, auto S0C, auto ZPC, auto BUFC) {
      constexpr int s0 = decltype(S0C)::value;
      constexpr int zp = decltype(ZPC)::value;
      constexpr int bf_ = decltype(BUFC)::value;
      const bool zin = zl >= 1 && zl <= n - 2;
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          T v = PU[bf_][i][o];
          if constexpr (IN == kInProlong) {
            constexpr int mz = zp ? 2 : 1;
            const T wz = zp ? T(0.5) : T(1);
            const int my = (i % 2 == 0) ? 2 : 1;
            const int rb = (i % 2 == 0) ? i / 2 : (i + 1) / 2;
            const T wy = (i % 2 == 0) ? T(0.5) : T(1);
            const int mx = o == 0 ? 2 : 1;
            const int cb = o == 0 ? 0 : 1;
            const T wx = o == 0 ? T(0.5) : T(1);
            T sum = T(0);
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
              if (a2 >= mz) break;
#pragma unroll
              for (int b2 = 0; b2 < my; ++b2)
#pragma unroll
                for (int c2 = 0; c2 < mx; ++c2)
                  sum = sum + (wz * wy * wx) * (a2 == 0 ? CA[bf_][rb + b2][cb + c2]
                                                        : CB[bf_][rb + b2][cb + c2]);
            }
            const bool in = zin && ((upd >> (2 * i + o)) & 1u);
            if (in) v = v + sum;
          }
          U[s0][i][o] = v;
          F[s0][i][o] = PF[bf_][i][o];
          if constexpr (VAR) K[s0][i][o] = PK[bf_][i][o];
        }
    };

    // final plane pout (queue slot SO) -> uout, if it belongs to this z-chunk
    auto store = [&](int pout, auto SOC) {
      constexpr int so = decltype(SOC)::value;
      if (REF || pout < z0 || pout >= z1) return;  // REF: the correction is not stored
      const PlaneBuf bo = plane_buf(uout, (size_t)pout * planeb, planeb);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if constexpr (LW == 64) {
          if (!((rowout >> i) & 1u)) continue;
#pragma unroll
          for (int o = 0; o < 2; ++o) buf_store(U[so][i][o], bo, sxb[o], rowb[i]);
        } else {
          // per-lane rows: a row that is not an output row takes the out-of-range offset
          const bool ro = (rowout >> i) & 1u;
#pragma unroll
          for (int o = 0; o < 2; ++o)
            buf_store(U[so][i][o], bo,
                      (ro && sxb[o] != 0x80000000u) ? sxb[o] + rowb[i] : 0x80000000u, 0u);
        }
      }
    };

    const int zbeg = z0 - H - ZR, zend = z1 + H + ZR;  // planes loaded: [zbeg, zend)
    // RES: one more step completes the restriction of the last residual plane
    const int zstop = zend + (RES == 1 ? 1 : 0);
    int zl = zbeg;

    // Fused restriction (RES): lane column 1 is the even fine column 2X of coarse column X
    // (tile origins are odd), rows with odd i are the even fine rows 2Y.  Coarse nodes owned
    // by this tile: 2X in [ox + 2, ox + 2 + TXO), from 2 in the first tile (ox = 1), 2Y
    // likewise, 2Z in [z0, z1) -- a partition of the coarse interior.  Each lies at least 6
    // nodes inside the loaded tile, or next to the grid boundary, whose values are exact.
    const int gxc = gxa + 1;
    const int xlo = ox == 1 ? 2 : ox + 2, ylo = oy == 1 ? 2 : oy + 2;
    const bool cown = RES == 1 && gxc >= xlo && gxc < ox + 2 + TXO && gxc <= n - 3;
    unsigned crown = 0;
#pragma unroll
    for (int i = 1; i < RPW; i += 2) {
      const int gy = gyw + i;
      crown |= (gy >= ylo && gy < oy + 2 + TYO && gy <= n - 3) ? 1u << i : 0u;
    }
    T rxprev[RPW], acc[RPW / 2];
#pragma unroll
    for (int i = 0; i < RPW; ++i) rxprev[i] = T(0);
#pragma unroll
    for (int i = 0; i < RPW / 2; ++i) acc[i] = T(0);
    load(zl, IC<(B0 + 1) & 1>{}, IC<0>{});
    if constexpr (PD == 2) load(zl + 1, IC<B0 & 1>{}, IC<1>{});

    // One step for phase P = step mod Q: the plane zl - d sits in queue slot (P - d) mod Q.
    // The update column of row i in this step is o_i = (B0 + i + P) & 1, because the
    // colour of (x, y, p) is (x + y + p) & 1 and, at stage j, colour j&1 and p = zl-1-j
    // make x's parity depend on zl only.  Tile origins are odd, so B0 = (z0 - 1 + ZR) & 1,
    // and zl = z0 - H - ZR + step with H and Q even: zl has the parity (B0 + 1 + P) & 1,
    // and the step that of P.
    // RES, at the end of step zl (phase P): (1) full weighting in y and z of the residual
    // plane zl-H-2, x-filtered in the previous step; (2) residual of plane q = zl-H-1 (its
    // neighbours q-1, q, q+1 are final) and its full weighting in x; (3) both columns of the
    // edge rows of the plane zl-H that became final in this step, for the next step's
    // residual.  Same operations, in the same order, as the stand-alone restriction pass.
    auto restrict_step = [&](auto PC) {
      constexpr int P = decltype(PC)::value;
      constexpr int rb = (P + 1) & 1, wb = P & 1;
      constexpr int zpar = (B0 + 1 + P) & 1;  // parity of zl, of zl-H-2 and of zl-H
      const int qp = zl - H - 2;
      if (qp >= z0 - 1 && qp <= z1) {
        T ry[RPW / 2];
#pragma unroll
        for (int i = 1; i < RPW; i += 2) {
          const T below = i + 1 < RPW ? rxprev[i + 1] : sh.erx[rb][wp][lane];
          ry[i / 2] = (T(0.25) * rxprev[i - 1] + T(0.5) * rxprev[i]) + T(0.25) * below;
        }
        if constexpr (zpar == 1) {
          // odd plane qp = 2Z+1 completes coarse plane Z and starts plane Z+1
          const int Z = (qp - 1) >> 1;
          const bool zown = 2 * Z >= z0 && 2 * Z < z1 && Z >= 1 && Z <= nc - 2;
#pragma unroll
          for (int i = 1; i < RPW; i += 2) {
            const T done = acc[i / 2] + T(0.25) * ry[i / 2];
            if (zown && cown && ((crown >> i) & 1u))
              fc[((size_t)Z * nc + (size_t)((gyw + i) >> 1)) * (size_t)nc + (size_t)(gxc >> 1)] = done;
            acc[i / 2] = T(0.25) * ry[i / 2];
          }
        } else {
#pragma unroll
          for (int i = 1; i < RPW; i += 2) acc[i / 2] = acc[i / 2] + T(0.5) * ry[i / 2];
        }
      }
      const int q = zl - H - 1;
      if (q >= z0 - 1 && q <= z1) {
        constexpr int cq = imod(P - H - 1, Q), cm = imod(P - H - 2, Q), cp = imod(P - H, Q);
        const bool zin = q >= 1 && q <= n - 2;
        T r[RPW][2];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const T l1 = from_lane_below(U[cq][i][1]);
          const T r0 = from_lane_above(U[cq][i][0]);
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const T xm = o == 0 ? l1 : U[cq][i][0];
            const T xp = o == 0 ? U[cq][i][1] : r0;
            const T ym = i > 0 ? U[cq][i - 1][o] : sh.er[rb][wm][1][o][lane];
            const T yp = i < RPW - 1 ? U[cq][i + 1][o] : sh.er[rb][wp][0][o][lane];
            const T au = au_const<T, 3>(ih2, U[cq][i][o], xm, xp, ym, yp, U[cm][i][o], U[cp][i][o]);
            const T rv = F[cq][i][o] - au;
            // fine nodes outside the interior carry no residual
            r[i][o] = (zin && ((upd >> (2 * i + o)) & 1u)) ? rv : T(0);
          }
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i)
          rxprev[i] = (T(0.25) * r[i][0] + T(0.5) * r[i][1]) + T(0.25) * from_lane_above(r[i][0]);
        sh.erx[wb][w][lane] = rxprev[0];
      }
      constexpr int cf = imod(P - H, Q);
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        sh.er[wb][w][0][o][lane] = U[cf][0][o];
        sh.er[wb][w][1][o][lane] = U[cf][RPW - 1][o];
      }
    };

    // Fused refinement (REF).  Nodes whose residual this tile owns: columns [rxlo, rxhi) and
    // rows [rylo, ryhi) (from 1 in the first tile; tiles advance by TXO, TYO), planes
    // [z0, z1); each lies at least H + 1 nodes inside the loaded tile, or next to the grid
    // boundary.  The FP64 iterate is loaded on the owned nodes and one node around them,
    // f on the owned nodes; other lanes' accesses take an out-of-range offset (no traffic).
    constexpr uint32_t kOff = 0x80000000u;
    unsigned rown = 0, rneed = 0;  // bit 2i+o: owned node; node whose iterate is loaded
    uint32_t dxo[2] = {kOff, kOff}, dxn[2] = {kOff, kOff};  // FP64 column byte offsets
    if constexpr (REF) {
      const int rxlo = ox == 1 ? 1 : ox + 1, rxhi = min(ox + 1 + TXO, n - 1);
      const int rylo = oy == 1 ? 1 : oy + 1, ryhi = min(oy + 1 + TYO, n - 1);
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int gx = gxa + o;
        const bool xo = gx >= rxlo && gx < rxhi, xn = gx >= rxlo - 1 && gx <= rxhi;
        dxo[o] = xo ? (uint32_t)gx * 8u : kOff;
        dxn[o] = xn ? (uint32_t)gx * 8u : kOff;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int gy = gyw + i;
          const bool yo = gy >= rylo && gy < ryhi, yn = gy >= rylo - 1 && gy <= ryhi;
          rown |= (xo && yo) ? 1u << (2 * i + o) : 0u;
          rneed |= (xn && yn) ? 1u << (2 * i + o) : 0u;
        }
      }
    }
    const uint32_t planed = 2u * planeb;  // FP64 plane bytes
    // FP64 access at node (i, o): the lane offset (out of range where `mask` has no bit)
    // plus the row offset (rows are 2 x the FP32 row offsets)
    auto ld8 = [&](PlaneBuf b, unsigned mask, int i, int o, const uint32_t (&dx)[2]) -> double {
      const uint32_t co = ((mask >> (2 * i + o)) & 1u) ? dx[o] : kOff;
      if constexpr (LW == 64) return buf_load<double>(b, co, 2u * rowb[i]);
      else return buf_load<double>(b, co + 2u * rowb[i], 0u);
    };
    // corrected planes, ring slot = phase mod 3; the slot of plane zl-H receives its
    // iterate's loads at the start of step zl (its previous plane, zl-H-3, was last read in
    // step zl-1) and the correction at the end
    double UN[REF ? 3 : 1][REF ? RPW : 1][2];
    double PFD[REF ? RPW : 1][2];  // f of plane zl-H-1
#pragma unroll
    for (int a3 = 0; a3 < (REF ? 3 : 1); ++a3)
#pragma unroll
      for (int i = 0; i < (REF ? RPW : 1); ++i) UN[a3][i][0] = UN[a3][i][1] = 0.0;
    double sumsq = 0.0;
    double se = 0.0, sr = 1.0;  // correction scale, r32 = r * sr
    if constexpr (REF) {
      se = ra.scale_e[0];
      sr = 1.0 / ra.scale_r[0];
    }
    // loads of the step that completes plane zl-H: its iterate, and f of plane zl-H-1
    auto refine_load = [&](auto PC) {
      constexpr int sn = imod(decltype(PC)::value, 3);
      const int pf = zl - H, q = pf - 1;
      if (pf >= z0 - 1 && pf <= z1) {
        const PlaneBuf bu = plane_buf(ra.u, (size_t)pf * planed, planed);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int o = 0; o < 2; ++o) UN[sn][i][o] = ld8(bu, rneed, i, o, dxn);
      }
      if (q >= z0 && q < z1) {
        const PlaneBuf bf = plane_buf(ra.f, (size_t)q * planed, planed);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int o = 0; o < 2; ++o) PFD[i][o] = ld8(bf, rown, i, o, dxo);
      }
    };
    // End of step zl (phase P): (1) plane pf = zl-H is final: its corrected iterate
    // u + s_e e (interior nodes; u elsewhere) enters ring slot P mod 3 and its edge rows go
    // to LDS; (2) the residual of plane q = pf-1 (the corrected planes q-1, q, q+1 are in the
    // ring, the adjacent groups' edge rows of q in the LDS buffer of the previous step),
    // stored with the corrected iterate on the owned nodes.  The operations and their order
    // are those of the separate refinement pass.
    auto refine_step = [&](auto PC) {
      constexpr int P = decltype(PC)::value;
      constexpr int rb = (P + 1) & 1, wb = P & 1;
      constexpr int sn = imod(P, 3), sq = imod(P - 1, 3), sm = imod(P - 2, 3);
      constexpr int cfin = imod(P - H, Q);  // queue slot of plane zl-H
      const int pf = zl - H, q = pf - 1;
      if (pf >= z0 - 1 && pf <= z1) {
        const bool zin = pf >= 1 && pf <= n - 2;
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const bool in = zin && ((upd >> (2 * i + o)) & 1u);
            if (in) UN[sn][i][o] = UN[sn][i][o] + se * (double)U[cfin][i][o];
          }
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          sh.eun[wb][w][0][o][lane] = UN[sn][0][o];
          sh.eun[wb][w][1][o][lane] = UN[sn][RPW - 1][o];
        }
      }
      if (q >= z0 && q < z1) {
        const PlaneBuf bo = plane_buf(ra.out, (size_t)q * planed, planed);
        const PlaneBuf br = plane_buf(ra.r32, (size_t)q * planeb, planeb);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const double l1 = from_lane_below(UN[sq][i][1]);
          const double r0 = from_lane_above(UN[sq][i][0]);
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const double ui = UN[sq][i][o];
            const double xm = o == 0 ? l1 : UN[sq][i][0];
            const double xp = o == 0 ? UN[sq][i][1] : r0;
            const double ym = i > 0 ? UN[sq][i - 1][o] : sh.eun[rb][wm][1][o][lane];
            const double yp = i < RPW - 1 ? UN[sq][i + 1][o] : sh.eun[rb][wp][0][o][lane];
            const double au =
                au_const<double, 3>(ra.ih2, ui, xm, xp, ym, yp, UN[sm][i][o], UN[sn][i][o]);
            const double r = PFD[i][o] - au;
            const bool own = (rown >> (2 * i + o)) & 1u;
            if (own) sumsq += r * r;
            const float rk = (float)(r * sr);
            const uint32_t cd = own ? dxo[o] : kOff;
            const uint32_t cs = own ? dxo[o] >> 1 : kOff;  // FP32 column offset
            if constexpr (LW == 64) {
              buf_store(ui, bo, cd, 2u * rowb[i]);
              buf_store(rk, br, cs, rowb[i]);
            } else {
              buf_store(ui, bo, cd + 2u * rowb[i], 0u);
              buf_store(rk, br, cs + rowb[i], 0u);
            }
          }
        }
      }
    };

    auto body = [&](auto PC) -> bool {
      constexpr int P = decltype(PC)::value;
      constexpr int s0 = imod(P, Q);
      constexpr int zpar = (B0 + 1 + P) & 1;
      constexpr int buf = PD == 2 ? (P & 1) : 0;
      // the prefetched plane zl enters the queue
      insert(zl, IC<s0>{}, IC<zpar>{}, IC<buf>{});
      // Finish the inserted values here: left to the optimiser, the interpolation sinks
      // to the first use in the stages, keeping the previous loads and partial sums live
      // alongside the next plane's loads (an empty asm statement emits no instruction).
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int o = 0; o < 2; ++o) asm volatile("" : "+v"(U[s0][i][o]));
      __syncthreads();
      // Plane zl-1-H became final in the previous step and is still queued (slot
      // P-H-1): storing it here, just before the next loads, lets the stores complete in
      // the shadow of the loads instead of delaying the next step's wait for them.
      store(zl - 1 - H, IC<imod(P - H - 1, Q)>{});
      // REF: the FP64 loads, consumed at the end of this step, go first -- memory
      // instructions complete in order, so the wait for them then leaves the prefetch of
      // the next plane in flight
      if constexpr (REF) refine_load(IC<P>{});
      if (zl + PD < zend) load(zl + PD, IC<PD == 2 ? zpar : 1 - zpar>{}, IC<buf>{});
      constexpr int rb = (P + 1) & 1;  // LDS buffer written in the previous step
      constexpr int wb = P & 1;        // LDS buffer written in this step

#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int p = zl - 1 - j;
        if (p < 1 || p > n - 2) continue;  // boundary planes keep their values (uniform)
        const int cs = imod(P - 1 - j, Q);  // centre plane p
        const int cm = imod(P - 2 - j, Q);  // plane p - 1
        const int cp = imod(P - j, Q);      // plane p + 1
        const int pslot = imod(p, H);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
          const int o = (B0 + i + P) & 1;
          // x-neighbours: own other column, or the neighbouring lane's
          T xm, xp, kxm = T(0), kxp = T(0);
          if (o == 0) {
            xm = from_lane_below(U[cs][i][1]);
            xp = U[cs][i][1];
            if constexpr (VAR) { kxm = from_lane_below(K[cs][i][1]); kxp = K[cs][i][1]; }
          } else {
            xm = U[cs][i][0];
            xp = from_lane_above(U[cs][i][0]);
            if constexpr (VAR) { kxm = K[cs][i][0]; kxp = from_lane_above(K[cs][i][0]); }
          }
          // y-neighbours in column o: own rows, or the adjacent wave's edge row (the first
          // and the last wave read their own rows there: tile-edge values, never exact)
          T ym, yp, kym = T(0), kyp = T(0);
          if (i > 0) {
            ym = U[cs][i - 1][o];
            if constexpr (VAR) kym = K[cs][i - 1][o];
          } else {
            ym = sh.eu[rb][pslot][wm][1][lane];
            if constexpr (VAR) kym = sh.ek[rb][pslot][wm][1][lane];
          }
          if (i < RPW - 1) {
            yp = U[cs][i + 1][o];
            if constexpr (VAR) kyp = K[cs][i + 1][o];
          } else {
            yp = sh.eu[rb][pslot][wp][0][lane];
            if constexpr (VAR) kyp = sh.ek[rb][pslot][wp][0][lane];
          }
          T zm = U[cm][i][o], zp = U[cp][i][o];
          if (IN == kInZero && j == 0) {
            // from a zero guess the first stage's neighbours are all still 0 (the other
            // colour of planes p-1, p, p+1 and the boundary): the same formula on literal
            // zeros, which the compiler folds
            xm = xp = ym = yp = zm = zp = T(0);
          }
          const T h2f = h2 * F[cs][i][o];
          T v;
          if (!VAR) {
            v = gs_const<T, 3>(h2f, xm, xp, ym, yp, zm, zp);
          } else {
            v = gs_var<T, 3>(h2f, K[cs][i][o], xm, kxm, xp, kxp, ym, kym, yp, kyp, zm,
                             K[cm][i][o], zp, K[cp][i][o]);
          }
          const bool act = (upd >> (2 * i + o)) & 1u;
          U[cs][i][o] = act ? v : U[cs][i][o];
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
          constexpr int o = (B0 + i + P) & 1;
          sh.eu[wb][pslot][w][0][lane] = U[sl][i][o];
          if constexpr (VAR) sh.ek[wb][pslot][w][0][lane] = K[sl][i][o];
        }
        {
          constexpr int i = RPW - 1;
          constexpr int o = (B0 + i + P) & 1;
          sh.eu[wb][pslot][w][1][lane] = U[sl][i][o];
          if constexpr (VAR) sh.ek[wb][pslot][w][1][lane] = K[sl][i][o];
        }
      }

      if constexpr (RES == 1) restrict_step(IC<P>{});
      if constexpr (REF) refine_step(IC<P>{});
      // the last step stores its own finished plane zl - H
      if (zl + 1 == zend) store(zl - H, IC<imod(P - H, Q)>{});
      ++zl;
      return zl < zstop;
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
    if constexpr (REF) {
      // per-workgroup sum of r^2: lanes, then waves in order
#pragma unroll
      for (int o2 = 32; o2 >= 1; o2 >>= 1) sumsq += __shfl_xor(sumsq, o2, 64);
      if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = sumsq;
      __syncthreads();
      if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int v = 0; v < W; ++v) tot += sh.red[v];
        ra.partial[blockIdx.x] = tot;
      }
    }
  }
};

template <typename T, bool VAR, int S, int W, int RPW, int PD, int IN, int RES, int LW>
__global__ void __launch_bounds__(64 * W)
    k_rbgs_tiled(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ f,
                 const T* __restrict__ k, const T* __restrict__ ec, int nc, int n, T h2,
                 T ih2, T* __restrict__ fc, int tiles_x, int tiles_y, int zlen, RefineArgs ra)
{
  using C = Tiled<T, VAR, S, W, RPW, PD, RES, LW>;
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
  // parity of (x of column 0) + (y of row 0) + z0 - 1 + ZR; RPW is even, so it is the
  // same for every row group's first row
  const int b0 = ((ox - C::H) + (oy - C::H) + z0 - 1 + C::ZR) & 1;
  if (b0) C::template run<1, IN>(uin, uout, f, k, ec, nc, n, h2, ox, oy, z0, z1, ih2, fc, ra, sh);
  else C::template run<0, IN>(uin, uout, f, k, ec, nc, n, h2, ox, oy, z0, z1, ih2, fc, ra, sh);
}

struct LaunchShape {
  int tiles_x, tiles_y, nchunks, zlen, blocks;
  long long cost;  // rounds of resident workgroups x planes per workgroup
};

// Workgroups of this kernel that fit on the device at once (CUs x resident per CU), queried
// once per device, kernel and block size (every instantiation of k_rbgs_tiled has the same
// function type, so the kernel's address is part of the key).
template <typename Kernel>
int resident_capacity(Kernel kernel, int block)
{
  struct Entry {
    const void* k;
    int block, dev, cap;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  const void* key = reinterpret_cast<const void*>(kernel);
  {
    std::lock_guard<std::mutex> g(mu);
    for (const Entry& e : cache)
      if (e.k == key && e.block == block && e.dev == dev) return e.cap;
  }
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  std::lock_guard<std::mutex> g(mu);
  cache.push_back({key, block, dev, cus * per_cu});
  return cus * per_cu;
}

// Tiles cover the interior in x and y; z is cut into chunks.  Each chunk costs its length
// plus 2(H + ZR) warm-up planes, and workgroups run in rounds of `capacity`; the chunk count that
// minimises (rounds x planes per workgroup) -- the critical path -- is chosen.  Chunks may be
// shorter than their warm-up: on a small level the launch is bound by the latency of its
// plane steps, and more, shorter chunks cut the steps per workgroup (at 129^3 the FP32
// post-smoothing pass takes 12 steps on 256 workgroups instead of 17 on 120; FP32-refined
// solve at 513^3: 19.93 ms against 20.13 with chunks of at least 2H planes).
template <typename C>
LaunchShape shape_for(int n, int capacity)
{
  LaunchShape L;
  const int m = n - 2;
  L.tiles_x = (m + C::TXO - 1) / C::TXO;
  L.tiles_y = (m + C::TYO - 1) / C::TYO;
  const int per = L.tiles_x * L.tiles_y;
  const int maxchunks = m;
  long long best = -1;
  L.zlen = m;
  for (int c = 1; c <= maxchunks; ++c) {
    const int zlen = (m + c - 1) / c;
    const int chunks = (m + zlen - 1) / zlen;
    const long long blocks = (long long)per * chunks;
    const long long rounds = (blocks + capacity - 1) / capacity;
    const long long cost = rounds * (zlen + 2 * (C::H + C::ZR));
    if (best < 0 || cost < best) {
      best = cost;
      L.zlen = zlen;
    }
  }
  L.nchunks = (m + L.zlen - 1) / L.zlen;
  L.blocks = per * L.nchunks;
  L.cost = best;
  return L;
}

// Tile shape (waves x rows per wave), prefetch depth and whether the 64-column layout is
// compiled, per pass, from timing sweeps on MI355X at 513^3 (the FP32 passes of the
// refinement cycle were timed inside the whole solve).
#ifndef MG_SMOOTH_W
#define MG_SMOOTH_W 8
#endif
#ifndef MG_SMOOTH_RPW
#define MG_SMOOTH_RPW 4
#endif
#ifndef MG_SMOOTH32_PROLONG_W
#define MG_SMOOTH32_PROLONG_W 8
#endif
#ifndef MG_SMOOTH32_PROLONG_PD
#define MG_SMOOTH32_PROLONG_PD 1
#endif
#ifndef MG_SMOOTH32_ZERO_PD
#define MG_SMOOTH32_ZERO_PD 2
#endif
#ifndef MG_SMOOTH64_ZERO_PD
#define MG_SMOOTH64_ZERO_PD 2
#endif
#ifndef MG_SMOOTH32_ZERO_W
#define MG_SMOOTH32_ZERO_W 8
#endif
#ifndef MG_SMOOTH32_READ_W
#define MG_SMOOTH32_READ_W 12
#endif
#ifndef MG_SMOOTH32_READ_PD
#define MG_SMOOTH32_READ_PD 2
#endif
#ifndef MG_SMOOTH32_RES_W
#define MG_SMOOTH32_RES_W 8
#endif
#ifndef MG_SMOOTH32_RES_RPW
#define MG_SMOOTH32_RES_RPW 4
#endif
#ifndef MG_SMOOTH32_PROLONG_RPW
#define MG_SMOOTH32_PROLONG_RPW 6
#endif
#ifndef MG_SMOOTH32_READ_RPW
#define MG_SMOOTH32_READ_RPW 4
#endif
#ifndef MG_SMOOTH32_RES_PD
#define MG_SMOOTH32_RES_PD 1
#endif
#ifndef MG_SMOOTH32_RES_NARROW
#define MG_SMOOTH32_RES_NARROW 1
#endif
#ifndef MG_SMOOTH32_PROLONG_NARROW
#define MG_SMOOTH32_PROLONG_NARROW 1
#endif
// The FP64 post-smoothing pass with the prolongation holds the coarse correction's planes
// as well: 10 waves of 2 rows (64 x 40-node tiles in the 64-column layout) keep it within
// 152 VGPRs; 8 x 4 spills.  Timed inside the FP64 solve at 513^3 (29.0 ms against 29.3 for
// 12 x 2, 29.8 for 8 x 2 with a second prefetch buffer and 32.3 with the separate pass).
// The FP64 pre-smoothing pass with the residual restriction holds two more planes: 8 waves
// of 2 rows (64 x 32-node tiles) fit in 200-208 VGPRs; 10 x 2 and 8 x 4 spill, 12 x 2
// exceeds the LDS.  FP64 solve at 513^3: 27.3 ms against 29.0 with the separate
// restriction pass.
// The FP64 variable-coefficient pass holds k beside u and f: with 2 sweeps per pass, 8
// waves of 2 rows (both layouts) fit in 192-214 VGPRs; 8 x 4 spills.  Workload 4's FP64
// solve at 257^3: 16.5 ms, against 21.7 ms with one sweep per pass.
#ifndef MG_SMOOTH64_VAR_W
#define MG_SMOOTH64_VAR_W 8
#endif
#ifndef MG_SMOOTH64_VAR_RPW
#define MG_SMOOTH64_VAR_RPW 2
#endif
#ifndef MG_SMOOTH64_VAR_NARROW
#define MG_SMOOTH64_VAR_NARROW 1
#endif
#ifndef MG_SMOOTH64_RES_W
#define MG_SMOOTH64_RES_W 8
#endif
#ifndef MG_SMOOTH64_RES_RPW
#define MG_SMOOTH64_RES_RPW 2
#endif
#ifndef MG_SMOOTH64_PROLONG_W
#define MG_SMOOTH64_PROLONG_W 10
#endif
#ifndef MG_SMOOTH64_PROLONG_RPW
#define MG_SMOOTH64_PROLONG_RPW 2
#endif
// The FP32 post-smoothing pass with the refinement step also holds three corrected FP64
// planes and f of a step: 12 waves of 2 rows (64 x 48-node tiles in the 64-column layout)
// fit in 167 VGPRs, 3 waves per SIMD.  FP32-refined solve at 513^3: 20.17 ms against 20.32
// for 8 x 4 in the 128-column layout (249 VGPRs; the 64-column layout spills) and 20.40
// with the separate passes.
#ifndef MG_SMOOTH32_REF_W
#define MG_SMOOTH32_REF_W 12
#endif
#ifndef MG_SMOOTH32_REF_RPW
#define MG_SMOOTH32_REF_RPW 2
#endif
#ifndef MG_SMOOTH32_REF_NARROW
#define MG_SMOOTH32_REF_NARROW 1
#endif
template <typename T, bool VAR, int S, int IN, int RES>
struct Shape {
  static constexpr bool f32 = sizeof(T) == 4, plain = !VAR && S == 2;
  static constexpr int W = RES == 2           ? MG_SMOOTH32_REF_W
                           : RES              ? (f32 ? MG_SMOOTH32_RES_W : MG_SMOOTH64_RES_W)
                           : (!f32 && VAR && S == 2) ? MG_SMOOTH64_VAR_W
                           : (!f32 && plain && IN == kInProlong) ? MG_SMOOTH64_PROLONG_W
                           : !(f32 && plain)   ? MG_SMOOTH_W
                           : IN == kInProlong ? MG_SMOOTH32_PROLONG_W
                           : IN == kInZero    ? MG_SMOOTH32_ZERO_W
                                              : MG_SMOOTH32_READ_W;
  static constexpr int RPW = RES == 2           ? MG_SMOOTH32_REF_RPW
                             : RES              ? (f32 ? MG_SMOOTH32_RES_RPW : MG_SMOOTH64_RES_RPW)
                             : (!f32 && VAR && S == 2) ? MG_SMOOTH64_VAR_RPW
                             : (!f32 && plain && IN == kInProlong) ? MG_SMOOTH64_PROLONG_RPW
                             : !(f32 && plain)   ? MG_SMOOTH_RPW
                             : IN == kInProlong ? MG_SMOOTH32_PROLONG_RPW
                             : IN == kInRead    ? MG_SMOOTH32_READ_RPW
                                                : MG_SMOOTH_RPW;
  static constexpr int PD = RES == 2 ? 1
                            : RES ? (f32 ? MG_SMOOTH32_RES_PD : 1)
                            : !plain ? 1
                            : IN == kInProlong ? (f32 ? MG_SMOOTH32_PROLONG_PD : 1)
                            : IN == kInZero    ? (f32 ? MG_SMOOTH32_ZERO_PD : MG_SMOOTH64_ZERO_PD)
                                               : (f32 ? MG_SMOOTH32_READ_PD : 1);
  // whether the 64-column layout (LW = 32) is compiled for this pass: its per-lane row
  // offsets cost ~20-40 VGPRs, which the FP64 variable-coefficient pass does not have to
  // spare (it would spill; so would the FP32 restriction and prolongation passes with a
  // second prefetch buffer or 6 rows per wave in the restriction)
  static constexpr bool NARROW = RES == 2 ? MG_SMOOTH32_REF_NARROW
                                 : RES ? MG_SMOOTH32_RES_NARROW
                                 : IN == kInProlong ? MG_SMOOTH32_PROLONG_NARROW
                                 : (!f32 && VAR && S == 2) ? MG_SMOOTH64_VAR_NARROW
                                                    : !(VAR && !f32);
};

// The two tile layouts of a pass (128 columns x W*RPW rows, or 64 columns x 2*W*RPW rows)
// hold the same nodes per workgroup; the one whose launch shape costs fewer planes per
// workgroup on the critical path at this grid size is launched (the 128-column layout on
// a tie).  Both give bitwise the same result.
template <typename T, bool VAR, int S, int IN, int RES = 0>
int launch_in(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin, T* uout,
              const T* ec, T* fc = nullptr, RefineArgs ra = {})
{
  using Sh = Shape<T, VAR, S, IN, RES>;
  constexpr int W = Sh::W, RPW = Sh::RPW, PD = Sh::PD;
  const T h2 = (T)(h * h);
  const int nc = (n - 1) / 2 + 1;
  const T ih2 = (T)(1.0 / (h * h));
  auto k64 = k_rbgs_tiled<T, VAR, S, W, RPW, PD, IN, RES, 64>;
  const LaunchShape L64 = shape_for<Tiled<T, VAR, S, W, RPW, PD, RES, 64>>(n, resident_capacity(k64, 64 * W));
  if constexpr (Sh::NARROW) {
    auto k32 = k_rbgs_tiled<T, VAR, S, W, RPW, PD, IN, RES, 32>;
    const LaunchShape L32 = shape_for<Tiled<T, VAR, S, W, RPW, PD, RES, 32>>(n, resident_capacity(k32, 64 * W));
    if (L32.cost < L64.cost) {
      if (RES == 2 && L32.blocks > kStreamPartials) return -1;  // one partial sum per workgroup
      k32<<<L32.blocks, 64 * W, 0, s>>>(uin, uout, f, k, ec, nc, n, h2, ih2, fc, L32.tiles_x,
                                        L32.tiles_y, L32.zlen, ra);
      return L32.blocks;
    }
  }
  if (RES == 2 && L64.blocks > kStreamPartials) return -1;
  k64<<<L64.blocks, 64 * W, 0, s>>>(uin, uout, f, k, ec, nc, n, h2, ih2, fc, L64.tiles_x,
                                    L64.tiles_y, L64.zlen, ra);
  return L64.blocks;
}

template <typename T, bool VAR, int S>
void launch_cfg(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin, T* uout,
                bool zero_in, const T* ec)
{
  if (ec) {
    // FP32 passes and 2-sweep FP64 passes fuse the prolongation (rbgs_tiled_fuses_prolong);
    // a one-sweep FP64 pass, which the host does not ask for, adds it first
    if constexpr (sizeof(T) == 4 || S == 2) {
      launch_in<T, VAR, S, kInProlong>(s, n, h, k, f, uin, uout, ec);
    } else {
      prolong_add<T>(s, 3, (n - 1) / 2 + 1, ec, const_cast<T*>(uin));
      launch_in<T, VAR, S, kInRead>(s, n, h, k, f, uin, uout, ec);
    }
  } else if (zero_in) launch_in<T, VAR, S, kInZero>(s, n, h, k, f, uin, uout, ec);
  else launch_in<T, VAR, S, kInRead>(s, n, h, k, f, uin, uout, ec);
}

}  // namespace

// The per-colour kernel is faster up to 65^3 (a 3D level that small streams too few
// planes per workgroup to hide the pipeline's start-up); from 129^3 on, the two launches
// per level and cycle of the fused kernels beat the ten of the per-colour path.
#ifndef MG_TILED_MIN_N
#define MG_TILED_MIN_N 65
#endif
bool rbgs_tiled_supported(int dim, int n) { return dim == 3 && n > MG_TILED_MIN_N; }

bool rbgs_tiled_fuses_prolong(size_t value_bytes, bool var)
{
  // every 2-sweep pass takes the coarse-grid correction (the FP64 variable-coefficient one
  // on its 8 x 2-row tiles: 220-234 VGPRs)
  (void)value_bytes;
  (void)var;
  return true;
}

int rbgs_tiled_max_sweeps(bool var, size_t value_bytes)
{
  // every pass fuses two sweeps (the FP64 variable-coefficient pass on 8 x 2-row tiles)
  (void)var;
  (void)value_bytes;
  return 2;
}

bool rbgs_tiled_fuses_restrict(size_t value_bytes, bool var)
{
  return !var;
}

template <typename T>
void rbgs_tiled(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin, T* uout,
                int sweeps, bool zero_in, const T* ec, T* fc)
{
  if (fc) {
    // two sweeps with the residual restricted into fc; the host asks for it only where
    // rbgs_tiled_fuses_restrict holds
    if (!k && sweeps == 2 && !ec) {
      if (zero_in) launch_in<T, false, 2, kInZero, 1>(s, n, h, k, f, uin, uout, ec, fc);
      else launch_in<T, false, 2, kInRead, 1>(s, n, h, k, f, uin, uout, ec, fc);
      return;
    }
  }
  if (sweeps == 2) {
    if (k) {
      launch_cfg<T, true, 2>(s, n, h, k, f, uin, uout, zero_in, ec);
    } else {
      launch_cfg<T, false, 2>(s, n, h, k, f, uin, uout, zero_in, ec);
    }
  } else {
    if (k) launch_cfg<T, true, 1>(s, n, h, k, f, uin, uout, zero_in, ec);
    else launch_cfg<T, false, 1>(s, n, h, k, f, uin, uout, zero_in, ec);
  }
}

namespace {
// The power of two nearest in log2 to the root mean square of a residual whose squares sum
// to norm2 over `interior` nodes (1 if that is 0 or not finite).  The FP32 right-hand side
// of a correction cycle is the residual divided by it: any power of two changes no float
// result and keeps the values away from the float range limits.
__device__ double ir_scale_of(double norm2, double interior)
{
  const double rms = sqrt(norm2 / interior);
  if (!(rms > 0.0) || !__builtin_isfinite(rms)) return 1.0;
  int e = 0;
  const double m = frexp(rms, &e);  // rms = m 2^e, 0.5 <= m < 1
  return ldexp(1.0, m >= 0.70710678118654752 ? e : e - 1);
}

// norm2[0] = fixed-order sum of the per-workgroup partials, scale[0] = its scale
__global__ void __launch_bounds__(256)
    k_sum_scale(const double* __restrict__ partial, int count, double* __restrict__ norm2,
                double interior, double* __restrict__ scale)
{
  __shared__ double part[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = (part[0] + part[1]) + (part[2] + part[3]);
    norm2[0] = tot;
    scale[0] = ir_scale_of(tot, interior);
  }
}

__global__ void k_scale_init(const double* __restrict__ norm2, double s0, double interior,
                             double* __restrict__ ss)
{
  if (threadIdx.x == 0) {
    ss[0] = s0;
    ss[1] = ir_scale_of(norm2[0], interior);
  }
}
}  // namespace

bool rbgs_tiled_refine(hipStream_t s, int n, double h, const float* rhs, const float* ein,
                       const float* ec, const double* f, const double* u, double* uout,
                       float* r32, const double* scale_e, const double* scale_r,
                       double* partial, double* norm2, double* scale_next)
{
  RefineArgs ra{u, uout, f, r32, scale_e, scale_r, 1.0 / (h * h), partial};
  const int blocks = launch_in<float, false, 2, kInProlong, 2>(s, n, h, nullptr, rhs, ein,
                                                               nullptr, ec, nullptr, ra);
  if (blocks < 0) return false;
  const double interior = (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  k_sum_scale<<<1, 256, 0, s>>>(partial, blocks, norm2, interior, scale_next);
  return true;
}

bool rbgs_tiled_refine_fits(int n)
{
  // the launch shape launch_in picks for the fused pass
  using Sh = Shape<float, false, 2, kInProlong, 2>;
  constexpr int W = Sh::W, RPW = Sh::RPW, PD = Sh::PD;
  auto k64 = k_rbgs_tiled<float, false, 2, W, RPW, PD, kInProlong, 2, 64>;
  LaunchShape L = shape_for<Tiled<float, false, 2, W, RPW, PD, 2, 64>>(n, resident_capacity(k64, 64 * W));
  if constexpr (Sh::NARROW) {
    auto k32 = k_rbgs_tiled<float, false, 2, W, RPW, PD, kInProlong, 2, 32>;
    const LaunchShape L32 =
        shape_for<Tiled<float, false, 2, W, RPW, PD, 2, 32>>(n, resident_capacity(k32, 64 * W));
    if (L32.cost < L.cost) L = L32;
  }
  return L.blocks <= kStreamPartials;
}

void ir_scales_init(hipStream_t s, int n, const double* norm2, double scale0, double* ss)
{
  const double interior = (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  k_scale_init<<<1, 64, 0, s>>>(norm2, scale0, interior, ss);
}

template void rbgs_tiled<double>(hipStream_t, int, double, const double*, const double*,
                                 const double*, double*, int, bool, const double*, double*);
template void rbgs_tiled<float>(hipStream_t, int, double, const float*, const float*,
                                const float*, float*, int, bool, const float*, float*);

}  // namespace mgk
