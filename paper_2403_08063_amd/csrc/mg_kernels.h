// Internal launch interface between the C-ABI host code (mg_api.hip) and the HIP kernels.
// Every launcher enqueues on the given stream and returns without synchronising.
// Arrays are device pointers to n^dim node values in C order [z][y][x], boundary included;
// k == nullptr selects the constant-coefficient operator.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace mgk {

constexpr int kNormBlocks = 1024;  // fixed grid of the norm kernels: the reduction order
                                   // depends on nothing but the grid size
constexpr int kStreamPartials = 16384;  // per-workgroup partial sums of the streaming passes

// One red-black half-sweep of one colour, in place (every level, 2D and 3D).
template <typename T>
void rbgs_colour(hipStream_t s, int dim, int n, double h, const T* k, const T* f, T* u,
                 int colour);

// The first colour-0 half-sweep of a smoothing, in place: ec == nullptr: from a zero guess
// (colour-0 nodes get the Gauss-Seidel value of the zero iterate, colour-1 nodes are set to
// 0; boundary nodes must already be 0); ec != nullptr: of u + P ec (ec on the next coarser
// level), the correction read on the fly and not stored -- valid as the first half-sweep of
// a full sweep, whose colour-1 half-sweep overwrites every colour-1 node.  Bitwise equal to
// the fill or prolong_add followed by rbgs_colour(.., 0).
template <typename T>
void rbgs_first(hipStream_t s, int dim, int n, double h, const T* k, const T* f, T* u,
                const T* ec);

// `sweeps` (1 or 2) full red-black sweeps fused in one pass over a 3D level, out of place:
// uout = RBGS^sweeps(uin).  zero_in: treat uin as identically 0 (not read).  ec != nullptr:
// the input is uin + P ec (coarse-grid correction with (n-1)/2+1 nodes per side, added on
// interior nodes as prolong_add does).  fc != nullptr (2 sweeps, constant coefficient:
// rbgs_tiled_fuses_restrict): the pass also writes the full-weighting
// restriction of the residual f - A uout to the interior of fc, the next coarser level's
// right-hand side, with the arithmetic of restrict_residual_tiled.  The boundary of uout
// (and of fc) is not written.
template <typename T>
void rbgs_tiled(hipStream_t s, int n, double h, const T* k, const T* f, const T* uin,
                T* uout, int sweeps, bool zero_in, const T* ec = nullptr, T* fc = nullptr);
// Whether the fused pass serves this level (3D, large enough for its tiles), and how many
// sweeps one pass may fuse.
bool rbgs_tiled_supported(int dim, int n);
int rbgs_tiled_max_sweeps(bool var, size_t value_bytes);
bool rbgs_tiled_fuses_prolong(size_t value_bytes, bool var);
bool rbgs_tiled_fuses_restrict(size_t value_bytes, bool var);
// The last FP32 post-smoothing of a correction cycle (constant coefficient, two sweeps, the
// coarse-grid correction ec taken in, right-hand side rhs, input ein) fused with the
// refinement step that follows it: with e the smoothed correction (not stored),
// uout = u + s_e e on interior nodes (boundary of uout not written), r = f - A uout,
// r32 = (float)(r / s_r), norm2[0] = sum of r^2 over interior nodes, scale_next[0] = the
// scale of the next right-hand side (the power of two nearest in log2 to the residual's
// root mean square).  s_e = scale_e[0], s_r = scale_r[0] are device scalars, read by the
// kernel.  The arithmetic of uout and r32 is that of rbgs_tiled followed by ir_pass_tiled;
// the sum runs in another order.  partial: kStreamPartials doubles.  r32 and rhs, uout and
// u must not overlap.  Returns false, launching nothing, if the grid needs more than
// kStreamPartials workgroups.
bool rbgs_tiled_refine(hipStream_t s, int n, double h, const float* rhs, const float* ein,
                       const float* ec, const double* f, const double* u, double* uout,
                       float* r32, const double* scale_e, const double* scale_r,
                       double* partial, double* norm2, double* scale_next);
// Whether rbgs_tiled_refine's launch at n nodes a side fits its partial sums.
bool rbgs_tiled_refine_fits(int n);
// ss[0] = scale0, ss[1] = the scale (as rbgs_tiled_refine's scale_next) of the residual whose
// squares sum to norm2[0]: the scales of the first two right-hand sides of a fused solve.
void ir_scales_init(hipStream_t s, int n, const double* norm2, double scale0, double* ss);

// r = f - A u (interior), 0 on the boundary.
template <typename T>
void residual(hipStream_t s, int dim, int n, double h, const T* k, const T* f, const T* u,
              T* r);

// fc = FW(f - A u) on coarse interior nodes (coarse boundary not written).
template <typename T>
void restrict_residual(hipStream_t s, int dim, int nf, double h, const T* k, const T* f,
                       const T* u, T* fc);

// Streaming versions for large 3D levels (mg_resid_tiled.hip): same results up to the
// summation order.  restrict_residual_tiled writes the coarse interior only.
template <typename T>
void restrict_residual_tiled(hipStream_t s, int nf, double h, const T* k, const T* f,
                             const T* u, T* fc);
// mode 0: ||f - A u||^2; mode 1: interior of u read as 0.  partial: kStreamPartials doubles.
void resid_norm2_tiled(hipStream_t s, int n, double h, const double* k, const double* f,
                       const double* u, int mode, double* partial, double* out);
// Both in one pass (constant coefficient): out[0] as mode 0, out[1] as mode 1, each summed
// in the order of its own pass.  partial, partial_b: kStreamPartials doubles each.
void resid_norm2_both_tiled(hipStream_t s, int n, double h, const double* f, const double* u,
                            double* partial, double* partial_b, double* out);
// Refinement pass: uout = u + scale * e on interior nodes (boundary of uout not written),
// r = f - A uout, r32 = (float)(r * inv_scale), out[0] = sum of r^2 (interior).
// partial_b (constant coefficient, e == nullptr: the first pass of a solve): also out[1] =
// the sum of squares of the full right-hand side f - A u_B (interior of u read as 0), equal
// to resid_norm2_tiled's mode 1 (same tiles and summation order); kStreamPartials doubles.
void ir_pass_tiled(hipStream_t s, int n, double h, const double* k, const double* f,
                   const double* u, const float* e, double scale, double inv_scale, double* uout,
                   float* r32, double* partial, double* out, double* partial_b = nullptr);

// u += P ec on fine interior nodes (nc = coarse nodes per side).
template <typename T>
void prolong_add(hipStream_t s, int dim, int nc, const T* ec, T* u);

// Coarsest level: assemble the interior operator, Cholesky-factor it and form its inverse
// (one workgroup).  work: m*m doubles; ainv: m*m doubles; flag: set to 1 if the matrix is
// not positive definite.
void coarsest_factor(hipStream_t s, int dim, int n, double h, const double* k, double* work,
                     double* ainv, int* flag);
// Interior of u = ainv * (interior of f), computed in double; boundary untouched.
template <typename T>
void coarsest_solve(hipStream_t s, int dim, int n, const double* ainv, const T* f, T* u);

// partial[0..kNormBlocks) = per-block sums of squares of f - A u over interior nodes
// (mode 0), or of f - A u_B with u_B = u with zero interior (mode 1: the full right-hand
// side).  Then out[0] = fixed-order sum of the partials.
void resid_norm2(hipStream_t s, int dim, int n, double h, const double* k, const double* f,
                 const double* u, int mode, double* partial, double* out);

// Iterative refinement: r32 = (float)((f - A u) * inv_scale) on interior nodes, plus the
// norm as in resid_norm2 (mode 0) into out[0].
void ir_residual(hipStream_t s, int dim, int n, double h, const double* k, const double* f,
                 const double* u, double inv_scale, float* r32, double* partial, double* out);
// u += scale * (double)e32 on interior nodes.
void ir_update(hipStream_t s, int dim, int n, double scale, const float* e32, double* u);

// Coefficient hierarchy: kc = coarse coefficient of k (exp of full-weighted log k in the
// interior, injection on the boundary).
void coarsen_k(hipStream_t s, int dim, int nf, const double* k, double* kc);
void cast_to_f32(hipStream_t s, size_t count, const double* src, float* dst);

// Gradient pass: dk (nullable), df (nullable) from u and lambda on all nodes.
void grad(hipStream_t s, int dim, int n, const double* u, const double* lam, double* dk,
          double* df);

// Coarse tail (mg_tail.hip): one workgroup runs the whole V-cycle on levels
// lv[0] .. lv[nlev-1] (the last one the coarsest, solved with ainv) from a zero guess on
// every level; lv[0].f is the right-hand side, lv[0].u receives the result.
constexpr int kTailMaxNodes = 4096;  // interior nodes of the finest tail level
constexpr int kMaxTail = 16;
template <typename T>
struct TailLevel {
  T* u;
  T* f;
  const T* k;  // nullptr: constant coefficient
  int n;
  T h2, ih2;   // h^2 and 1/h^2 of the level, as the per-level kernels round them
};
template <typename T>
struct TailArgs {
  TailLevel<T> lv[kMaxTail];
  int nlev, nu1, nu2;
  const double* ainv;
};
bool tail_fits(int dim, int n);
template <typename T>
void tail_cycle(hipStream_t s, int dim, const TailArgs<T>& a);

template <typename T>
void fill(hipStream_t s, size_t count, T value, T* p);
template <typename T>
void copy(hipStream_t s, size_t count, const T* src, T* dst);
// Copies the boundary nodes of src into dst.
void copy_boundary(hipStream_t s, int dim, int n, const double* src, double* dst);
// Sets the boundary nodes of p to 0.
void zero_boundary(hipStream_t s, int dim, int n, double* p);

// ---- cell-centred finite volumes (N^3 cells, arrays of (N+2)^3 values with a ghost layer
// holding the Dirichlet value at the adjacent face centre; a ghost neighbour enters the
// 7-point operator as 2 g - u_i).
// Exact-partition streaming passes for N >= 128 (mg_resid_tiled.hip):
bool fv_tiled_supported(int N);
// one damped Jacobi sweep, uout = u + omega h^2/6 (f - A u) on the cells (ghosts untouched)
// zero_u: u is identically 0, ghost layer included (not read)
void fv_jacobi_tiled(hipStream_t s, int N, double h, double omega, const double* f,
                     const double* u, double* uout, double* partial, bool zero_u = false);
// the first post-smoothing sweep of a V-cycle: uout = Jacobi(u + P ec), with ec the coarse
// correction ((N/2 + 2)^3 values, ghost layer not read) interpolated as the stand-alone
// prolongation does; u itself is not modified
void fv_jacobi_prolong_tiled(hipStream_t s, int N, double h, double omega, const double* f,
                             const double* u, const double* ec, double* uout, double* partial);
// fc = mean of the 8 children's residuals f - A u on the coarse cells (N/2 per side);
// fc's ghost layer is not written
void fv_restrict_tiled(hipStream_t s, int N, double h, const double* f, const double* u,
                       double* fc, double* partial);
// out = sum over cells of (f - A u)^2 (partial: kStreamPartials doubles)
void fv_norm2_tiled(hipStream_t s, int N, double h, const double* f, const double* u,
                    double* partial, double* out);

}  // namespace mgk
