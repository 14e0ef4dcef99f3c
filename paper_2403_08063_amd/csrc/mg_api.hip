// C-ABI of libmg.so: argument validation, workspace layout, and the host drivers of the
// V-cycle, the FP32-inner / FP64-outer iterative refinement, the adjoint solve and the
// gradient pass.  All arithmetic runs in the kernels of mg_kernels.hip and
// mg_smooth_tiled.hip; the host only sequences launches and reads one norm per cycle.
//
// Paper: Angersbach, Kuckuk, Koestler, "Towards Code Generation for Octree-Based Multigrid
// Solvers": V-cycle Sect. 1 and 5, residual-norm termination Sect. 5, per-level scalars
// (level size, mesh width) passed to the kernels as arguments as in Sect. 4.3.
#include "../../include/mg.h"
#include "mg_kernels.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>

namespace {

constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 1024;  // interior unknowns of the coarsest level
constexpr size_t kAlign = 256;

thread_local char g_err[512] = "no error";

struct Level {
  int n = 0;
  size_t N = 0;  // nodes
  double h = 0;
  double *u = nullptr, *f = nullptr, *t = nullptr, *k = nullptr;
  float *u32 = nullptr, *f32 = nullptr, *t32 = nullptr, *k32 = nullptr;
};

}  // namespace

struct mg_ctx {
  mg_grid g{};
  hipStream_t s = nullptr;
  Level lv[kMaxLevels];
  int m = 0;  // coarsest interior unknowns
  double* chol = nullptr;
  double* ainv = nullptr;
  int* flag = nullptr;
  double* partial = nullptr;
  double* partial_b = nullptr;  // second partial sums (right-hand-side norm of the first pass)
  double* scal = nullptr;  // device scalars: [0] norm2, [1] rhs norm2, [4..5] fused-solve scales
  double last_bn = 0.0;    // right-hand-side norm of the previous solve (0: none)
  bool coeffs = false;
  int fuse = MG_FUSE_ALL;  // kernel-fusion flags (mg_set_fusion)
  int tail_first = -1;  // first level handled by the one-launch coarse tail (-1: none)
  // norm read-back without draining the stream: a pinned host word and an event after the
  // copy (nullptr: synchronous reads only)
  double* hnorm = nullptr;
  hipEvent_t ev = nullptr;
  char err[512] = "no error";
  ~mg_ctx()
  {
    if (ev) (void)hipEventDestroy(ev);
    if (hnorm) (void)hipHostFree(hnorm);
  }
};

namespace {

mg_status fail(mg_ctx* c, mg_status st, const char* fmt, ...)
{
  char* buf = c ? c->err : g_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
  return st;
}

size_t nodes(int dim, int n) { return dim == 3 ? (size_t)n * n * n : (size_t)n * n; }

mg_status validate(const mg_grid* g, mg_ctx* c)
{
  if (!g) return fail(c, MG_EINVAL, "grid description is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(c, MG_EINVAL, "dim must be 2 or 3 (got %d)", g->dim);
  if (g->levels < 2 || g->levels > kMaxLevels)
    return fail(c, MG_EINVAL, "levels must be in [2, %d] (got %d)", kMaxLevels, g->levels);
  if (g->n < 5) return fail(c, MG_EINVAL, "n must be >= 5 (got %d)", g->n);
  if ((g->dim == 3 && g->n > 4097) || (g->dim == 2 && g->n > 65537))
    return fail(c, MG_EINVAL, "n = %d too large", g->n);
  const int step = 1 << (g->levels - 1);
  if ((g->n - 1) % step != 0)
    return fail(c, MG_EINVAL, "n - 1 = %d is not divisible by 2^(levels-1) = %d", g->n - 1, step);
  const int nc = (g->n - 1) / step + 1;
  if (nc < 3) return fail(c, MG_EINVAL, "coarsest level has %d nodes per side (< 3)", nc);
  const long long m = g->dim == 3 ? (long long)(nc - 2) * (nc - 2) * (nc - 2)
                                  : (long long)(nc - 2) * (nc - 2);
  if (m > kMaxCoarse)
    return fail(c, MG_EINVAL, "coarsest level has %lld interior nodes (> %d): use more levels",
                m, kMaxCoarse);
  if (g->nu1 < 0 || g->nu2 < 0 || g->nu1 + g->nu2 < 1)
    return fail(c, MG_EINVAL, "nu1, nu2 must be >= 0 with nu1 + nu2 >= 1");
  if (g->max_cycles < 1) return fail(c, MG_EINVAL, "max_cycles must be >= 1");
  if (g->precision != MG_F64 && g->precision != MG_F32_IR)
    return fail(c, MG_EINVAL, "precision must be MG_F64 or MG_F32_IR");
  if (g->variable != 0 && g->variable != 1) return fail(c, MG_EINVAL, "variable must be 0 or 1");
  return MG_OK;
}

// Workspace layout, shared by mg_workspace_bytes (p == nullptr: count only) and mg_setup.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count)
  {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

void layout(const mg_grid* g, Carver& cv, mg_ctx* c)
{
  Level tmp[kMaxLevels];
  Level* lv = c ? c->lv : tmp;
  const bool ir = g->precision == MG_F32_IR;
  for (int l = 0; l < g->levels; ++l) {
    Level& L = lv[l];
    L.n = (g->n - 1) / (1 << l) + 1;
    L.N = nodes(g->dim, L.n);
    L.h = (double)(1 << l) / (double)(g->n - 1);
    L.t = cv.take<double>(L.N);
    if (l > 0) {
      L.u = cv.take<double>(L.N);
      L.f = cv.take<double>(L.N);
    }
    if (g->variable) L.k = cv.take<double>(L.N);
    if (ir) {
      L.u32 = cv.take<float>(L.N);
      L.f32 = cv.take<float>(L.N);
      L.t32 = cv.take<float>(L.N);
      if (g->variable) L.k32 = cv.take<float>(L.N);
    }
  }
  const int nc = lv[g->levels - 1].n;
  const int m = g->dim == 3 ? (nc - 2) * (nc - 2) * (nc - 2) : (nc - 2) * (nc - 2);
  double* chol = cv.take<double>((size_t)m * m);
  double* ainv = cv.take<double>((size_t)m * m);
  double* partial = cv.take<double>(mgk::kStreamPartials);
  double* partial_b = cv.take<double>(mgk::kStreamPartials);
  double* scal = cv.take<double>(8);
  int* flag = cv.take<int>(4);
  if (c) {
    c->m = m;
    c->chol = chol;
    c->ainv = ainv;
    c->partial = partial;
    c->partial_b = partial_b;
    c->scal = scal;
    c->flag = flag;
  }
}

mg_status hip_check(mg_ctx* c, hipError_t e, const char* what)
{
  if (e == hipSuccess) return MG_OK;
  return fail(c, MG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

mg_status launch_check(mg_ctx* c, const char* what)
{
  return hip_check(c, hipGetLastError(), what);
}

// ---------------------------------------------------------------- level views
template <typename T>
struct View {
  T *u, *f, *t;
  const T* k;
};

template <typename T>
View<T> view(mg_ctx* c, int l);
template <>
View<double> view<double>(mg_ctx* c, int l)
{
  Level& L = c->lv[l];
  return {L.u, L.f, L.t, L.k};
}
template <>
View<float> view<float>(mg_ctx* c, int l)
{
  Level& L = c->lv[l];
  return {L.u32, L.f32, L.t32, L.k32};
}

bool use_tiled(const mg_ctx* c, int l)
{
  return (c->fuse & MG_FUSE_BLOCKED) && mgk::rbgs_tiled_supported(c->g.dim, c->lv[l].n);
}

// `sweeps` red-black sweeps on level l.  u holds the iterate, t is the level's second
// buffer (same boundary values as u).  Returns the buffer that holds the result: the
// fused kernel works out of place and alternates between u and t.  zero_guess: u is known
// to be 0 (a coarse-grid correction) and is not read.
template <typename T>
T* smooth(mg_ctx* c, int l, T* u, T* t, const T* f, const T* k, int sweeps, bool zero_guess,
          const T* ec = nullptr, T* fc = nullptr)
{
  const Level& L = c->lv[l];
  const int dim = c->g.dim;
  const bool tiled = use_tiled(c, l);
  // the blocked pass that takes the correction is the first one: two sweeps unless only one
  // is asked for (FP64 passes fuse the correction into 2-sweep passes only)
  const bool pair = sweeps >= 2 && mgk::rbgs_tiled_max_sweeps(k != nullptr, sizeof(T)) == 2;
  if (ec && (sweeps == 0 || !(c->fuse & MG_FUSE_PROLONG) ||
             (tiled && (!mgk::rbgs_tiled_fuses_prolong(sizeof(T), k != nullptr) ||
                        (sizeof(T) == 8 && !pair))))) {
    // coarse-grid correction as a separate pass when it cannot ride on a fused sweep
    mgk::prolong_add<T>(c->s, dim, c->lv[l + 1].n, ec, u);
    ec = nullptr;
  }
  if (sweeps == 0) {
    if (zero_guess) mgk::fill<T>(c->s, L.N, T(0), u);
    return u;
  }
  if (zero_guess && !(c->fuse & MG_FUSE_ZERO)) {
    mgk::fill<T>(c->s, L.N, T(0), u);
    zero_guess = false;
  }
  if (tiled) {
    T* cur = u;
    T* other = t;
    int left = sweeps;
    bool zero = zero_guess;
    const int maxsw = mgk::rbgs_tiled_max_sweeps(k != nullptr, sizeof(T));
    while (left > 0) {
      const int sw = left >= maxsw ? maxsw : left;
      // fc: the residual restriction rides on the (single) pre-smoothing pass
      mgk::rbgs_tiled<T>(c->s, L.n, L.h, k, f, cur, other, sw, zero, ec, left == sw ? fc : nullptr);
      T* x = cur;
      cur = other;
      other = x;
      left -= sw;
      zero = false;
      ec = nullptr;
    }
    return cur;
  }
  // per-colour kernels; the zero guess or the coarse-grid correction rides on the first
  // colour-0 half-sweep (the boundary of a zero-guess level, a coarse level, is 0)
  for (int s = 0; s < sweeps; ++s) {
    if (s == 0 && (zero_guess || ec)) mgk::rbgs_first<T>(c->s, dim, L.n, L.h, k, f, u, ec);
    else mgk::rbgs_colour<T>(c->s, dim, L.n, L.h, k, f, u, 0);
    mgk::rbgs_colour<T>(c->s, dim, L.n, L.h, k, f, u, 1);
  }
  return u;
}

// One V(nu1,nu2)-cycle on level l for A_l x = f with x in u (or, when zero_guess, x = 0).
// Returns the buffer (u or t) holding the new iterate.
template <typename T>
T* cycle(mg_ctx* c, int l, T* u, T* t, const T* f, bool zero_guess)
{
  const int dim = c->g.dim;
  const Level& L = c->lv[l];
  const View<T> V = view<T>(c, l);
  if ((c->fuse & MG_FUSE_TAIL) && l == c->tail_first && zero_guess && u == V.u && f == V.f) {
    // levels l .. coarsest in one launch (same arithmetic as the per-level kernels)
    mgk::TailArgs<T> a{};
    a.nlev = c->g.levels - l;
    a.nu1 = c->g.nu1;
    a.nu2 = c->g.nu2;
    a.ainv = c->ainv;
    for (int q = 0; q < a.nlev; ++q) {
      const View<T> W = view<T>(c, l + q);
      const double h = c->lv[l + q].h;
      a.lv[q] = {W.u, W.f, W.k, c->lv[l + q].n, (T)(h * h), (T)(1.0 / (h * h))};
    }
    mgk::tail_cycle<T>(c->s, dim, a);
    return u;
  }
  if (l == c->g.levels - 1) {
    mgk::coarsest_solve<T>(c->s, dim, L.n, c->ainv, f, u);
    return u;
  }
  const View<T> C = view<T>(c, l + 1);
  // residual + restriction inside the pre-smoothing pass: one 2-sweep pass with constant
  // coefficients (rbgs_tiled_fuses_restrict)
  const bool fuse_r = use_tiled(c, l) && (c->fuse & MG_FUSE_RESTRICT) && c->g.nu1 == 2 &&
                      mgk::rbgs_tiled_max_sweeps(V.k != nullptr, sizeof(T)) == 2 &&
                      mgk::rbgs_tiled_fuses_restrict(sizeof(T), V.k != nullptr);
  T* cur = smooth<T>(c, l, u, t, f, V.k, c->g.nu1, zero_guess, nullptr, fuse_r ? C.f : nullptr);
  if (!fuse_r) {
    if (use_tiled(c, l)) mgk::restrict_residual_tiled<T>(c->s, L.n, L.h, V.k, f, cur, C.f);
    else mgk::restrict_residual<T>(c->s, dim, L.n, L.h, V.k, f, cur, C.f);
  }
  T* ec = cycle<T>(c, l + 1, C.u, C.t, C.f, true);
  // u += P ec, fused into the first post-smoothing pass on large 3D levels (FP32)
  T* other = cur == u ? t : u;
  return smooth<T>(c, l, cur, other, f, V.k, c->g.nu2, false, ec);
}

mg_status read_scalar(mg_ctx* c, const double* dev, double* host)
{
  mg_status st = hip_check(c, hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, c->s),
                           "reading a norm");
  if (st) return st;
  return hip_check(c, hipStreamSynchronize(c->s), "stream synchronisation");
}

// Power of two nearest (in log2) to the root-mean-square of a residual of norm rn.  The
// FP32 right-hand side is r / scale; a power of two changes no float result and keeps the
// values far from the float range limits.
double ir_scale(const mg_ctx* c, double rn)
{
  const int n = c->g.n;
  const double m = c->g.dim == 3 ? (double)(n - 2) * (n - 2) * (n - 2) : (double)(n - 2) * (n - 2);
  const double rms = rn / std::sqrt(m);
  if (!(rms > 0) || !std::isfinite(rms)) return 1.0;
  return std::ldexp(1.0, (int)std::lround(std::log2(rms)));
}

// ||f - A u||^2 (mode 0) or of the full right-hand side (mode 1) into c->scal[slot].
void norm2(mg_ctx* c, const double* f, const double* u, int mode, int slot)
{
  const Level& L0 = c->lv[0];
  if (use_tiled(c, 0))
    mgk::resid_norm2_tiled(c->s, L0.n, L0.h, L0.k, f, u, mode, c->partial, c->scal + slot);
  else
    mgk::resid_norm2(c->s, c->g.dim, L0.n, L0.h, L0.k, f, u, mode, c->partial, c->scal + slot);
}

// One outer step of iterative refinement (FP64 u, f) with the per-step kernels:
// r32 = (f - A u)/scale, e32 = one FP32 V-cycle from e = 0, u += scale * e32.
mg_status ir_step(mg_ctx* c, const double* f, double* u, double scale)
{
  const int dim = c->g.dim;
  Level& L0 = c->lv[0];
  mgk::ir_residual(c->s, dim, L0.n, L0.h, L0.k, f, u, 1.0 / scale, L0.f32, c->partial,
                   c->scal);
  float* e = cycle<float>(c, 0, L0.u32, L0.t32, L0.f32, true);
  mgk::ir_update(c->s, dim, L0.n, scale, e, u);
  return launch_check(c, "refinement step");
}

// One FP64 cycle on the caller's (f, u); the result ends in u.
mg_status f64_cycle(mg_ctx* c, const double* f, double* u)
{
  Level& L0 = c->lv[0];
  double* r = cycle<double>(c, 0, u, L0.t, f, false);
  if (r != u) mgk::copy<double>(c->s, L0.N, r, u);
  return launch_check(c, "V-cycle");
}

mg_status check_ready(mg_ctx* c)
{
  if (!c) return fail(nullptr, MG_EINVAL, "context is NULL");
  if (c->g.variable && !c->coeffs)
    return fail(c, MG_ESTATE, "variable-coefficient context: call mg_set_coefficients first");
  return MG_OK;
}

mg_status finish(mg_ctx* c, int k, double rel, double tol, int* cycles, double* relres,
                 mg_status st)
{
  if (cycles) *cycles = k;
  if (relres) *relres = rel;
  if (st) return st;
  if (!std::isfinite(rel)) return fail(c, MG_ENAN, "residual norm is not finite after %d cycles", k);
  if (rel > tol)
    return fail(c, MG_ENOCONV, "relative residual %.3e > tol %.3e after %d cycles", rel, tol, k);
  return MG_OK;
}

// Enqueues the copy of `count` device scalars to the pinned host words and the event after it.
mg_status read_scalar_start(mg_ctx* c, const double* dev, int count = 1)
{
  mg_status st = hip_check(c, hipMemcpyAsync(c->hnorm, dev, count * sizeof(double),
                                             hipMemcpyDeviceToHost, c->s), "reading a norm");
  if (!st) st = hip_check(c, hipEventRecord(c->ev, c->s), "recording the norm event");
  return st;
}

mg_status read_scalar_finish(mg_ctx* c, double* host, int count = 1)
{
  if (mg_status st = hip_check(c, hipEventSynchronize(c->ev), "waiting for a norm")) return st;
  for (int i = 0; i < count; ++i) host[i] = c->hnorm[i];
  return MG_OK;
}

// Whether the FP32 correction cycle's last level-0 post-smoothing pass can also perform the
// refinement step (rbgs_tiled_refine): a blocked level 0 with a constant coefficient, one
// 2-sweep post-smoothing pass that takes the coarse-grid correction, and a launch whose
// workgroups' partial sums fit the partial-sum buffer.
bool refine_fusable(const mg_ctx* c)
{
  return (c->fuse & MG_FUSE_REFINE) && (c->fuse & MG_FUSE_PROLONG) && use_tiled(c, 0) &&
         !c->g.variable && c->g.nu2 == 2 && mgk::rbgs_tiled_max_sweeps(false, 4) == 2 &&
         mgk::rbgs_tiled_refine_fits(c->lv[0].n);
}

// Level-0 FP32 buffers of a fused solve: the cycle's right-hand side and the two buffers of
// its correction.  The fused pass writes the next right-hand side into the buffer that
// holds neither the correction nor the current right-hand side, so the three rotate.  k
// counts the cycles: the right-hand side's scale is the device scalar ss[k mod 2], the next
// one's ss[(k+1) mod 2].
struct FusedIr {
  float *rhs, *u, *t;
  int k;
};

// One FP32 correction cycle from e = 0 on the right-hand side st.rhs, with its last pass
// fused with the refinement step: uout = u + s e, the next right-hand side, the residual
// norm into scal[0] and the scale after the next one into ss[k mod 2] (read by the cycle
// after next, stream-ordered).
mg_status fused_ir_cycle(mg_ctx* c, const double* f, const double* u, double* uout, FusedIr& st)
{
  const Level& L0 = c->lv[0];
  const View<float> C = view<float>(c, 1);
  const bool fuse_r = (c->fuse & MG_FUSE_RESTRICT) && c->g.nu1 == 2 &&
                      mgk::rbgs_tiled_fuses_restrict(sizeof(float), false);
  float* cur = smooth<float>(c, 0, st.u, st.t, st.rhs, nullptr, c->g.nu1, true, nullptr,
                             fuse_r ? C.f : nullptr);
  if (!fuse_r) mgk::restrict_residual_tiled<float>(c->s, L0.n, L0.h, nullptr, st.rhs, cur, C.f);
  float* ec = cycle<float>(c, 1, C.u, C.t, C.f, true);
  float* next = cur == st.u ? st.t : st.u;
  double* ss = c->scal + 4;
  if (!mgk::rbgs_tiled_refine(c->s, L0.n, L0.h, st.rhs, cur, ec, f, u, uout, next,
                              ss + (st.k & 1), ss + ((st.k + 1) & 1), c->partial, c->scal,
                              ss + (st.k & 1)))
    return fail(c, MG_EINVAL, "grid too large for the fused refinement pass");
  st.u = st.rhs;
  st.t = cur;
  st.rhs = next;
  ++st.k;
  return launch_check(c, "V-cycle with the refinement step");
}

// Refinement on a large 3D grid with the fused pass (mg_resid_tiled.hip): every pass
// applies the previous FP32 correction, forms the FP64 residual, its norm and the scaled
// FP32 right-hand side of the next cycle, writing the updated iterate out of place (u and
// the level's second buffer alternate).  The scale of a pass's r32 is a power of two taken
// from the previous residual norm; powers of two change no float result.
//
// Norm read-back overlaps the next FP32 V-cycle: when the contraction observed so far says
// the norm being read will still be above the tolerance, the next cycle (which writes only
// the FP32 correction and the coarse levels, never the iterate or r32) is enqueued before
// the host waits for the norm.  If the tolerance was reached after all, that cycle's
// results are never used: the iterate, the cycle count and the stopping decision are those
// of the plain loop, only GPU time is lost.
//
// bn: the right-hand-side norm, or 0 to have the first pass compute it beside the residual
// norm (same operations and summation order as the separate norm pass); that pass then
// scales r32 by the previous solve's right-hand side and is repeated with the right scale
// in the rare case that this is more than 2^40 off (powers of two within that range change
// no float result).
mg_status solve_ir_streamed(mg_ctx* c, const double* f, double* u, double tol, double bn,
                            int* cycles, double* relres)
{
  Level& L0 = c->lv[0];
  double* cur = u;
  double* other = L0.t;
  const bool fused_rhs = !(bn > 0);
  // The correction cycle's last pass may also apply the correction and form the next
  // residual (refine_fusable): the speculative cycle below then writes the iterate (out of
  // place, into `other`) and the scales of the right-hand sides live on the device.
  const bool fused = refine_fusable(c);
  FusedIr fst{L0.f32, L0.u32, L0.t32, 0};
  double scale = ir_scale(c, fused_rhs ? c->last_bn : bn);  // scale of the r32 being written
  double rn2 = 0;
  const bool overlap = c->hnorm != nullptr && c->ev != nullptr;
  mgk::ir_pass_tiled(c->s, L0.n, L0.h, L0.k, f, cur, nullptr, 0.0, 1.0 / scale, other, L0.f32,
                     c->partial, c->scal, fused_rhs ? c->partial_b : nullptr);
  std::swap(cur, other);
  if (fused) mgk::ir_scales_init(c->s, L0.n, c->scal, scale, c->scal + 4);
  mg_status st = launch_check(c, "refinement pass");
  // relative residual predicted for the norm in flight (infinite: no history yet)
  double predicted = INFINITY, rel_prev = NAN;
  float* spec = nullptr;  // a V-cycle enqueued ahead of the norm read
  // reads `count` norms from scal (residual, then right-hand side), overlapping the next
  // V-cycle when the prediction says one is needed
  auto read_norm = [&](double* out, int count) -> mg_status {
    if (!overlap) {
      mg_status s2 = MG_OK;
      for (int i = 0; i < count && !s2; ++i) s2 = read_scalar(c, c->scal + i, &out[i]);
      return s2;
    }
    mg_status s2 = read_scalar_start(c, c->scal, count);
    if (!s2 && predicted > 4.0 * tol && c->g.max_cycles > 0) {
      if (fused) {
        s2 = fused_ir_cycle(c, f, cur, other, fst);
        spec = fst.rhs;  // marks the cycle as enqueued
      } else {
        spec = cycle<float>(c, 0, L0.u32, L0.t32, L0.f32, true);
        s2 = launch_check(c, "V-cycle");
      }
    }
    if (!s2) s2 = read_scalar_finish(c, out, count);
    return s2;
  };
  if (!st && fused_rhs) {
    double two[2] = {0, 0};
    st = read_norm(two, 2);
    rn2 = two[0];
    bn = std::sqrt(two[1]);
    if (!(bn > 0)) bn = 1.0;
    const double ideal = ir_scale(c, bn);
    if (!st && (ideal / scale > 0x1p40 || scale / ideal > 0x1p40)) {
      // redo the first pass with the right scale (its r32 feeds the first cycle: a cycle
      // enqueued ahead is discarded, with its buffer rotation).  It reads the first pass's
      // output, a copy of the iterate: a cycle enqueued ahead may have written `other`.
      spec = nullptr;
      fst = FusedIr{L0.f32, L0.u32, L0.t32, 0};
      scale = ideal;
      mgk::ir_pass_tiled(c->s, L0.n, L0.h, L0.k, f, cur, nullptr, 0.0, 1.0 / scale, other,
                         L0.f32, c->partial, c->scal);
      std::swap(cur, other);
      if (fused) mgk::ir_scales_init(c->s, L0.n, c->scal, scale, c->scal + 4);
      st = launch_check(c, "refinement pass");
      if (!st) st = read_norm(&rn2, 1);
    }
  } else if (!st) {
    st = read_norm(&rn2, 1);
  }
  c->last_bn = bn;
  double rel = std::sqrt(rn2) / bn;
  int k = 0;
  while (!st && std::isfinite(rel) && rel > tol && k < c->g.max_cycles) {
    if (fused) {
      if (!spec) st = fused_ir_cycle(c, f, cur, other, fst);
      spec = nullptr;
      std::swap(cur, other);
      ++k;
      if (st) break;
    } else {
      float* e = spec ? spec : cycle<float>(c, 0, L0.u32, L0.t32, L0.f32, true);
      spec = nullptr;
      const double next = ir_scale(c, std::sqrt(rn2));
      mgk::ir_pass_tiled(c->s, L0.n, L0.h, L0.k, f, cur, e, scale, 1.0 / next, other, L0.f32,
                         c->partial, c->scal);
      std::swap(cur, other);
      scale = next;
      ++k;
      if ((st = launch_check(c, "refinement pass"))) break;
    }
    // contraction so far: the next relative residual is about rel * (rel / rel_prev)
    const double rho = std::isfinite(rel_prev) && rel_prev > 0 ? rel / rel_prev : 1.0;
    predicted = k < c->g.max_cycles ? rel * rho : 0.0;
    rel_prev = rel;
    if ((st = read_norm(&rn2, 1))) break;
    rel = std::sqrt(rn2) / bn;
  }
  if (cur != u) mgk::copy<double>(c->s, L0.N, cur, u);
  if (!st) st = launch_check(c, "copy");
  return finish(c, k, rel, tol, cycles, relres, st);
}

mg_status solve_impl(mg_ctx* c, const double* f, double* u, double tol, int* cycles,
                     double* relres)
{
  if (mg_status st = check_ready(c)) return st;
  if (!f || !u) return fail(c, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(c, MG_EINVAL, "tol must be > 0");
  Level& L0 = c->lv[0];
  if (use_tiled(c, 0)) mgk::copy_boundary(c->s, c->g.dim, L0.n, u, L0.t);
  // FP32 refinement with the fused pass: once a previous solve gave a right-hand-side
  // scale, the first pass computes the right-hand-side norm itself
  if (c->g.precision == MG_F32_IR && use_tiled(c, 0) && !c->g.variable && c->last_bn > 0)
    return solve_ir_streamed(c, f, u, tol, 0.0, cycles, relres);
  double bn2 = 0, rn2 = 0;
  const bool both = use_tiled(c, 0) && !c->g.variable && c->g.precision == MG_F64;
  if (both) {
    // residual and right-hand-side norms in one pass (each in its own pass's order)
    mgk::resid_norm2_both_tiled(c->s, L0.n, L0.h, f, u, c->partial, c->partial_b, c->scal);
    if (mg_status st = launch_check(c, "norm")) return st;
    if (mg_status st = read_scalar(c, c->scal + 1, &bn2)) return st;
    if (mg_status st = read_scalar(c, c->scal, &rn2)) return st;
  } else {
    norm2(c, f, u, 1, 1);
    if (mg_status st = launch_check(c, "norm")) return st;
    if (mg_status st = read_scalar(c, c->scal + 1, &bn2)) return st;
  }
  double bn = std::sqrt(bn2);
  if (!(bn > 0)) bn = 1.0;
  if (c->g.precision == MG_F32_IR && use_tiled(c, 0))
    return solve_ir_streamed(c, f, u, tol, bn, cycles, relres);
  if (!both) {
    norm2(c, f, u, 0, 0);
    if (mg_status st = launch_check(c, "norm")) return st;
    if (mg_status st = read_scalar(c, c->scal, &rn2)) return st;
  }
  double rn = std::sqrt(rn2);
  double rel = rn / bn;
  int k = 0;
  mg_status st = MG_OK;
  while (std::isfinite(rel) && rel > tol && k < c->g.max_cycles) {
    if (c->g.precision == MG_F32_IR) st = ir_step(c, f, u, ir_scale(c, rn));
    else st = f64_cycle(c, f, u);
    if (st) break;
    ++k;
    norm2(c, f, u, 0, 0);
    if ((st = launch_check(c, "norm"))) break;
    if ((st = read_scalar(c, c->scal, &rn2))) break;
    rn = std::sqrt(rn2);
    rel = rn / bn;
  }
  return finish(c, k, rel, tol, cycles, relres, st);
}

mg_status level_check(mg_ctx* c, int level, bool needs_coarser)
{
  if (mg_status st = check_ready(c)) return st;
  if (level < 0 || level >= c->g.levels || (needs_coarser && level >= c->g.levels - 1))
    return fail(c, MG_EINVAL, "level %d out of range", level);
  return MG_OK;
}

template <typename T>
mg_status smooth_impl(mg_ctx* c, int level, const T* f, T* u, int sweeps)
{
  if (mg_status st = level_check(c, level, false)) return st;
  if (!f || !u || sweeps < 0) return fail(c, MG_EINVAL, "bad smoothing arguments");
  const Level& L = c->lv[level];
  const View<T> V = view<T>(c, level);
  if (!V.t) return fail(c, MG_ESTATE, "FP32 arrays exist only in MG_F32_IR contexts");
  if (c->g.variable && !V.k) return fail(c, MG_ESTATE, "no coefficients for this precision");
  // the level's second buffer holds the Dirichlet data of u while the fused kernel
  // alternates between the two
  T* t = V.t;
  if (use_tiled(c, level)) {
    if (sizeof(T) == 8)
      mgk::copy_boundary(c->s, c->g.dim, L.n, reinterpret_cast<const double*>(u),
                         reinterpret_cast<double*>(t));
    else
      mgk::copy<T>(c->s, L.N, u, t);
  }
  T* r = smooth<T>(c, level, u, t, f, V.k, sweeps, false);
  if (r != u) mgk::copy<T>(c->s, L.N, r, u);
  return launch_check(c, "smoothing");
}

// Lays a context out on `workspace` (`need` bytes) and enqueues the workspace's
// initialisation: shared by mg_setup and mg_solve_noalloc.
mg_status init_ctx(mg_ctx* c, const mg_grid* grid, void* workspace, size_t need, hipStream_t s)
{
  c->g = *grid;
  c->s = s;
  Carver cv{static_cast<char*>(workspace)};
  layout(grid, cv, c);
  for (int l = 1; l + 1 < grid->levels && l - 1 < mgk::kMaxTail; ++l)
    if (mgk::tail_fits(grid->dim, c->lv[l].n) && grid->levels - l <= mgk::kMaxTail) {
      c->tail_first = l;
      break;
    }
  // zero the whole workspace once: coarse boundaries (zero Dirichlet data of corrections)
  // and the boundaries of the second buffers are never written afterwards
  mgk::fill<double>(c->s, need / sizeof(double), 0.0, static_cast<double*>(workspace));
  if (!grid->variable) {
    const Level& Lc = c->lv[grid->levels - 1];
    mgk::coarsest_factor(c->s, grid->dim, Lc.n, Lc.h, nullptr, c->chol, c->ainv, c->flag);
  }
  return launch_check(c, "setup");
}

// Copies k into the workspace and builds the coefficient hierarchy and the coarsest factor.
mg_status set_coefficients_impl(mg_ctx* c, const double* k)
{
  const int dim = c->g.dim;
  mgk::copy<double>(c->s, c->lv[0].N, k, c->lv[0].k);
  for (int l = 1; l < c->g.levels; ++l) mgk::coarsen_k(c->s, dim, c->lv[l - 1].n, c->lv[l - 1].k, c->lv[l].k);
  if (c->g.precision == MG_F32_IR)
    for (int l = 0; l < c->g.levels; ++l) mgk::cast_to_f32(c->s, c->lv[l].N, c->lv[l].k, c->lv[l].k32);
  const Level& Lc = c->lv[c->g.levels - 1];
  mgk::coarsest_factor(c->s, dim, Lc.n, Lc.h, Lc.k, c->chol, c->ainv, c->flag);
  if (mg_status st = launch_check(c, "set_coefficients")) return st;
  c->coeffs = true;
  return MG_OK;
}

}  // namespace

// ------------------------------------------------- device memory of mg_solve_noalloc
// A file-scope array: every GPU the library runs on holds its own copy from the loading of
// this code object there until the process ends.  In host code the name `scratch` is only a
// host-side stand-in, never a device address: host code uses the address that
// hipGetSymbolAddress returns for the current device (scratch_address below).
static __device__ __align__(256) unsigned char scratch[MG_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per device with
// that device current.
mg_status scratch_address(void** out)
{
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, MG_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(nullptr, MG_EINVAL, "device %d: at most %d devices are supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, MG_EHIP, "hipGetSymbolAddress of the static scratch array: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MG_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

mg_status mg_validate(const mg_grid* grid) { return validate(grid, nullptr); }

size_t mg_workspace_bytes(const mg_grid* grid)
{
  if (validate(grid, nullptr) != MG_OK) return 0;
  Carver cv{nullptr};
  layout(grid, cv, nullptr);
  return cv.off + kAlign;
}

mg_status mg_setup(const mg_grid* grid, void* workspace, size_t bytes, void* stream, mg_ctx** out)
{
  if (!out) return fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (mg_status st = validate(grid, nullptr)) return st;
  if (!workspace) return fail(nullptr, MG_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(nullptr, MG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  const size_t need = mg_workspace_bytes(grid);
  if (bytes < need)
    return fail(nullptr, MG_ENOMEM, "workspace of %zu bytes < %zu required", bytes, need);
  mg_ctx* c = new (std::nothrow) mg_ctx;
  if (!c) return fail(nullptr, MG_ENOMEM, "host allocation of the context failed");
  mg_status st = init_ctx(c, grid, workspace, need, static_cast<hipStream_t>(stream));
  // one pinned host word for overlapped norm reads (FP32 refinement); without it the solve
  // reads synchronously
  if (!st && grid->precision == MG_F32_IR) {
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 64, hipHostMallocDefault) == hipSuccess) {
      c->hnorm = static_cast<double*>(hp);
      if (hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) c->ev = nullptr;
    }
    (void)hipGetLastError();  // a failed pinned allocation only disables the overlap
  }
  if (st) {
    snprintf(g_err, sizeof g_err, "%s", c->err);
    delete c;
    return st;
  }
  *out = c;
  return MG_OK;
}

mg_status mg_set_coefficients(mg_ctx* c, const double* k)
{
  if (!c) return fail(nullptr, MG_EINVAL, "context is NULL");
  if (!c->g.variable) return fail(c, MG_ESTATE, "constant-coefficient context");
  if (!k) return fail(c, MG_EINVAL, "k is NULL");
  return set_coefficients_impl(c, k);
}

mg_status mg_vcycle(mg_ctx* c, const double* f, double* u)
{
  if (mg_status st = check_ready(c)) return st;
  if (!f || !u) return fail(c, MG_EINVAL, "f and u must be non-NULL");
  Level& L0 = c->lv[0];
  if (use_tiled(c, 0)) mgk::copy_boundary(c->s, c->g.dim, L0.n, u, L0.t);
  if (c->g.precision == MG_F32_IR) {
    double rn2 = 0;
    norm2(c, f, u, 0, 0);
    if (mg_status st = read_scalar(c, c->scal, &rn2)) return st;
    return ir_step(c, f, u, ir_scale(c, std::sqrt(rn2)));
  }
  return f64_cycle(c, f, u);
}

mg_status mg_solve(mg_ctx* c, const double* f, double* u, double tol, int* cycles,
                   double* relres)
{
  return solve_impl(c, f, u, tol, cycles, relres);
}

mg_status mg_solve_adjoint(mg_ctx* c, const double* g, double* lambda, double tol, int* cycles,
                           double* relres)
{
  if (mg_status st = check_ready(c)) return st;
  if (!g || !lambda) return fail(c, MG_EINVAL, "g and lambda must be non-NULL");
  mgk::zero_boundary(c->s, c->g.dim, c->g.n, lambda);
  return solve_impl(c, g, lambda, tol, cycles, relres);
}

mg_status mg_grad(mg_ctx* c, const double* u, const double* lambda, double* dk, double* df)
{
  if (!c) return fail(nullptr, MG_EINVAL, "context is NULL");
  if (!u || !lambda) return fail(c, MG_EINVAL, "u and lambda must be non-NULL");
  mgk::grad(c->s, c->g.dim, c->g.n, u, lambda, dk, df);
  return launch_check(c, "gradient");
}

mg_status mg_smooth(mg_ctx* c, int level, const double* f, double* u, int sweeps)
{
  return smooth_impl<double>(c, level, f, u, sweeps);
}

mg_status mg_smooth_f32(mg_ctx* c, int level, const float* f, float* u, int sweeps)
{
  return smooth_impl<float>(c, level, f, u, sweeps);
}

mg_status mg_residual(mg_ctx* c, int level, const double* f, const double* u, double* r)
{
  if (mg_status st = level_check(c, level, false)) return st;
  if (!f || !u || !r) return fail(c, MG_EINVAL, "NULL array");
  const Level& L = c->lv[level];
  mgk::residual<double>(c->s, c->g.dim, L.n, L.h, L.k, f, u, r);
  return launch_check(c, "residual");
}

mg_status mg_restrict_residual(mg_ctx* c, int level, const double* f, const double* u, double* fc)
{
  if (mg_status st = level_check(c, level, true)) return st;
  if (!f || !u || !fc) return fail(c, MG_EINVAL, "NULL array");
  const Level& L = c->lv[level];
  mgk::zero_boundary(c->s, c->g.dim, c->lv[level + 1].n, fc);
  if (use_tiled(c, level)) mgk::restrict_residual_tiled<double>(c->s, L.n, L.h, L.k, f, u, fc);
  else mgk::restrict_residual<double>(c->s, c->g.dim, L.n, L.h, L.k, f, u, fc);
  return launch_check(c, "restriction");
}

mg_status mg_restrict_residual_f32(mg_ctx* c, int level, const float* f, const float* u, float* fc)
{
  if (mg_status st = level_check(c, level, true)) return st;
  if (!f || !u || !fc) return fail(c, MG_EINVAL, "NULL array");
  if (c->g.precision != MG_F32_IR) return fail(c, MG_ESTATE, "FP32 path needs an MG_F32_IR context");
  const Level& L = c->lv[level];
  mgk::fill<float>(c->s, c->lv[level + 1].N, 0.0f, fc);
  if (use_tiled(c, level)) mgk::restrict_residual_tiled<float>(c->s, L.n, L.h, L.k32, f, u, fc);
  else mgk::restrict_residual<float>(c->s, c->g.dim, L.n, L.h, L.k32, f, u, fc);
  return launch_check(c, "restriction");
}

mg_status mg_prolong_correct(mg_ctx* c, int level, const double* ec, double* u)
{
  if (mg_status st = level_check(c, level, true)) return st;
  if (!ec || !u) return fail(c, MG_EINVAL, "NULL array");
  mgk::prolong_add<double>(c->s, c->g.dim, c->lv[level + 1].n, ec, u);
  return launch_check(c, "prolongation");
}

mg_status mg_prolong_correct_f32(mg_ctx* c, int level, const float* ec, float* u)
{
  if (mg_status st = level_check(c, level, true)) return st;
  if (!ec || !u) return fail(c, MG_EINVAL, "NULL array");
  mgk::prolong_add<float>(c->s, c->g.dim, c->lv[level + 1].n, ec, u);
  return launch_check(c, "prolongation");
}

mg_status mg_coarsest_solve(mg_ctx* c, const double* f, double* u)
{
  if (mg_status st = check_ready(c)) return st;
  if (!f || !u) return fail(c, MG_EINVAL, "NULL array");
  const Level& L = c->lv[c->g.levels - 1];
  mgk::coarsest_solve<double>(c->s, c->g.dim, L.n, c->ainv, f, u);
  return launch_check(c, "coarsest solve");
}

mg_status mg_residual_norm2(mg_ctx* c, const double* f, const double* u, double* out)
{
  if (mg_status st = check_ready(c)) return st;
  if (!f || !u || !out) return fail(c, MG_EINVAL, "NULL argument");
  norm2(c, f, u, 0, 0);
  if (mg_status st = launch_check(c, "norm")) return st;
  return read_scalar(c, c->scal, out);
}

mg_status mg_solve_noalloc(const mg_grid* grid, const double* k, const double* f, double* u,
                           double tol, void* stream, int* cycles, double* relres)
{
  // every argument is checked before the first HIP call
  if (mg_status st = validate(grid, nullptr)) return st;
  if (grid->variable && !k) return fail(nullptr, MG_EINVAL, "variable-coefficient grid: k is NULL");
  if (!grid->variable && k) return fail(nullptr, MG_EINVAL, "k given for a constant-coefficient grid");
  if (!f || !u) return fail(nullptr, MG_EINVAL, "f and u must be non-NULL");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(nullptr, MG_EINVAL, "tol must be > 0");
  const size_t need = mg_workspace_bytes(grid);
  if (need > MG_NOALLOC_MAX_BYTES)
    return fail(nullptr, MG_ENOMEM,
                "grid needs %zu bytes of device workspace, more than the %zu bytes of the "
                "allocation-free solve: use mg_setup with a workspace", need,
                (size_t)MG_NOALLOC_MAX_BYTES);
  void* ws = nullptr;
  if (mg_status st = scratch_address(&ws)) return st;
  mg_ctx c;  // on the stack: no host allocation either (no pinned word: synchronous norm reads)
  mg_status st = init_ctx(&c, grid, ws, need, static_cast<hipStream_t>(stream));
  if (!st && grid->variable) st = set_coefficients_impl(&c, k);
  if (!st) st = solve_impl(&c, f, u, tol, cycles, relres);
  if (st) snprintf(g_err, sizeof g_err, "%s", c.err);
  return st;
}

mg_status mg_set_fusion(mg_ctx* c, int flags)
{
  if (!c) return fail(nullptr, MG_EINVAL, "context is NULL");
  if (flags & ~MG_FUSE_ALL) return fail(c, MG_EINVAL, "unknown fusion flags 0x%x", flags);
  c->fuse = flags;
  return MG_OK;
}

const char* mg_last_error(const mg_ctx* c) { return c ? c->err : g_err; }

void mg_destroy(mg_ctx* c) { delete c; }

}  // extern "C"
