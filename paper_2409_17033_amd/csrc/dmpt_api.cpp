// Host runtime of libdmpt: argument validation, workspace carve-up, bounds,
// the chunked step loop with device-side sigma/stop decisions, projection,
// outputs.  Implements the C ABI declared in include/dmpt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <string>
#include <vector>

#include "dmpt_fermi.h"
#include "dmpt_internal.h"
#include "dmpt_lists.h"
#include "dmpt_scf.h"
#include "sp2_rule.h"

namespace dmpt {
namespace {

thread_local std::string g_last_error;

dmpt_status fail(dmpt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define DMPT_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(DMPT_ERR_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                   \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
constexpr int kOutBlocks = 1024;
constexpr int kChunk = 8;   // step launches between host polls of the done flag

struct Opts {
  int n, nocc, prec, bounds, lanczos_steps, max_iter, min_iter, sweep, project, profile, ckpt, refine;
  double emin, emax, idem_tol, spin, sweep_tol;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
};

dmpt_status normalise(const dmpt_opts* o, Opts* r) {
  if (!o) return fail(DMPT_ERR_ARG, "opts is NULL");
  if (o->n < 1 || o->n > 65536) return fail(DMPT_ERR_ARG, "n = %d out of range [1, 65536]", o->n);
  if (o->nocc < 0 || o->nocc > o->n) return fail(DMPT_ERR_ARG, "nocc = %d out of range [0, n]", o->nocc);
  if (o->precision < 0 || o->precision > DMPT_SPLIT_FP16) return fail(DMPT_ERR_ARG, "unknown precision %d", o->precision);
  if (o->bounds < 0 || o->bounds > DMPT_BOUNDS_GIVEN) return fail(DMPT_ERR_ARG, "unknown bounds mode %d", o->bounds);
  if (o->bounds == DMPT_BOUNDS_GIVEN && !(std::isfinite(o->emin) && std::isfinite(o->emax) && o->emax > o->emin))
    return fail(DMPT_ERR_ARG, "given bounds need finite emin < emax");
  if (o->lanczos_steps < 0 || o->lanczos_steps > 512) return fail(DMPT_ERR_ARG, "lanczos_steps out of range [0, 512]");
  if (o->max_iter < 0 || o->max_iter > DMPT_MAX_STEPS) return fail(DMPT_ERR_ARG, "max_iter out of range [0, %d]", DMPT_MAX_STEPS);
  if (o->sweep != DMPT_SWEEP_FORWARD && o->sweep != DMPT_SWEEP_ADJOINT) return fail(DMPT_ERR_ARG, "unknown sweep %d", o->sweep);
  if (!(std::isfinite(o->idem_tol) && o->idem_tol >= 0)) return fail(DMPT_ERR_ARG, "idem_tol must be finite and >= 0");
  if (!std::isfinite(o->spin)) return fail(DMPT_ERR_ARG, "spin must be finite");
  if (o->project < 0 || o->project > 2) return fail(DMPT_ERR_ARG, "project must be 0, 1 or 2");
  if (o->project == 2 && (o->precision != DMPT_SPLIT3X_BF16 || !o->refine))
    return fail(DMPT_ERR_ARG, "project = 2 needs DMPT_SPLIT3X_BF16 with refine");
  if (o->profile != 0 && o->profile != 1) return fail(DMPT_ERR_ARG, "profile must be 0 or 1");
  if (o->ckpt_interval < 0 || o->ckpt_interval > DMPT_MAX_STEPS)
    return fail(DMPT_ERR_ARG, "ckpt_interval out of range [0, %d]", DMPT_MAX_STEPS);
  if (o->refine < 0 || o->refine > 2) return fail(DMPT_ERR_ARG, "refine must be 0, 1 or 2");
  if (o->refine && (o->sweep != DMPT_SWEEP_FORWARD || !o->project))
    return fail(DMPT_ERR_ARG, "refine needs the forward sweep with the projection");
  if (!(std::isfinite(o->sweep_tol) && o->sweep_tol >= 0.0 && o->sweep_tol < 0.25))
    return fail(DMPT_ERR_ARG, "sweep_tol must be in [0, 1/4)");
  if (o->sweep_tol > 0.0 && !o->refine)
    return fail(DMPT_ERR_ARG, "sweep_tol needs refine (the residual correction removes the truncation error)");
  r->n = o->n;
  r->nocc = o->nocc;
  r->prec = o->precision == DMPT_FP32 ? kFP32
          : o->precision == DMPT_SPLIT_BF16 ? kSplit2
          : o->precision == DMPT_SPLIT3_BF16 ? kSplit3
          : o->precision == DMPT_SPLIT3X_BF16 ? kSplit32
          : o->precision == DMPT_SPLIT_FP16 ? kSplitH : kBF16;
  r->bounds = o->bounds;
  r->lanczos_steps = o->lanczos_steps ? o->lanczos_steps : 32;
  r->max_iter = o->max_iter ? o->max_iter : 100;
  r->min_iter = o->min_iter < 0 ? 10 : o->min_iter;
  r->sweep = o->sweep;
  r->project = o->project;
  r->profile = o->profile;
  r->ckpt = o->ckpt_interval;
  r->refine = o->refine;
  r->emin = o->emin;
  r->emax = o->emax;
  r->idem_tol = o->idem_tol;
  r->spin = o->spin == 0.0 ? 2.0 : o->spin;
  r->sweep_tol = o->sweep_tol;
  r->stream = (hipStream_t)o->stream;
  r->ws = (char*)o->workspace;
  r->ws_bytes = o->workspace_bytes;
  return DMPT_OK;
}

// Workspace plan.  All offsets are from the workspace base.
struct Plan {
  int n, n_pad, nobs, prec, tile, ntile, nb64, nparts_step;
  int xslots;
  int ckpt, nckpt;                 // adjoint checkpoint interval (0: every X_n kept) and slot count
  size_t mat_f32, mat_op, mat_op2, mat_meta; // bytes per matrix: master, operand copy (and the
                                             // two-term copy of the three-term-X^2 option), metadata
  size_t off_ctl, off_part[2], off_jobs, off_jobs_proj, off_gersh, off_lz, off_a0, off_x, off_y;
  size_t x_slot_bytes, y_obs_bytes, y_slot_bytes;
  // residual refinement (opts.refine): operand copies of D, H, A_k, Y_k in the
  // residual's format, two FP32 product buffers, the BF16 copies of R_k and
  // D, the BF16 sweep's X and Y slots, and the norm partials
  int rprec;
  size_t rf_copy_bytes, rf_bslot_bytes;
  size_t off_rf_copy, off_rf_v, off_rf_r, off_rf_hist, off_rf_x, off_rf_y, off_rf_norm;
  // K-split tail tiles of the step and sweep lists (runs with the residual
  // correction): list-position -> slot tables, the combine lists and the
  // scratch of partial tile sums
  size_t off_split_slot, off_split_slot_proj, off_cjobs, off_cjobs_proj, off_split_buf;
  size_t total;
  int njobs_max, njobs_proj_max, lz_steps;
};

// Two-level accumulation: the MFMA accumulator is added into the running tile
// sum every `flush` groups of 4 pipeline stages.  Balancing the inner chain
// (F stages x MFMAs per stage per block) against the outer one (stages / F)
// gives F ~ sqrt(stages / chain); the constant is measured: the chi error
// against the closed form is U-shaped in F, with its minimum at about 3/8 of
// sqrt(stages / chain) for FP32, the FP16 split and the three-term BF16 split
// at N = 4096 and 8192 (outer FP32 sums cost more than inner MFMA ones).
int flush_interval(int prec, int n_pad) {
  // FP32 operands: each accumulator block goes into the FP64 tile sum every
  // 4 stages (64 k values, 32 MFMAs); the outer sum is exact, so a short
  // chain is best; 4 is the shortest interval the rotating schedule keeps
  // in the shadow of the MFMAs (measured at N = 8192: chi 7.0e-6 against
  // 1.67e-5 with two FP32 levels).
  if (prec == kFP32) return 4;
  const int chain = prec == kFP32 ? 8 : prec == kSplit3 ? 6 : (prec == kSplit2 || prec == kSplit32 || prec == kSplitH) ? 3 : 2;
  const int stages = n_pad / stage_k(prec);
  const double f = std::sqrt((double)stages / chain) * 0.375;
  return std::max(1, (int)std::lround(f));
}

void make_plan(const Opts& o, int nobs, Plan* p) {
  p->n = o.n;
  p->n_pad = (o.n + kPadTo - 1) / kPadTo * kPadTo;
  p->nobs = nobs;
  p->prec = o.prec;
  p->tile = kStepTM;
  p->ntile = p->n_pad / kStepTN;                       // 128-column blocks
  p->nb64 = p->n_pad / 64;
  p->nparts_step = step_tile_count(p->n_pad);
  const bool adjoint = nobs > 0 && o.sweep == DMPT_SWEEP_ADJOINT;
  // The adjoint keeps X_1 .. X_{max_iter+2} (slot n = X_n; the last launch may
  // write one iterate past the result before the stop is seen), or with a
  // checkpoint interval k: two working slots, one slot per X_n with
  // (n - 1) % k == 0, and k - 1 slots to recompute a segment.
  p->ckpt = adjoint ? o.ckpt : 0;
  p->nckpt = p->ckpt ? (o.max_iter + 1) / p->ckpt + 1 : 0;
  p->xslots = !adjoint ? 2 : p->ckpt ? 2 + p->nckpt + (p->ckpt - 1) : o.max_iter + 3;
  const size_t np2 = (size_t)p->n_pad * p->n_pad;
  p->mat_f32 = np2 * 4;
  p->mat_op = o.prec == kFP32 ? 0 : np2 * operand_bytes(o.prec);
  p->mat_op2 = np2 * operand2_bytes(o.prec);
  p->mat_meta = meta_bytes(std::max(p->nb64 * p->nb64, p->nparts_step));
  p->lz_steps = o.lanczos_steps;
  const int ut = p->nparts_step;                       // step tiles covering the upper triangle
  p->njobs_max = ut * (1 + std::max(nobs, 0)) + kMaxSplit;
  p->njobs_proj_max = ut * std::max(nobs, 1) + kMaxSplit;
  size_t off = 0;
  p->off_ctl = off; off = align_up(off + sizeof(Ctl));
  const size_t part_bytes = (size_t)p->nb64 * p->nb64 * sizeof(Part);
  p->off_part[0] = off; off = align_up(off + part_bytes);
  p->off_part[1] = off; off = align_up(off + part_bytes);
  p->off_jobs = off; off = align_up(off + (size_t)p->njobs_max * 4);
  p->off_jobs_proj = off; off = align_up(off + (size_t)p->njobs_proj_max * 4);
  p->off_gersh = off; off = align_up(off + (size_t)gershgorin_blocks(o.n) * sizeof(double2));
  p->off_lz = off; off = align_up(off + (size_t)(3 * o.n + 2 * (p->lz_steps + 2)) * sizeof(double));
  p->off_a0 = off; off = align_up(off + (size_t)kOutBlocks * std::max(nobs, 1) * sizeof(double));
  p->x_slot_bytes = align_up(p->mat_f32) + align_up(p->mat_op) + align_up(p->mat_op2) + align_up(p->mat_meta);
  p->off_x = off; off = align_up(off + p->x_slot_bytes * p->xslots);
  p->y_obs_bytes = p->x_slot_bytes;
  p->y_slot_bytes = p->y_obs_bytes * std::max(nobs, 0);
  p->off_y = off; off = align_up(off + p->y_slot_bytes * 2);
  p->rprec = o.prec == kSplitH ? kSplitH : o.prec == kFP32 ? kFP32 : kSplit3;
  if (o.refine && nobs > 0 && !adjoint) {
    const int k = std::max(nobs, 0);
    p->rf_copy_bytes = align_up(np2 * (p->rprec == kFP32 ? 4 : operand_bytes(p->rprec)));
    p->rf_bslot_bytes = align_up(np2 * 4) + align_up(np2 * 2) + align_up(p->mat_meta);
    p->off_rf_copy = off; off = align_up(off + p->rf_copy_bytes * (2 + 2 * (size_t)k));
    p->off_rf_v = off; off = align_up(off + np2 * 4 * 2);
    p->off_rf_r = off; off = align_up(off + np2 * 2 * k);
    // plain BF16 copies of X_1 .. X_{max_iter + 2} (slot n = X_n), written by the steps
    p->off_rf_hist = off; off = align_up(off + np2 * 2 * (size_t)(o.max_iter + 3));
    p->off_rf_x = off; off = align_up(off + p->rf_bslot_bytes);
    p->off_rf_y = off; off = align_up(off + p->rf_bslot_bytes * 2 * k);
    p->off_rf_norm = off; off = align_up(off + sizeof(double) * kNormBlocks * (2 + 2 * (size_t)k));
    p->off_split_slot = off; off = align_up(off + (size_t)p->njobs_max * 4);
    p->off_split_slot_proj = off; off = align_up(off + (size_t)p->njobs_proj_max * 4);
    p->off_cjobs = off; off = align_up(off + (size_t)kMaxSplit * 4);
    p->off_cjobs_proj = off; off = align_up(off + (size_t)kMaxSplit * 4);
    p->off_split_buf = off; off = align_up(off + (size_t)kMaxSplit * 2 * kSplitTileFloats * sizeof(float));
  }
  p->total = off;
}

// Plain BF16 matrix set of the refinement sweep: slot q (0/1) of X, or of
// observable k's Y (stride between observables).
MatRef bf16_ref(const Plan& p, char* ws, size_t off, int slot, int nmat) {
  const size_t np2 = (size_t)p.n_pad * p.n_pad;
  char* base = ws + off + (size_t)slot * p.rf_bslot_bytes * nmat;
  MatRef m;
  m.f32 = (float*)base;
  m.op = base + align_up(np2 * 4);
  m.meta = base + align_up(np2 * 4) + align_up(np2 * 2);
  m.stride_f32 = p.rf_bslot_bytes / 4;
  m.stride_op = p.rf_bslot_bytes;
  return m;
}

MatRef x_ref(const Plan& p, char* ws, int slot) {
  char* base = ws + p.off_x + (size_t)slot * p.x_slot_bytes;
  MatRef m;
  m.f32 = (float*)base;
  m.op = p.prec == kFP32 ? (void*)base : (void*)(base + align_up(p.mat_f32));
  m.op2 = p.mat_op2 ? (void*)(base + align_up(p.mat_f32) + align_up(p.mat_op)) : nullptr;
  m.stride_f32 = 0;
  m.stride_op = 0;
  m.meta = base + align_up(p.mat_f32) + align_up(p.mat_op) + align_up(p.mat_op2);
  return m;
}

MatRef y_ref(const Plan& p, char* ws, int slot) {
  char* base = ws + p.off_y + (size_t)slot * p.y_slot_bytes;
  MatRef m;
  m.f32 = (float*)base;
  m.op = p.prec == kFP32 ? (void*)base : (void*)(base + align_up(p.mat_f32));
  m.stride_f32 = p.y_obs_bytes / 4;
  m.stride_op = p.y_obs_bytes;
  m.meta = base + align_up(p.mat_f32) + align_up(p.mat_op) + align_up(p.mat_op2);
  return m;
}

// The X operand of a sweep (Z-job) launch: for the three-term-X^2 option the
// two-term copy, otherwise the matrix set itself.
MatRef sweep_x(MatRef m) {
  if (m.op2) m.op = m.op2;
  m.op2 = nullptr;
  return m;
}

// FP32 view of a matrix set (the masters) for the FP32 projection sweep.
MatRef as_fp32(MatRef m) {
  m.op = m.f32;
  m.stride_op = m.stride_f32 * 4;
  return m;
}

// ---------------------------------------------------------------- Lanczos (host part)

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm count).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// k-th smallest eigenvalue (0-based) by bisection.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi) + std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for the extreme eigenvalue
// theta, by two steps of inverse iteration with shift just outside the
// spectrum (T - shift I is then definite and the LDL^T solve is stable).
double last_component(const std::vector<double>& a, const std::vector<double>& b, double theta,
                      double shift_dir, double width) {
  const size_t k = a.size();
  const double sh = theta + shift_dir * 1e-10 * std::max(width, 1e-300);
  std::vector<double> x(k, 1.0), d(k), l(k), y(k);
  for (int it = 0; it < 3; ++it) {
    // LDL^T of (T - sh I), forward/back solve
    d[0] = a[0] - sh;
    for (size_t i = 1; i < k; ++i) {
      l[i] = b[i - 1] / d[i - 1];
      d[i] = a[i] - sh - l[i] * b[i - 1];
    }
    y[0] = x[0];
    for (size_t i = 1; i < k; ++i) y[i] = x[i] - l[i] * y[i - 1];
    for (size_t i = 0; i < k; ++i) y[i] /= d[i];
    for (size_t i = k - 1; i-- > 0;) y[i] -= l[i + 1] * y[i + 1];
    double nrm = 0.0;
    for (double v : y) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < k; ++i) x[i] = y[i] / nrm;
  }
  return std::fabs(x[k - 1]);
}

struct ScopedEvents {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~ScopedEvents() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Optional per-launch timing: event markers recorded on the call's stream.
struct Profiler {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  ~Profiler() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  // Records a marker and returns its index (-1 when profiling is off).
  int mark() {
    if (!on) return -1;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    if (hipEventRecord(e, s) != hipSuccess) {
      (void)hipEventDestroy(e);
      return -1;
    }
    ev.push_back(e);
    return (int)ev.size() - 1;
  }
  double ms(int a, int b) const {
    if (a < 0 || b < 0) return 0.0;
    float t = 0.f;
    return hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess ? (double)t : 0.0;
  }
};

dmpt_status decide_to_status(int code) {
  switch (code) {
    case kDecideStop: return DMPT_OK;
    case kDecideNotConverged: return DMPT_ERR_NOT_CONVERGED;
    case kDecideBounds: return DMPT_ERR_BOUNDS;
    case kDecideNonfinite: return DMPT_ERR_NONFINITE;
    default: return DMPT_ERR_DEVICE;
  }
}

// Spectral bounds into ctl (alpha, beta).  Gershgorin always runs (it also
// scans H for NaN/Inf).  Lanczos: extreme Ritz values widened by
// max(residual, 1% of the width), clipped to the Gershgorin interval.
dmpt_status compute_bounds(const Opts& o, const Plan& p, const float* H, Ctl* ctl, double* lz,
                           double2* gs, hipStream_t s) {
  DMPT_HIP(launch_gershgorin(H, o.n, gs, gershgorin_blocks(o.n), ctl, o.bounds == DMPT_BOUNDS_GERSHGORIN, s));
  if (o.bounds == DMPT_BOUNDS_GIVEN) {
    DMPT_HIP(launch_set_bounds(ctl, o.emin, o.emax, s));
    return DMPT_OK;
  }
  if (o.bounds == DMPT_BOUNDS_GERSHGORIN) return DMPT_OK;
  const int k = std::min(p.lz_steps, o.n);
  double* v = lz;
  double* vprev = lz + o.n;
  double* w = lz + 2 * o.n;
  double* ab = lz + 3 * o.n;
  DMPT_HIP(launch_lanczos_start(v, vprev, o.n, s));
  for (int j = 0; j < k; ++j) DMPT_HIP(launch_lanczos_step(H, o.n, v, vprev, w, ab, j, s));
  std::vector<double> hab(2 * k);
  double g[2];
  int nonfinite = 0;
  DMPT_HIP(hipMemcpyAsync(hab.data(), ab, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipMemcpyAsync(g, &ctl->gmin, sizeof(g), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipMemcpyAsync(&nonfinite, &ctl->nonfinite, sizeof(int), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (nonfinite) {
    DMPT_HIP(launch_set_bounds(ctl, g[0], g[1], s));
    return DMPT_OK;   // the step kernel reports DMPT_ERR_NONFINITE
  }
  // Truncate at breakdown (invariant subspace: the Ritz values are exact).
  std::vector<double> a, b;
  double scale = 0.0;
  for (int j = 0; j < k; ++j) scale = std::max(scale, std::fabs(hab[2 * j]) + std::fabs(hab[2 * j + 1]));
  int kk = k;
  for (int j = 0; j < k; ++j) {
    a.push_back(hab[2 * j]);
    if (hab[2 * j + 1] <= 1e-12 * std::max(scale, 1e-300)) { kk = j + 1; break; }
    if (j + 1 < k) b.push_back(hab[2 * j + 1]);
  }
  const double beta_last = kk < k ? 0.0 : hab[2 * k - 1];
  b.resize(a.size() > 0 ? a.size() - 1 : 0);
  const double tmin = tridiag_eig(a, b, 0);
  const double tmax = tridiag_eig(a, b, (int)a.size() - 1);
  const double width = std::max(tmax - tmin, 1e-12 * std::max(1.0, std::fabs(tmax)));
  const double rmin = beta_last * last_component(a, b, tmin, -1.0, width);
  const double rmax = beta_last * last_component(a, b, tmax, +1.0, width);
  double emin = tmin - std::max(rmin, 0.01 * width);
  double emax = tmax + std::max(rmax, 0.01 * width);
  emin = std::max(emin, g[0]);
  emax = std::min(emax, g[1]);
  if (!(emax > emin)) { emin = g[0]; emax = g[1]; }
  DMPT_HIP(launch_set_bounds(ctl, emin, emax, s));
  return DMPT_OK;
}

// Trivial occupations: nocc = 0 -> D = 0, nocc = n -> D = I; chi = 0 either way.
__global__ void k_trivial(float* d, float* chi, int n, int nobs, int full, const float* a, double* a0_part) {
  const size_t n2 = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += (size_t)gridDim.x * blockDim.x) {
    const bool dg = (e / n) == (e % n);
    if (d) d[e] = (full && dg) ? 1.0f : 0.0f;
    if (chi) for (int k = 0; k < nobs; ++k) chi[(size_t)k * n2 + e] = 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && a0_part) {
    for (int k = 0; k < nobs; ++k) {
      double t = 0.0;
      if (full) for (int i = 0; i < n; ++i) t += a[(size_t)k * n2 + (size_t)i * n + i];
      a0_part[k] = t;
    }
  }
}

// The shared driver of dmpt_sp2_density and dmpt_susceptibility.
// One solve.  reuse_x: the workspace already holds the bounds, the control
// block and every stored X_n of an earlier adjoint solve with the same H and
// options (the self-consistent loop sweeps new observables over one SP2
// recursion); only the backward sweep, projection and outputs run.
dmpt_status run(const float* H, const float* A, int nobs, float* chi, float* D, double* a0,
                const dmpt_opts* opts, dmpt_info* info, bool reuse_x = false) {
  Opts o;
  dmpt_status st = normalise(opts, &o);
  if (st != DMPT_OK) return st;
  if (!H) return fail(DMPT_ERR_ARG, "H is NULL");
  if (nobs < 0 || nobs > kMaxObs) return fail(DMPT_ERR_ARG, "nobs = %d out of range [0, %d]", nobs, kMaxObs);
  if (nobs > 0 && (!A || !chi)) return fail(DMPT_ERR_ARG, "A and chi must not be NULL");
  if (nobs == 0 && !D) return fail(DMPT_ERR_ARG, "D is NULL");
  const bool adjoint = nobs > 0 && o.sweep == DMPT_SWEEP_ADJOINT;
  Plan p;
  make_plan(o, nobs, &p);
  if (!o.ws) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", p.total);
  if (o.ws_bytes < p.total) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", o.ws_bytes, p.total);
  if (info) std::memset(info, 0, sizeof(*info));

  hipStream_t s = o.stream;
  char* ws = o.ws;
  Ctl* ctl = (Ctl*)(ws + p.off_ctl);
  double* a0_part = (double*)(ws + p.off_a0);
  ScopedEvents ev;
  DMPT_HIP(hipEventCreate(&ev.e0));
  DMPT_HIP(hipEventCreate(&ev.e1));
  DMPT_HIP(hipEventRecord(ev.e0, s));

  if (o.nocc == 0 || o.nocc == o.n) {
    const bool full = o.nocc == o.n;
    hipLaunchKernelGGL(k_trivial, dim3(256), dim3(256), 0, s, D, nobs ? chi : nullptr, o.n, nobs, full ? 1 : 0, A, a0_part);
    DMPT_HIP(hipGetLastError());
    std::vector<double> h(std::max(nobs, 1));
    if (nobs) DMPT_HIP(hipMemcpyAsync(h.data(), a0_part, sizeof(double) * nobs, hipMemcpyDeviceToHost, s));
    DMPT_HIP(hipEventRecord(ev.e1, s));
    DMPT_HIP(hipStreamSynchronize(s));
    if (a0) for (int k = 0; k < nobs; ++k) a0[k] = o.spin * h[k];
    if (info) {
      info->status = DMPT_OK;
      info->trace_d = full ? o.n : 0;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
      info->elapsed_ms = ms;
    }
    return DMPT_OK;
  }

  // Precision of the SP2 products (P-jobs) and of the sweep products
  // (Z-jobs).  When they differ the step is two launches over the same
  // control state: Z-jobs first, then P-jobs (which write the partials the
  // next step's controller reads).
  const int xprec = p.prec == kSplit32 ? kSplit3 : p.prec;
  const int yprec = p.prec == kSplit32 ? kSplit2 : p.prec;
  const bool split_launch = xprec != yprec && nobs > 0 && !adjoint;
  // launches of P-jobs only: for the three-term-X^2 option the mixed kernel,
  // whose P-jobs also write X's two-term copy (the sweep reads it)
  const int xlaunch = p.prec == kSplit32 ? kSplit32 : xprec;

  const bool refining = nobs > 0 && o.refine && !adjoint;
  // 256 x 256 sweep-product tiles (one accumulation level) when the residual
  // correction follows: the three-term-X^2 option's steps and projection, and
  // the correction's own launches
  const bool wide = refining && o.refine == 1 && split_launch;
  const int cus = persistent_grid(1 << 30);
  // job tables: [Z-jobs][P-jobs] (one combined table when the step is one launch)
  std::vector<uint32_t> jobs;
  // K-split tail tiles (runs on the wide lists): slot tables and combine lists
  std::vector<uint32_t> slots_main, cjobs_main;
  if (split_launch && wide) {
    const JobList& L = cached_wide_list(p.n_pad, nobs, true, cus);
    jobs = L.jobs;
    slots_main = L.slots;
    cjobs_main = L.cjobs;
  } else if (split_launch) {
    const std::vector<uint32_t> pj = build_jobs(p.n_pad, 0, true);
    jobs = build_jobs(p.n_pad, nobs, false);
    jobs.insert(jobs.end(), pj.begin(), pj.end());
  } else {
    jobs = build_jobs(p.n_pad, adjoint ? 0 : nobs, true);
  }
  uint32_t* d_jobs = (uint32_t*)(ws + p.off_jobs);
  DMPT_HIP(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * 4, hipMemcpyHostToDevice, s));
  const int njobs_main = (int)jobs.size();
  uint32_t* d_slots_main = wide ? (uint32_t*)(ws + p.off_split_slot) : nullptr;
  uint32_t* d_cjobs_main = wide ? (uint32_t*)(ws + p.off_cjobs) : nullptr;
  float* d_split_buf = wide ? (float*)(ws + p.off_split_buf) : nullptr;
  if (!cjobs_main.empty()) {
    DMPT_HIP(hipMemcpyAsync(d_slots_main, slots_main.data(), slots_main.size() * 4, hipMemcpyHostToDevice, s));
    DMPT_HIP(hipMemcpyAsync(d_cjobs_main, cjobs_main.data(), cjobs_main.size() * 4, hipMemcpyHostToDevice, s));
  }
  // a step launch, then the combine launch of its K-split tiles
  auto combine = [&](int prec_, const StepArgs& args, const uint32_t* cj, size_t nc) {
    return nc ? launch_step_combine(prec_, args, cj, (int)nc, s) : hipSuccess;
  };

  Profiler prof;
  prof.on = o.profile != 0;
  prof.s = s;
  if (reuse_x && !adjoint) return fail(DMPT_ERR_ARG, "reusing the recursion needs the adjoint sweep");
  const int mb0 = prof.mark();
  if (!reuse_x) {
    DMPT_HIP(launch_ctl_reset(ctl, s));
    st = compute_bounds(o, p, H, ctl, (double*)(ws + p.off_lz), (double2*)(ws + p.off_gersh), s);
    if (st != DMPT_OK) return st;
  }
  // Every step launch takes the next queue counter set (zeroed here, then
  // kept clean by the launches themselves).
  DMPT_HIP(launch_queue_reset(ctl, s));
  unsigned qseq = 0;
  auto run_step = [&](int prec_, StepArgs& args, int nj, bool wide_ = false) {
    if (nj <= 0) return hipSuccess;   // no launch: the counter sets stay in step
    step_queue_sets(ctl, qseq++, &args);
    return launch_step(prec_, args, nj, s, wide_);
  };

  // Slot of X_n: forward sweep 2 ping-pong slots; adjoint slot n, or with
  // checkpoints the checkpoint slot / a working slot (forward run) and the
  // recomputation ring (backward sweep).
  const int k_ck = p.ckpt;
  auto is_ckpt = [&](int n) { return (n - 1) % k_ck == 0; };
  auto xslot = [&](int n) {
    if (!adjoint) return n & 1;
    if (!k_ck) return n;
    return is_ckpt(n) ? 2 + (n - 1) / k_ck : (n & 1);
  };
  auto xslot_bwd = [&](int n) {
    if (!k_ck) return n;
    return is_ckpt(n) ? 2 + (n - 1) / k_ck : 2 + p.nckpt + ((n - 1) % k_ck - 1);
  };
  Part* part[2] = {(Part*)(ws + p.off_part[0]), (Part*)(ws + p.off_part[1])};
  // X_1 (and Y_1 = beta A for the forward sweep) into slot of step 1
  if (!reuse_x) {
    DMPT_HIP(launch_init(p.prec, p.tile, H, A, o.n, p.n_pad, adjoint ? 0 : nobs, nullptr, 0,
                         x_ref(p, ws, xslot(1)), y_ref(p, ws, 1), 0.0, part[1], ctl, s));
    // FP16 split: the Y copies are written once their norms are known
    if (p.prec == kSplitH && !adjoint && nobs > 0) DMPT_HIP(launch_resplit(p.prec, y_ref(p, ws, 1), p.n_pad, nobs, s));
  }
  const int mb1 = prof.mark();
  std::vector<std::pair<int, int>> step_marks;

  // SP2 steps: chunks of launches, host polls the done flag between chunks.
  // Launch n decides sigma_n from X_n's traces and applies the stopping test
  // to X_{n-1} (its idempotency error is a by-product of launch n-1), so the
  // stop is seen one launch late; that launch returns before writing and
  // X_{n-1}, Y_{n-1} are still in their slots.
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = o.n;
  a.n_pad = p.n_pad;
  a.ntile = p.ntile;
  a.max_iter = o.max_iter;
  a.min_iter = o.min_iter;
  a.nocc = o.nocc;
  a.idem_tol = o.idem_tol;
  a.decide = 1;
  a.unit = sp2_unit(xprec);   // both launches of a split step take the same decision
  // sweep stop (opts.sweep_tol, with the residual correction only)
  a.ytol2 = refining && o.sweep_tol > 0.0 ? o.sweep_tol * o.sweep_tol : 0.0;
  a.write_split = 1;
  a.flush = flush_interval(xprec, p.n_pad);
  a.jobs = d_jobs;
  a.ctl = ctl;
  a.split_slot = d_slots_main;
  a.split_buf = d_split_buf;
  if (refining) {   // every X_{n+1} also as plain BF16 for the correction sweep
    a.hist = ws + p.off_rf_hist;
    a.hist_stride = (size_t)p.n_pad * p.n_pad * 2;
  }
  const int njobs_step = adjoint ? p.nparts_step : njobs_main;
  const uint32_t* step_jobs = adjoint ? d_jobs + 0 : d_jobs;
  // adjoint X-only run uses the P-jobs only (the table holds no Z-jobs then)
  int done = reuse_x ? 1 : 0;
  int launched = 0;
  for (int n = 1; n <= o.max_iter + 2 && !done;) {
    const int end = std::min(o.max_iter + 2, n + kChunk - 1);
    for (; n <= end; ++n) {
      a.step = n;
      a.x_in = x_ref(p, ws, xslot(n));
      a.x_out = x_ref(p, ws, xslot(n + 1));
      a.y_in = y_ref(p, ws, n & 1);
      a.y_out = y_ref(p, ws, (n + 1) & 1);
      a.part_in = part[n & 1];
      a.part_out = part[(n + 1) & 1];
      // X_1's partials come from its initialisation; later ones from the
      // previous step launch, and 3 more per K-split tile from its combine
      a.nparts = n == 1 ? p.nb64 * p.nb64 : p.nparts_step + 3 * (int)cjobs_main.size();
      const int ma = prof.mark();
      if (split_launch) {
        // one mixed launch: Z-jobs on two-term copies, then P-jobs on
        // three-term ones (which also write X_{n+1}'s two-term copy)
        a.jobs = d_jobs;
        a.flush = flush_interval(xprec, p.n_pad);
        a.flush_z = flush_interval(yprec, p.n_pad);
        DMPT_HIP(run_step(kSplit32, a, njobs_main, wide));
        DMPT_HIP(combine(kSplit32, a, d_cjobs_main, cjobs_main.size()));
      } else {
        a.jobs = step_jobs;
        DMPT_HIP(run_step(xlaunch, a, njobs_step));
      }
      step_marks.emplace_back(ma, prof.mark());
      ++launched;
    }
    DMPT_HIP(hipMemcpyAsync(&done, &ctl->done, sizeof(int), hipMemcpyDeviceToHost, s));
    DMPT_HIP(hipStreamSynchronize(s));
  }
  Ctl hctl;
  DMPT_HIP(hipMemcpyAsync(&hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (!hctl.done) return fail(DMPT_ERR_DEVICE, "step loop ended without a decision");
  const int m = hctl.m;
  st = decide_to_status(hctl.code);
  const int xfin = xslot(m + 1);
  int yfin = (m + 1) & 1;
  // The sweep stopped at Y_k (opts.sweep_tol): later launches left it in its slot.
  const int ystop = a.ytol2 > 0.0 && st == DMPT_OK ? hctl.ystop : 0;
  if (ystop > 0) yfin = ystop & 1;

  const int mp0 = prof.mark();
  if (nobs > 0 && st == DMPT_OK && adjoint) {
    // Eq. DM2: Y_M = A; for n = M..1, Y_{n-1} from Y_n with X_n, sigma_n; chi = beta Y_0.
    DMPT_HIP(launch_init(p.prec, p.tile, nullptr, A, o.n, p.n_pad, -nobs, nullptr, 0,
                         x_ref(p, ws, 0), y_ref(p, ws, 0), 1.0, nullptr, ctl, s));
    if (p.prec == kSplitH) DMPT_HIP(launch_resplit(p.prec, y_ref(p, ws, 0), p.n_pad, nobs, s));
    const std::vector<uint32_t> zjobs = build_jobs(p.n_pad, nobs, false);
    uint32_t* d_zjobs = d_jobs + p.nparts_step;
    DMPT_HIP(hipMemcpyAsync(d_zjobs, zjobs.data(), zjobs.size() * 4, hipMemcpyHostToDevice, s));
    StepArgs b = a;
    b.decide = 0;
    b.flush = flush_interval(yprec, p.n_pad);
    b.sigma_src = ctl->rec;
    b.jobs = d_zjobs;
    // recomputation launches: P-jobs with the recorded sigma_n (same kernel
    // and inputs as the forward run, so X_n is reproduced bit for bit)
    StepArgs r = a;
    r.decide = 0;
    r.sigma_src = ctl->rec;
    r.jobs = d_jobs;
    r.part_in = part[0];
    r.part_out = part[1];
    r.nparts = p.nparts_step;
    int ys = 0;
    for (int n1 = m; n1 >= 1;) {
      const int n0 = k_ck ? ((n1 - 1) / k_ck) * k_ck + 1 : 1;   // first step of the segment
      for (int n = n0; k_ck && n < n1; ++n) {
        r.step = n;
        r.x_in = x_ref(p, ws, xslot_bwd(n));
        r.x_out = x_ref(p, ws, xslot_bwd(n + 1));
        DMPT_HIP(run_step(xlaunch, r, p.nparts_step));
      }
      for (int n = n1; n >= n0; --n) {
        b.step = n;
        b.x_in = sweep_x(x_ref(p, ws, xslot_bwd(n)));
        b.y_in = y_ref(p, ws, ys);
        b.y_out = y_ref(p, ws, ys ^ 1);
        DMPT_HIP(run_step(yprec, b, (int)zjobs.size()));
        ys ^= 1;
      }
      n1 = n0 - 1;
    }
    yfin = ys;
  }

  int njobs_proj = 0;
  // the projection's list (also the correction's) and its K-split tail
  std::vector<uint32_t> slots_proj, cjobs_proj;
  uint32_t* d_slots_proj = wide ? (uint32_t*)(ws + p.off_split_slot_proj) : nullptr;
  uint32_t* d_cjobs_proj = wide ? (uint32_t*)(ws + p.off_cjobs_proj) : nullptr;
  if (nobs > 0 && o.project && st == DMPT_OK) {
    // Occupied-virtual projection: two sweep steps with X frozen at D
    // (sigma = +1 then -1) multiply the eigenbasis blocks of Y by
    // (f_i + f_j)(2 - f_i - f_j): 1 on occupied-virtual pairs, 0 elsewhere.
    // They run in the precision of the sweep products (FP32 for plain BF16),
    // on the operand copies of D and Y the last step wrote.
    // project = 2 (three-term-X^2 option): Y is projected in the three-term
    // split, from a three-term copy of Y and D's three-term copy, on the
    // regular tiles (in the main list's buffer, free once the steps are done)
    const bool proj3 = o.project == 2;
    const int pprec = proj3 ? kSplit3 : p.prec == kBF16 ? kFP32 : yprec;
    // (the list also serves the launches of the residual correction)
    std::vector<uint32_t> pjobs;
    if (wide) {
      const JobList& L = cached_wide_list(p.n_pad, nobs, false, cus);
      pjobs = L.jobs;
      slots_proj = L.slots;
      cjobs_proj = L.cjobs;
    } else {
      pjobs = build_jobs(p.n_pad, nobs, false);
    }
    uint32_t* d_pjobs = (uint32_t*)(ws + p.off_jobs_proj);
    DMPT_HIP(hipMemcpyAsync(d_pjobs, pjobs.data(), pjobs.size() * 4, hipMemcpyHostToDevice, s));
    if (!cjobs_proj.empty()) {
      DMPT_HIP(hipMemcpyAsync(d_slots_proj, slots_proj.data(), slots_proj.size() * 4, hipMemcpyHostToDevice, s));
      DMPT_HIP(hipMemcpyAsync(d_cjobs_proj, cjobs_proj.data(), cjobs_proj.size() * 4, hipMemcpyHostToDevice, s));
    }
    njobs_proj = (int)pjobs.size();
    StepArgs b;
    std::memset(&b, 0, sizeof(b));
    b.n = o.n;
    b.n_pad = p.n_pad;
    b.ntile = p.ntile;
    b.decide = 0;
    b.flush = flush_interval(pprec, p.n_pad);
    b.jobs = d_pjobs;
    b.ctl = ctl;
    b.split_slot = d_slots_proj;
    b.split_buf = d_split_buf;
    auto view = [&](MatRef m) { return pprec == kFP32 ? as_fp32(m) : m; };
    b.x_in = pprec == kFP32 ? as_fp32(x_ref(p, ws, xfin)) : proj3 ? x_ref(p, ws, xfin) : sweep_x(x_ref(p, ws, xfin));
    std::vector<uint32_t> rjobs;
    if (proj3) {
      rjobs = build_jobs(p.n_pad, nobs, false);
      DMPT_HIP(hipMemcpyAsync(d_jobs, rjobs.data(), rjobs.size() * 4, hipMemcpyHostToDevice, s));
      b.jobs = d_jobs;
      b.split_slot = nullptr;
      b.split_buf = nullptr;
      const MatRef y0 = y_ref(p, ws, yfin);   // its operand area holds the three-term copy
      for (int k = 0; k < nobs; ++k)
        DMPT_HIP(launch_copy_src(kSplit3, y0.f32 + (size_t)k * y0.stride_f32, p.n_pad,
                                 (char*)y0.op + (size_t)k * y0.stride_op, p.n_pad, 0, s));
    }
    // The launch after the last step (it ran before the stop was seen, since
    // the stopping test needs its idempotency error) formed Z = D Y + Y D from
    // D = X_{m+1} and Y_{m+1}, the product of the first projection step.
    // When the projection runs in the precision of the sweep products, that
    // launch replaces the first projection step: with sigma = +1 its Y_{m+2} = Z is the product the
    // step would form, in the same precision (bit for bit unless the two
    // launches tile it differently, as the wide/regular mix of a corrected
    // run may); with sigma = -1, Y_{m+2} = 2 Y_{m+1} - Z and one elementwise pass
    // recovers Z = 2 Y_{m+1} - Y_{m+2} (one more FP32 rounding), with its
    // operand copy at the scale the step would use (Y_{m+2}'s own: both come
    // from Y_{m+1}) and fresh norm partials for the second step.
    const int sig_next = hctl.rec[m + 1].sigma;
    const bool reuse_first = !adjoint && pprec == yprec && hctl.code == kDecideStop && ystop == 0 &&
                             (sig_next == 1 || sig_next == -1);
    int q0 = 0;
    if (reuse_first) {
      if (sig_next == -1)
        DMPT_HIP(launch_reflect(pprec, y_ref(p, ws, yfin), y_ref(p, ws, yfin ^ 1), p.n_pad, nobs, s));
      yfin ^= 1;
      q0 = 1;
    }
    for (int q = q0; q < 2; ++q) {
      b.fixed_sigma = q == 0 ? 1 : -1;
      b.write_split = q == 0 && pprec != kFP32;   // the second step reads it
      b.y_in = view(y_ref(p, ws, yfin));
      b.y_out = view(y_ref(p, ws, yfin ^ 1));
      if (proj3) {
        DMPT_HIP(run_step(pprec, b, (int)rjobs.size()));
      } else {
        DMPT_HIP(run_step(pprec, b, (int)pjobs.size(), wide));
        DMPT_HIP(combine(pprec, b, d_cjobs_proj, cjobs_proj.size()));
      }
      yfin ^= 1;
    }
  }

  const int mp1 = prof.mark();
  int mcorr = 0;   // sweep steps of the residual correction
  if (nobs > 0 && o.refine && st == DMPT_OK) {
    // Residual correction of chi' (opts.refine; Appendix, proof of Eq.
    // Equivalence).  The exact chi' = L o A on the eigenbasis of H solves
    // [H, chi'] = [D, A] with no occupied-occupied / virtual-virtual blocks,
    // so for the projected sweep result Y the error E = chi' - Y satisfies
    // (lambda_i - lambda_j) E_ij = R_ij on the occupied-virtual pairs,
    // R = [D, A] - [H, Y].  The sweep of B = [D, R] = (f_i - f_j) R_ij applies
    // L again: L o B = R_ij / (lambda_i - lambda_j) = E_ij there and 0
    // elsewhere.  R needs FP32-accurate products (it is a small difference of
    // large terms); the sweep of B only needs accuracy relative to the small
    // correction, so it runs on plain BF16 products.
    //   R = W - W^T, W = D A + Y H (A, H symmetric: NT products)
    //   Y_1 = beta B = -beta (R D^T + D R^T): a sweep step with Y := R, X := D
    //   delta = Y_{m+1} of the BF16 recursion X_1 = alpha I + beta H, sigma_n as recorded
    //   Y <- Y + P(delta), P the two-step occupied-virtual projection with D
    const size_t np2 = (size_t)p.n_pad * p.n_pad;
    const int rp = p.rprec;
    const MatRef xf = x_ref(p, ws, xfin);
    const MatRef yf = y_ref(p, ws, yfin);
    char* cbase = ws + p.off_rf_copy;
    auto cpy = [&](int q) { return (void*)(cbase + (size_t)q * p.rf_copy_bytes); };   // 0 D, 1 H, 2+k A_k, 2+nobs+k Y_k
    float* v1 = (float*)(ws + p.off_rf_v);
    float* v2 = v1 + np2;
    // operand copies (kSplitH: power-of-two scales from entry bounds: |D_ij| <= 1,
    // |H_ij| <= max(|emin|, |emax|), |M_ij| <= ||M||_F for A_k and Y_k)
    std::vector<int> ex(2 + 2 * nobs, 0);
    if (rp == kSplitH) {
      double* np_ = (double*)(ws + p.off_rf_norm);
      for (int k = 0; k < nobs; ++k) {
        DMPT_HIP(launch_norm2(A + (size_t)k * o.n * o.n, (size_t)o.n * o.n, np_ + (size_t)(2 + k) * kNormBlocks, s));
        DMPT_HIP(launch_norm2(yf.f32 + (size_t)k * yf.stride_f32, np2, np_ + (size_t)(2 + nobs + k) * kNormBlocks, s));
      }
      std::vector<double> hn((size_t)(2 + 2 * nobs) * kNormBlocks, 0.0);
      DMPT_HIP(hipMemcpyAsync(hn.data() + 2 * kNormBlocks, np_ + 2 * kNormBlocks,
                              sizeof(double) * kNormBlocks * 2 * nobs, hipMemcpyDeviceToHost, s));
      DMPT_HIP(hipStreamSynchronize(s));
      auto expo = [](double bound) {
        if (!(bound > 0.0) || !std::isfinite(bound)) return 0;
        return std::max(-100, std::min(100, (int)std::floor(std::log2(32768.0 / bound))));
      };
      ex[0] = kXScaleExp;
      ex[1] = expo(std::max(std::fabs(hctl.emin), std::fabs(hctl.emax)));
      for (int q = 2; q < 2 + 2 * nobs; ++q) {
        double t = 0.0;
        for (int b = 0; b < kNormBlocks; ++b) t += hn[(size_t)q * kNormBlocks + b];
        ex[q] = expo(std::sqrt(t));
      }
    }
    // FP32 residual products read padded FP32 copies of H and A_k; D and Y
    // are their own masters
    auto src_of = [&](int q) -> const float* {
      if (q == 0) return xf.f32;
      if (q == 1) return H;
      if (q < 2 + nobs) return A + (size_t)(q - 2) * o.n * o.n;
      return yf.f32 + (size_t)(q - 2 - nobs) * yf.stride_f32;
    };
    auto nsrc_of = [&](int q) { return (q == 0 || q >= 2 + nobs) ? p.n_pad : o.n; };
    // D's own operand copy is already in the residual's format when the X
    // products run in it (written by the step that formed D, from the same
    // FP32 values and at the same scale): no second copy
    const bool d_has_copy = (rp == kSplit3 && (p.prec == kSplit3 || p.prec == kSplit32)) ||
                            (rp == kSplitH && p.prec == kSplitH);
    auto opnd = [&](int q) -> const void* {
      if (rp == kFP32 && (q == 0 || q >= 2 + nobs)) return src_of(q);
      if (q == 0 && d_has_copy) return xf.op;
      return cpy(q);
    };
    for (int q = 0; q < 2 + 2 * nobs; ++q) {
      if (q == 0 && d_has_copy) continue;
      if (rp == kFP32) {
        if (q == 1 || (q >= 2 && q < 2 + nobs)) DMPT_HIP(launch_pad(src_of(q), o.n, p.n_pad, (float*)cpy(q), 0, s));
      } else {
        DMPT_HIP(launch_copy_src(rp, src_of(q), nsrc_of(q), cpy(q), p.n_pad, ex[q], s));
      }
    }
    const int flr = flush_interval(rp, p.n_pad);
    char* rbase = ws + p.off_rf_r;
    for (int k = 0; k < nobs; ++k) {
      DMPT_HIP(launch_gemm_op(rp, opnd(0), opnd(2 + k), v1, p.n_pad, std::ldexp(1.0f, -(ex[0] + ex[2 + k])), flr, 0, s));
      DMPT_HIP(launch_gemm_op(rp, opnd(2 + nobs + k), opnd(1), v2, p.n_pad,
                              std::ldexp(1.0f, -(ex[2 + nobs + k] + ex[1])), flr, 0, s));
      DMPT_HIP(launch_antisym_bf16(v1, v2, p.n_pad, rbase + (size_t)k * np2 * 2, s));
    }
    // plain BF16 copies of the X_n: slot n of the history (X_1 from the
    // initialisation below, X_2 .. X_{m+1} = D written by the steps)
    char* hist = ws + p.off_rf_hist;
    const size_t hstride = np2 * 2;
    const int flb = flush_interval(kBF16, p.n_pad);
    MatRef dref;
    dref.f32 = xf.f32;
    dref.op = hist + (size_t)(m + 1) * hstride;
    dref.meta = xf.meta;
    dref.stride_f32 = 0;
    dref.stride_op = 0;
    MatRef rref;
    rref.f32 = xf.f32;          // not read: sigma = +1 Z-jobs use only the operand copies
    rref.op = rbase;
    rref.meta = xf.meta;
    rref.stride_f32 = 0;
    rref.stride_op = np2 * 2;
    auto bx = [&](int q) { return bf16_ref(p, ws, p.off_rf_x, q, 1); };
    auto by = [&](int q) { return bf16_ref(p, ws, p.off_rf_y, q, nobs); };
    const uint32_t* d_pjobs = (const uint32_t*)(ws + p.off_jobs_proj);   // Z-jobs of every observable
    const int nzj = njobs_proj;
    StepArgs b;
    std::memset(&b, 0, sizeof(b));
    b.n = o.n;
    b.n_pad = p.n_pad;
    b.ntile = p.ntile;
    b.decide = 0;
    b.flush = flb;
    b.ctl = ctl;
    b.fixed_sigma = 1;
    b.write_split = 1;
    b.jobs = d_pjobs;
    b.split_slot = d_slots_proj;
    b.split_buf = d_split_buf;
    b.x_in = dref;
    b.y_in = rref;
    b.y_out = by(1);
    b.oscale = (float)(-hctl.beta);
    DMPT_HIP(run_step(kBF16, b, nzj, wide));
    DMPT_HIP(combine(kBF16, b, d_cjobs_proj, cjobs_proj.size()));
    // X_1 = alpha I + beta H in plain BF16 (its copy lands in history slot 1)
    MatRef x1 = bx(0);
    x1.op = hist + hstride;
    DMPT_HIP(launch_init(kBF16, p.tile, H, nullptr, o.n, p.n_pad, 0, nullptr, 0, x1, by(1), 0.0, part[1], ctl, s));
    // the sweep of B: Z-jobs only, X_n from the history, sigma_n as recorded;
    // with opts.sweep_tol it stops after the first X_n within sqrt(sweep_tol)
    // of idempotency (the correction only needs accuracy relative to itself)
    mcorr = m;
    if (o.sweep_tol > 0.0)
      for (int q = 1; q <= m; ++q)
        if (hctl.rec[q].eps <= o.sweep_tol) {
          mcorr = q;
          break;
        }
    StepArgs r = b;
    r.sigma_src = ctl->rec;
    r.oscale = 1.0f;
    r.write_split = 1;
    for (int n = 1; n <= mcorr; ++n) {
      r.step = n;
      r.x_in = x1;
      r.x_in.op = hist + (size_t)n * hstride;
      r.y_in = by(n & 1);
      r.y_out = by((n + 1) & 1);
      DMPT_HIP(run_step(kBF16, r, nzj, wide));
      DMPT_HIP(combine(kBF16, r, d_cjobs_proj, cjobs_proj.size()));
    }
    // projection of delta with D, then Y += P(delta).  project = 2: delta is
    // copied to the two-term split and projected with D's two-term copy (D's
    // BF16 copy spans an occupied subspace turned by about 2^-8 against H's,
    // and delta from the BF16 sweep is occupied-virtual in that one); the
    // free Y slot holds the copies (its operand area and the one after it)
    int yd = (mcorr + 1) & 1;
    const bool proj3 = o.project == 2;
    const MatRef yfree = y_ref(p, ws, yfin ^ 1);
    if (proj3) {
      const MatRef dd = by(yd);
      for (int k = 0; k < nobs; ++k)
        DMPT_HIP(launch_copy_src(kSplit2, dd.f32 + (size_t)k * dd.stride_f32, p.n_pad,
                                 (char*)yfree.op + (size_t)k * yfree.stride_op, p.n_pad, 0, s));
      b.flush = flush_interval(kSplit2, p.n_pad);
      b.x_in = sweep_x(xf);
    }
    for (int q = 0; q < 2; ++q) {
      b.fixed_sigma = q == 0 ? 1 : -1;
      b.write_split = q == 0;
      b.oscale = 1.0f;
      b.y_in = by(yd);
      b.y_out = by(yd ^ 1);
      if (proj3) {
        char* copy2 = (char*)yfree.op + align_up(p.mat_op);   // step 1's output copy
        b.y_in.op = q == 0 ? yfree.op : (void*)copy2;
        b.y_in.stride_op = yfree.stride_op;
        b.y_in.meta = yfree.meta;
        b.y_out.op = copy2;
        b.y_out.stride_op = yfree.stride_op;
        b.y_out.meta = yfree.meta;
        DMPT_HIP(run_step(kSplit2, b, nzj, wide));
        DMPT_HIP(combine(kSplit2, b, d_cjobs_proj, cjobs_proj.size()));
      } else {
        DMPT_HIP(run_step(kBF16, b, nzj, wide));
        DMPT_HIP(combine(kBF16, b, d_cjobs_proj, cjobs_proj.size()));
      }
      yd ^= 1;
    }
    const MatRef dl = by(yd);
    DMPT_HIP(launch_add_into(yf.f32, yf.stride_f32, dl.f32, dl.stride_f32, p.n_pad, nobs, s));
  }
  const int mr1 = prof.mark();
  // outputs
  const MatRef xf = x_ref(p, ws, xfin);
  const MatRef yf = y_ref(p, ws, yfin);
  DMPT_HIP(launch_output(xf.f32, nobs ? yf.f32 : nullptr, yf.stride_f32, A, o.n, p.n_pad, nobs, D,
                         nobs ? chi : nullptr, o.spin, adjoint ? 1 : 0, nullptr, 0, 0, a0_part, ctl, s));
  const int mo1 = prof.mark();
  std::vector<double> hpart((size_t)kOutBlocks * std::max(nobs, 1));
  if (nobs) DMPT_HIP(hipMemcpyAsync(hpart.data(), a0_part, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipEventRecord(ev.e1, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (a0)
    for (int k = 0; k < nobs; ++k) {
      double t = 0.0;
      for (int b = 0; b < kOutBlocks; ++b) t += hpart[(size_t)k * kOutBlocks + b];
      a0[k] = o.spin * t;
    }
  if (info) {
    info->m = m;
    info->status = st;
    info->emin = hctl.emin;
    info->emax = hctl.emax;
    info->beta = hctl.beta;
    for (int q = 1; q <= m + 1 && q <= DMPT_MAX_STEPS + 1; ++q) {
      info->trace_x[q - 1] = hctl.rec[q].tr;
      info->sqnorm_x[q - 1] = hctl.rec[q].sq;
      info->idem_x[q - 1] = hctl.rec[q].eps;
      info->sigma[q - 1] = (int8_t)hctl.rec[q].sigma;   // q = m + 1: the launch after the last step (0 if it did not run)
    }
    info->trace_d = hctl.rec[m + 1].tr;
    info->idem_err = hctl.rec[m + 1].eps;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
    info->elapsed_ms = ms;
    info->step_launches = launched;
    info->tile = p.tile;
    info->sweep_steps = nobs > 0 && !adjoint ? (ystop > 0 ? ystop - 1 : m) : 0;
    info->correction_steps = mcorr;
    info->split_tiles = (int32_t)cjobs_main.size();
    info->split_tiles_sweep = (int32_t)cjobs_proj.size();
    if (prof.on) {
      info->bounds_ms = prof.ms(mb0, mb1);
      double t = 0.0;
      for (int q = 0; q < (int)step_marks.size() && q < m; ++q) t += prof.ms(step_marks[q].first, step_marks[q].second);
      info->step_ms = t;
      info->project_ms = prof.ms(mp0, mp1);
      info->refine_ms = prof.ms(mp1, mr1);
      info->output_ms = prof.ms(mr1, mo1);
    }
  }
  if (st != DMPT_OK) {
    const char* why = st == DMPT_ERR_NOT_CONVERGED ? "SP2 did not converge (step limit or no gap at nocc)"
                    : st == DMPT_ERR_BOUNDS ? "spectral bounds do not enclose the spectrum of H"
                    : st == DMPT_ERR_NONFINITE ? "H or A contains NaN/Inf" : "device error";
    return fail(st, "%s (after %d steps)", why, m);
  }
  return DMPT_OK;
}

}  // namespace
}  // namespace dmpt

namespace dmpt {

// Responses are formed in groups of up to kRespObs observables x kRespPert
// perturbations (one pass over the group's chi and H1 per group).
constexpr int kRespObs = 8, kRespPert = 64, kRespMax = 1 << 20;

dmpt_status report_error(dmpt_status st, const char* msg) { return fail(st, "%s", msg); }

size_t response_workspace_bytes(int32_t nobs, int32_t npert, int32_t n) {
  if (nobs < 1 || npert < 1 || (int64_t)nobs * npert > kRespMax || n < 1 || n > 65536) {
    fail(DMPT_ERR_ARG, "response sizes out of range (nobs, npert >= 1, nobs * npert <= %d, 1 <= n <= 65536)",
         kRespMax);
    return 0;
  }
  const size_t n2 = (size_t)n * n;
  const int ko = std::min(nobs, kRespObs), kp = std::min(npert, kRespPert);
  return align_up((size_t)response_blocks(n2) * ko * kp * sizeof(double)) +
         align_up((size_t)nobs * npert * sizeof(double));
}

dmpt_status response_run(const float* chi, int32_t nobs, const float* H1, int32_t npert, int32_t n,
                         double* out, void* stream, void* workspace, size_t workspace_bytes) {
  if (!chi || !H1 || !out) return fail(DMPT_ERR_ARG, "chi, H1 and out must not be NULL");
  const size_t need = response_workspace_bytes(nobs, npert, n);
  if (need == 0) return DMPT_ERR_ARG;   // message set by response_workspace_bytes
  if (!workspace) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (workspace_bytes < need) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", workspace_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  const size_t n2 = (size_t)n * n;
  const int nblk = response_blocks(n2);
  const int ko = std::min(nobs, kRespObs), kp = std::min(npert, kRespPert);
  double* part = (double*)workspace;
  double* outd = (double*)((char*)workspace + align_up((size_t)nblk * ko * kp * sizeof(double)));
  for (int k0 = 0; k0 < nobs; k0 += kRespObs)
    for (int p0 = 0; p0 < npert; p0 += kRespPert) {
      const int kc = std::min(kRespObs, nobs - k0), pc = std::min(kRespPert, npert - p0);
      DMPT_HIP(launch_response(chi + (size_t)k0 * n2, kc, H1 + (size_t)p0 * n2, pc, n2, part, nblk,
                               outd + (size_t)k0 * npert + p0, npert, s));
    }
  DMPT_HIP(hipMemcpyAsync(out, outd, sizeof(double) * nobs * npert, hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

}  // namespace dmpt

using namespace dmpt;

extern "C" {

int32_t dmpt_abi_version(void) { return DMPT_ABI_VERSION; }

void dmpt_opts_default(dmpt_opts* o, int32_t n, int32_t nocc) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n = n;
  o->nocc = nocc;
  o->precision = DMPT_FP32;
  o->bounds = DMPT_BOUNDS_LANCZOS;
  o->lanczos_steps = 32;
  o->max_iter = 100;
  o->min_iter = 10;
  o->sweep = DMPT_SWEEP_FORWARD;
  o->project = 1;
  o->profile = 0;
  o->spin = 2.0;
}

size_t dmpt_workspace_bytes(const dmpt_opts* opts, int32_t nobs) {
  Opts o;
  if (normalise(opts, &o) != DMPT_OK || nobs < 0 || nobs > kMaxObs) return 0;
  Plan p;
  make_plan(o, nobs, &p);
  return p.total;
}

dmpt_status dmpt_sp2_density(const float* H, float* D, const dmpt_opts* opts, dmpt_info* info) {
  return run(H, nullptr, 0, nullptr, D, nullptr, opts, info);
}

dmpt_status dmpt_susceptibility(const float* H, const float* A, int32_t nobs, float* chi, float* D,
                                double* a0, const dmpt_opts* opts, dmpt_info* info) {
  if (nobs < 1) return fail(DMPT_ERR_ARG, "nobs must be >= 1");
  return run(H, A, nobs, chi, D, a0, opts, info);
}

// ---------------------------------------------------------------- non-orthonormal basis

// Workspace of dmpt_susceptibility_nonorth: the orthonormal problem's
// workspace, then four n_pad x n_pad FP32 matrices (Z, Z^T, a product and a
// padded operand/result) and n x n FP32 matrices for H_perp, D_perp and
// nobs each of A_perp and chi_perp.
struct NonorthWS {
  size_t run, zp, ztp, tp, up, hperp, dperp, aperp, cperp, total;
};

static NonorthWS nonorth_ws(size_t run_bytes, int n, int n_pad, int nobs) {
  NonorthWS w;
  const size_t pad2 = (size_t)n_pad * n_pad * 4, n2 = (size_t)n * n * 4;
  size_t off = align_up(run_bytes);
  w.run = run_bytes;
  w.zp = off; off = align_up(off + pad2);
  w.ztp = off; off = align_up(off + pad2);
  w.tp = off; off = align_up(off + pad2);
  w.up = off; off = align_up(off + pad2);
  w.hperp = off; off = align_up(off + n2);
  w.dperp = off; off = align_up(off + n2);
  w.aperp = off; off = align_up(off + n2 * nobs);
  w.cperp = off; off = align_up(off + n2 * nobs);
  w.total = off;
  return w;
}

static dmpt_status nonorth_check(const dmpt_opts* opts, int nobs, Opts* o, Plan* p) {
  dmpt_status st = normalise(opts, o);
  if (st != DMPT_OK) return st;
  if (nobs < 1 || nobs > kMaxObs) return fail(DMPT_ERR_ARG, "nobs = %d out of range [1, %d]", nobs, kMaxObs);
  make_plan(*o, nobs, p);
  return DMPT_OK;
}

size_t dmpt_nonorth_workspace_bytes(const dmpt_opts* opts, int32_t nobs) {
  Opts o;
  Plan p;
  if (nonorth_check(opts, nobs, &o, &p) != DMPT_OK) return 0;
  return nonorth_ws(p.total, o.n, p.n_pad, nobs).total;
}

dmpt_status dmpt_susceptibility_nonorth(const float* H, const float* Z, const float* A, int32_t nobs,
                                        float* chi_perp, float* chi_ao, float* D, double* a0,
                                        const dmpt_opts* opts, dmpt_info* info) {
  Opts o;
  Plan p;
  dmpt_status st = nonorth_check(opts, nobs, &o, &p);
  if (st != DMPT_OK) return st;
  if (!H || !Z || !A) return fail(DMPT_ERR_ARG, "H, Z and A must not be NULL");
  const int n = o.n, np = p.n_pad;
  const NonorthWS w = nonorth_ws(p.total, n, np, nobs);
  if (!o.ws) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", w.total);
  if (o.ws_bytes < w.total) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", o.ws_bytes, w.total);
  hipStream_t s = o.stream;
  char* ws = o.ws;
  float* zp = (float*)(ws + w.zp);
  float* ztp = (float*)(ws + w.ztp);
  float* tp = (float*)(ws + w.tp);
  float* up = (float*)(ws + w.up);
  float* hperp = (float*)(ws + w.hperp);
  float* dperp = (float*)(ws + w.dperp);
  float* aperp = (float*)(ws + w.aperp);
  float* cperp = chi_perp ? chi_perp : (float*)(ws + w.cperp);
  const size_t n2 = (size_t)n * n;
  const int fl = flush_interval(kFP32, np);
  // M_perp = Z^T M Z for symmetric M: T = Z^T M^T = Z^T M, then Z^T T^T = Z^T M Z
  auto to_perp = [&](const float* m, float* out) -> dmpt_status {
    DMPT_HIP(launch_pad(m, n, np, up, 0, s));
    DMPT_HIP(launch_gemm_nt(ztp, up, tp, np, 1.0f, fl, s));
    DMPT_HIP(launch_gemm_nt(ztp, tp, up, np, 1.0f, fl, s));
    DMPT_HIP(launch_copy_out(up, n, np, out, s));
    return DMPT_OK;
  };
  // M = Z M_perp Z^T for symmetric M_perp: T = Z M_perp^T = Z M_perp, then T Z^T
  auto from_perp = [&](const float* m, float* out) -> dmpt_status {
    DMPT_HIP(launch_pad(m, n, np, up, 0, s));
    DMPT_HIP(launch_gemm_nt(zp, up, tp, np, 1.0f, fl, s));
    DMPT_HIP(launch_gemm_nt(tp, zp, up, np, 1.0f, fl, s));
    DMPT_HIP(launch_copy_out(up, n, np, out, s));
    return DMPT_OK;
  };
  DMPT_HIP(launch_pad(Z, n, np, zp, 0, s));
  DMPT_HIP(launch_pad(Z, n, np, ztp, 1, s));
  if ((st = to_perp(H, hperp)) != DMPT_OK) return st;
  for (int k = 0; k < nobs; ++k)
    if ((st = to_perp(A + k * n2, aperp + k * n2)) != DMPT_OK) return st;
  dmpt_opts o2 = *opts;
  o2.workspace = ws;
  o2.workspace_bytes = w.run;
  // the orthonormal problem: D_perp, chi_perp and a0 = s Tr[A_perp D_perp] = s Tr[A D]
  const dmpt_status rs = run(hperp, aperp, nobs, cperp, dperp, a0, &o2, info);
  if (rs != DMPT_OK && rs != DMPT_ERR_NOT_CONVERGED) return rs;
  if (D && (st = from_perp(dperp, D)) != DMPT_OK) return st;
  if (chi_ao)
    for (int k = 0; k < nobs; ++k)
      if ((st = from_perp(cperp + k * n2, chi_ao + k * n2)) != DMPT_OK) return st;
  DMPT_HIP(hipStreamSynchronize(s));
  return rs;
}

// ---------------------------------------------------------------- finite temperature

// Workspace of dmpt_susceptibility_fermi: the bounds part of the plan of an
// SP2 solve (control block, Lanczos and Gershgorin scratch), then n_pad x
// n_pad FP32 matrices E, E^2, R, T, V, E_next and, per observable, Y, four
// product temporaries, and for the FP16 split the operand copies of E, E^2,
// R, T, E_next, every Y, S and W; trace and a0 partials.
struct FermiWS {
  size_t e, e2, r, t, v, en, y, g, sm, u, w, ce, ce2, cr, ct, cen, cy, cs, cw, part, a0p, total;
};

// Operand copy format of the finite-temperature products: none (FP32
// masters), the scaled FP16 split, or the two- / three-term BF16 split.
static int fermi_copy_prec(int prec) {
  return prec == kSplitH ? kSplitH : prec == kSplit3 ? kSplit3 : prec == kSplit2 ? kSplit2 : kFP32;
}

static FermiWS fermi_ws(size_t base, int n_pad, int nobs, int cprec) {
  FermiWS w;
  const size_t m = (size_t)n_pad * n_pad * 4;
  const size_t mc = cprec == kFP32 ? 0 : (size_t)n_pad * n_pad * operand_bytes(cprec);   // operand copy
  size_t off = align_up(base);
  w.e = off; off = align_up(off + m);
  w.e2 = off; off = align_up(off + m);
  w.r = off; off = align_up(off + m);
  w.t = off; off = align_up(off + m);
  w.v = off; off = align_up(off + m);
  w.en = off; off = align_up(off + m);
  w.y = off; off = align_up(off + m * nobs);
  w.g = off; off = align_up(off + m);
  w.sm = off; off = align_up(off + m);
  w.u = off; off = align_up(off + m);
  w.w = off; off = align_up(off + m);
  w.ce = off; off = align_up(off + mc);
  w.ce2 = off; off = align_up(off + mc);
  w.cr = off; off = align_up(off + mc);
  w.ct = off; off = align_up(off + mc);
  w.cen = off; off = align_up(off + mc);
  w.cy = off; off = align_up(off + mc * nobs);
  w.cs = off; off = align_up(off + mc);
  w.cw = off; off = align_up(off + mc);
  w.part = off; off = align_up(off + sizeof(double) * 2 * (size_t)trace_sq_blocks(n_pad));
  w.a0p = off; off = align_up(off + sizeof(double) * kOutBlocks * (size_t)std::max(nobs, 1));
  w.total = off;
  return w;
}

static dmpt_status fermi_check(const dmpt_opts* opts, const dmpt_fermi_opts* f, int nobs, Opts* o, Plan* p) {
  dmpt_status st = normalise(opts, o);
  if (st != DMPT_OK) return st;
  if (!f) return fail(DMPT_ERR_ARG, "fermi options are NULL");
  if (o->prec != kFP32 && o->prec != kSplitH && o->prec != kSplit3 && o->prec != kSplit2)
    return fail(DMPT_ERR_UNSUPPORTED, "the finite-temperature path runs in DMPT_FP32, DMPT_SPLIT_FP16, "
                                      "DMPT_SPLIT3_BF16 or DMPT_SPLIT_BF16");
  if (o->refine) return fail(DMPT_ERR_UNSUPPORTED, "refine applies to the zero-temperature solve");
  if (nobs < 0 || nobs > kMaxObs) return fail(DMPT_ERR_ARG, "nobs = %d out of range [0, %d]", nobs, kMaxObs);
  if (!(std::isfinite(f->kt) && f->kt > 0)) return fail(DMPT_ERR_ARG, "kt must be finite and > 0");
  if (f->canonical != 0 && f->canonical != 1) return fail(DMPT_ERR_ARG, "canonical must be 0 or 1");
  if (f->canonical && (o->nocc <= 0 || o->nocc >= o->n))
    return fail(DMPT_ERR_ARG, "the canonical ensemble needs 0 < nocc < n");
  if (!f->canonical && !std::isfinite(f->mu)) return fail(DMPT_ERR_ARG, "the grand canonical ensemble needs a finite mu");
  if (f->doublings < 0 || f->doublings > 40) return fail(DMPT_ERR_ARG, "doublings out of range [0, 40]");
  if (f->newton_max < 0 || f->newton_max > 200) return fail(DMPT_ERR_ARG, "newton_max out of range [0, 200]");
  if (!(f->count_tol >= 0) || !std::isfinite(f->count_tol)) return fail(DMPT_ERR_ARG, "count_tol must be finite and >= 0");
  if (f->reserved != 0) return fail(DMPT_ERR_ARG, "reserved must be 0");
  make_plan(*o, 0, p);
  return DMPT_OK;
}

size_t dmpt_fermi_workspace_bytes(const dmpt_opts* opts, const dmpt_fermi_opts* fopts, int32_t nobs) {
  Opts o;
  Plan p;
  if (fermi_check(opts, fopts, nobs, &o, &p) != DMPT_OK) return 0;
  return fermi_ws(p.off_x, p.n_pad, nobs, fermi_copy_prec(o.prec)).total;
}

// An operand of the finite-temperature products: FP32 master, and for the
// split formats its tiled copy (FP16 split: at the scale 2^e; BF16: e = 0).
struct FMat {
  float* m;
  void* c;
  int e;
};

// Fixed exponents of the FP16 copies (entry bounds x 2^e <= 2^14..2^15):
// |E| <= 1/2 (E = D - I/2), |E^2| <= 1/4, |R| <= 1 and |T| <= 1 (spectra in
// [1/2, 1] and [0, 1]); Y, S and W take 2^15 / ||M||_F (|M_ij| <= ||M||_F).
constexpr int kExpE = 15, kExpE2 = 16, kExpR = 14, kExpT = 14;

dmpt_status dmpt_susceptibility_fermi(const float* H, const float* A, int32_t nobs, float* chi, float* D,
                                      double* a0, const dmpt_fermi_opts* fopts, const dmpt_opts* opts,
                                      dmpt_fermi_info* finfo) {
  Opts o;
  Plan p;
  dmpt_status st = fermi_check(opts, fopts, nobs, &o, &p);
  if (st != DMPT_OK) return st;
  if (!H) return fail(DMPT_ERR_ARG, "H is NULL");
  if (nobs > 0 && (!A || !chi)) return fail(DMPT_ERR_ARG, "A and chi must not be NULL");
  const int n = o.n, np = p.n_pad;
  const int cprec = fermi_copy_prec(o.prec);
  const bool split = cprec != kFP32;
  const size_t cbytes = split ? (size_t)operand_bytes(cprec) : 0;
  const FermiWS w = fermi_ws(p.off_x, np, nobs, cprec);
  if (!o.ws) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", w.total);
  if (o.ws_bytes < w.total) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", o.ws_bytes, w.total);
  if (finfo) std::memset(finfo, 0, sizeof(*finfo));
  hipStream_t s = o.stream;
  char* ws = o.ws;
  Ctl* ctl = (Ctl*)(ws + p.off_ctl);
  const size_t np2 = (size_t)np * np;
  auto fm = [&](size_t master, size_t copy, size_t k) {
    return FMat{(float*)(ws + master) + k * np2, split ? (void*)(ws + copy + k * np2 * cbytes) : nullptr, 0};
  };
  FMat E = fm(w.e, w.ce, 0), E2 = fm(w.e2, w.ce2, 0), R = fm(w.r, w.cr, 0), T = fm(w.t, w.ct, 0);
  FMat En = fm(w.en, w.cen, 0), Sm = fm(w.sm, w.cs, 0), Wm = fm(w.w, w.cw, 0);
  std::vector<FMat> Y(std::max(nobs, 1));
  for (int k = 0; k < nobs; ++k) Y[k] = fm(w.y, w.cy, k);
  float* V = (float*)(ws + w.v);
  float* G = (float*)(ws + w.g);
  float* U = (float*)(ws + w.u);
  double* part = (double*)(ws + w.part);
  const int fl = flush_interval(cprec, np);
  const double beta = 1.0 / fopts->kt;
  ScopedEvents ev;
  DMPT_HIP(hipEventCreate(&ev.e0));
  DMPT_HIP(hipEventCreate(&ev.e1));
  DMPT_HIP(hipEventRecord(ev.e0, s));

  // spectral bounds (also the NaN / Inf scan)
  DMPT_HIP(launch_ctl_reset(ctl, s));
  st = compute_bounds(o, p, H, ctl, (double*)(ws + p.off_lz), (double2*)(ws + p.off_gersh), s);
  if (st != DMPT_OK) return st;
  Ctl hctl;
  DMPT_HIP(hipMemcpyAsync(&hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (hctl.nonfinite) return fail(DMPT_ERR_NONFINITE, "H holds NaN or Inf");
  const double emin = hctl.emin, emax = hctl.emax;

  // traces over the leading n x n block: (Tr M, ||M||_F^2), fixed order
  auto trace_sq = [&](const float* m, double* tr, double* sq) -> dmpt_status {
    const int nb = trace_sq_blocks(np);
    std::vector<double> h(2 * nb);
    DMPT_HIP(launch_trace_sq(m, n, np, part, s));
    DMPT_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s));
    DMPT_HIP(hipStreamSynchronize(s));
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nb; ++i) { a += h[2 * i]; b += h[2 * i + 1]; }
    *tr = a;
    *sq = b;
    return DMPT_OK;
  };
  // operand copy at a fixed exponent, or at 2^15 / ||M||_F
  auto refresh = [&](FMat& a, int e) -> dmpt_status {
    if (!split) return DMPT_OK;
    if (cprec != kSplitH) {   // BF16 terms keep the FP32 exponent range: no scale
      a.e = 0;
      DMPT_HIP(launch_copy_src(cprec, a.m, np, a.c, np, 0, s));
      return DMPT_OK;
    }
    a.e = e;
    DMPT_HIP(launch_split_copy(a.m, a.c, np, e, s));
    return DMPT_OK;
  };
  auto refresh_dyn = [&](FMat& a) -> dmpt_status {
    if (!split) return DMPT_OK;
    if (cprec != kSplitH) return refresh(a, 0);
    double tr = 0.0, sq = 0.0;
    dmpt_status e = trace_sq(a.m, &tr, &sq);
    if (e != DMPT_OK) return e;
    const double nrm = std::sqrt(sq);
    int ex = 0;
    if (nrm > 0 && std::isfinite(nrm)) ex = std::max(-100, std::min(100, (int)std::floor(std::log2(32768.0 / nrm))));
    return refresh(a, ex);
  };
  int products = 0;
  // out = alpha a b^T (all tiles, or the symmetric triangle + mirror)
  auto prod = [&](const FMat& a, const FMat& b, float* out, double alpha, bool sym) -> dmpt_status {
    ++products;
    if (split)
      DMPT_HIP(launch_gemm_op(cprec, a.c, b.c, out, np, (float)std::ldexp(alpha, -(a.e + b.e)), fl, sym ? 1 : 0, s));
    else
      DMPT_HIP(launch_gemm_op(kFP32, a.m, b.m, out, np, (float)alpha, fl, sym ? 1 : 0, s));
    return DMPT_OK;
  };
  auto doublings_for = [&](double mu) {
    if (fopts->doublings > 0) return fopts->doublings;
    const double wmax = std::max(std::fabs(emax - mu), std::fabs(emin - mu));
    int m = 1;
    while (m < 40 && beta * wmax / std::ldexp(1.0, m) > std::ldexp(1.0, -8)) ++m;
    return m;
  };
  // The recursion at mu; with ny > 0 also the responses Y_k (k < ny) of the
  // observables.  Leaves E_m in E.m and E_m^2 in E2.m.
  auto recursion = [&](double mu, int ny, int* m_out) -> dmpt_status {
    const int m = doublings_for(mu);
    *m_out = m;
    const double c = beta / std::ldexp(1.0, m + 2);
    const double wmax = std::max(std::fabs(emax - mu), std::fabs(emin - mu));
    dmpt_status e;
    DMPT_HIP(launch_fermi_start(H, n, np, -c, mu, E.m, s));
    if ((e = refresh(E, kExpE)) != DMPT_OK) return e;
    for (int k = 0; k < ny; ++k) {
      DMPT_HIP(launch_fermi_start(A + (size_t)k * n * n, n, np, -c, 0.0, Y[k].m, s));
      if ((e = refresh_dyn(Y[k])) != DMPT_OK) return e;
    }
    for (int step = 0; step < m; ++step) {
      if ((e = prod(E, E, E2.m, 1.0, true)) != DMPT_OK) return e;
      if ((e = refresh(E2, kExpE2)) != DMPT_OK) return e;
      // R = (I + 4 E^2)^{-1}: spectrum in [1, b], b from |E_k| <= tanh(2^{k-1-m} beta w) / 2
      // (with a margin for the linearised start and rounding)
      const double th = std::tanh(std::ldexp(beta * wmax, step - 1 - m));
      const double b = 1.0 + std::min(1.0, 1.02 * th * th + 1e-6);
      const double alpha = 2.0 / (1.0 + b);
      double err = (b - 1.0) / (b + 1.0);
      int iters = 0;
      while (err > 1e-8 && iters < 8) { err *= err; ++iters; }
      DMPT_HIP(launch_axpby(R.m, E2.m, 0.0f, nullptr, 0.0f, (float)alpha, np, np, s));
      if ((e = refresh(R, kExpR)) != DMPT_OK) return e;
      for (int it = 0; it < iters; ++it) {
        // T = (I + 4 E^2) R, V = R T, R = 2 R - V
        if ((e = prod(E2, R, T.m, 4.0, true)) != DMPT_OK) return e;
        DMPT_HIP(launch_axpby(T.m, T.m, 1.0f, R.m, 1.0f, 0.0f, 0, np, s));
        if ((e = refresh(T, kExpT)) != DMPT_OK) return e;
        if ((e = prod(R, T, V, 1.0, true)) != DMPT_OK) return e;
        DMPT_HIP(launch_axpby(R.m, R.m, 2.0f, V, -1.0f, 0.0f, 0, np, s));
        if ((e = refresh(R, kExpR)) != DMPT_OK) return e;
      }
      // E_next = 2 E R
      if ((e = prod(E, R, En.m, 2.0, true)) != DMPT_OK) return e;
      if ((e = refresh(En, kExpE)) != DMPT_OK) return e;
      for (int k = 0; k < ny; ++k) {
        // S = Y E + E Y; U = E_next S; W = 2 Y - 4 U; Y = sym(W R)
        if ((e = prod(Y[k], E, G, 1.0, false)) != DMPT_OK) return e;
        DMPT_HIP(launch_symm(G, 1.0f, nullptr, 0.0f, Sm.m, np, s));
        if ((e = refresh_dyn(Sm)) != DMPT_OK) return e;
        if ((e = prod(En, Sm, U, 1.0, false)) != DMPT_OK) return e;
        DMPT_HIP(launch_axpby(Wm.m, Y[k].m, 2.0f, U, -4.0f, 0.0f, 0, np, s));
        if ((e = refresh_dyn(Wm)) != DMPT_OK) return e;
        if ((e = prod(Wm, R, G, 1.0, false)) != DMPT_OK) return e;
        DMPT_HIP(launch_symm(G, 0.5f, nullptr, 0.0f, Y[k].m, np, s));
        if (step + 1 < m && (e = refresh_dyn(Y[k])) != DMPT_OK) return e;
      }
      std::swap(E, En);
    }
    if ((e = prod(E, E, E2.m, 1.0, true)) != DMPT_OK) return e;
    return DMPT_OK;
  };

  // chemical potential (canonical): safeguarded Newton steps on Tr D(mu) = N_occ.
  // A run carries the observables' responses when it is expected to verify mu
  // (or at a mu the caller supplies), so the verifying run is usually also the
  // final one; if such a run misses the tolerance, Newton continues.
  double mu = fopts->mu;
  int newton = 0, m = 0;
  double tre = 0.0, sqe = 0.0;
  bool have_final = false;
  if (fopts->canonical) {
    const double nocc = o.nocc;
    const double tol = fopts->count_tol > 0 ? fopts->count_tol : 1e-6 * n;
    double lo = emin - 40.0 / beta, hi = emax + 40.0 / beta;
    const bool given = std::isfinite(mu) && mu > lo && mu < hi;
    if (!given) mu = emin + (emax - emin) * nocc / n;
    const int maxn = fopts->newton_max > 0 ? fopts->newton_max : 40;
    bool with_obs = given;
    for (newton = 1; newton <= maxn; ++newton) {
      products = 0;
      if ((st = recursion(mu, with_obs ? nobs : 0, &m)) != DMPT_OK) return st;
      if ((st = trace_sq(E.m, &tre, &sqe)) != DMPT_OK) return st;
      const double count = 0.5 * n + tre;
      const double slope = beta * (0.25 * n - sqe);   // dTr D / dmu = beta Tr[D - D^2]
      if (std::fabs(count - nocc) <= tol) { have_final = with_obs || nobs == 0; break; }
      if (count < nocc) lo = mu; else hi = mu;
      double next = slope > 0 ? mu - (count - nocc) / slope : 0.5 * (lo + hi);
      if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
      // |c''| <= beta c' for the Fermi count c(mu), so the error after this step
      // is at most beta |dmu| |c - N_occ| / 2: carry the responses when that is below tol
      with_obs = 0.5 * beta * std::fabs(next - mu) * std::fabs(count - nocc) <= 0.5 * tol;
      mu = next;
    }
    if (newton > maxn)
      return fail(DMPT_ERR_NOT_CONVERGED, "chemical potential: |Tr D - N_occ| above %g after %d steps", tol, maxn);
  }
  // final run with the responses (unless the last canonical run was one)
  if (!have_final) {
    products = 0;
    if ((st = recursion(mu, nobs, &m)) != DMPT_OK) return st;
    if ((st = trace_sq(E.m, &tre, &sqe)) != DMPT_OK) return st;
  }
  const double trdd = 0.25 * n - sqe;   // Tr[D - D^2]
  std::vector<double> mu1(std::max(nobs, 1), 0.0);
  for (int k = 0; k < nobs; ++k) {
    if (fopts->canonical && trdd > 0) {
      double try_ = 0.0, sqy = 0.0;
      if ((st = trace_sq(Y[k].m, &try_, &sqy)) != DMPT_OK) return st;
      mu1[k] = try_ / (beta * trdd);
      // chi' = Y + mu_1 chi_gc(I), chi_gc(I) = -beta (D - D^2) = -beta (I/4 - E^2)
      const float gam = (float)(-mu1[k] * beta);
      DMPT_HIP(launch_axpby(Y[k].m, Y[k].m, 1.0f, E2.m, -gam, 0.25f * gam, n, np, s));
    }
  }
  // D = I/2 + E (into E^2's buffer, no longer needed), outputs and a0 = s Tr[A D]
  DMPT_HIP(launch_axpby(E2.m, E.m, 1.0f, nullptr, 0.0f, 0.5f, n, np, s));
  double* a0p = (double*)(ws + w.a0p);
  DMPT_HIP(launch_output(E2.m, nobs ? Y[0].m : nullptr, np2, A, n, np, nobs, D, nobs ? chi : nullptr, o.spin, 0,
                         nullptr, 0, 0, a0p, ctl, s));
  std::vector<double> hpart((size_t)kOutBlocks * std::max(nobs, 1));
  if (nobs) DMPT_HIP(hipMemcpyAsync(hpart.data(), a0p, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipEventRecord(ev.e1, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (a0)
    for (int k = 0; k < nobs; ++k) {
      double t = 0.0;
      for (int b = 0; b < kOutBlocks; ++b) t += hpart[(size_t)k * kOutBlocks + b];
      a0[k] = o.spin * t;
    }
  if (finfo) {
    finfo->mu = mu;
    finfo->trace_d = 0.5 * n + tre;
    finfo->emin = emin;
    finfo->emax = emax;
    finfo->doublings = m;
    finfo->newton = newton;
    finfo->products = products;
    for (int k = 0; k < nobs && k < 64; ++k) finfo->mu1[k] = mu1[k];
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
    finfo->elapsed_ms = ms;
  }
  return DMPT_OK;
}

size_t dmpt_response_workspace_bytes(int32_t nobs, int32_t npert, int32_t n) {
  return dmpt::response_workspace_bytes(nobs, npert, n);
}

dmpt_status dmpt_response(const float* chi, int32_t nobs, const float* H1, int32_t npert, int32_t n,
                          double* out, void* stream, void* workspace, size_t workspace_bytes) {
  return dmpt::response_run(chi, nobs, H1, npert, n, out, stream, workspace, workspace_bytes);
}

// ---------------------------------------------------------------- learned mixer

namespace dmpt {
namespace {

constexpr int kMixerMaxSteps = 65536;
constexpr int kMixerMseBlocks = 256;

struct MixWS {
  size_t scratch, part, grad, loss, total;
};

static bool mixer_sizes_ok(int n, int w, int h, int batch) {
  return n >= 1 && n <= 65536 && w >= 0 && w <= 512 && h >= 1 && h <= 4096 && batch >= 1 &&
         (size_t)batch * n <= ((size_t)1 << 20) &&
         (size_t)batch * n * (mixer_features(w) + 2 * h) <= ((size_t)1 << 31);
}

static MixWS mixer_ws(int n, int w, int h, int batch) {
  MixWS m;
  size_t off = 0;
  m.scratch = off; off = align_up(off + mixer_scratch_floats(n, w, h, batch) * 4);
  m.part = off; off = align_up(off + (size_t)kMixerMseBlocks * 8);
  m.grad = off; off = align_up(off + mixer_param_count(w, h) * 4);
  m.loss = off; off = align_up(off + (size_t)kMixerMaxSteps * 8);
  m.total = off;
  return m;
}

static dmpt_status mixer_check(int n, int w, int h, int batch, void* ws, size_t wsb, MixWS* m) {
  if (!mixer_sizes_ok(n, w, h, batch))
    return fail(DMPT_ERR_ARG, "mixer sizes out of range (n %d, window %d, hidden %d, batch %d)", n, w, h, batch);
  *m = mixer_ws(n, w, h, batch);
  if (!ws) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", m->total);
  if (wsb < m->total) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", wsb, m->total);
  return DMPT_OK;
}

// ---------------------------------------------------------------- self-consistent loop

struct ScfWS {
  size_t run_bytes;
  size_t ca, cw[2], wmat, da, v, f, r, vt, ft, rt, vb, rb, x, y, ediag, mlp, dv, dr, tab, coef, dot, total;
};

// History depth and hidden width the mixer uses (0 when it uses none).
static int scf_depth(const dmpt_scf_opts* scf) {
  return scf->mixer == DMPT_MIX_ANDERSON || scf->mixer == DMPT_MIX_LEARNED_ANDERSON ? scf->anderson_depth : 0;
}
static int scf_hidden(const dmpt_scf_opts* scf) {
  return scf->mixer == DMPT_MIX_LEARNED || scf->mixer == DMPT_MIX_LEARNED_ANDERSON ? scf->mlp_hidden : 0;
}

static ScfWS scf_ws(size_t run_bytes, int n, int depth, int window, int hidden) {
  ScfWS w;
  size_t off = align_up(run_bytes);
  const size_t mat = align_up((size_t)n * n * 4), vec = align_up((size_t)n * 8);
  w.run_bytes = run_bytes;
  w.ca = off; off += mat;
  w.cw[0] = off; off += mat;
  w.cw[1] = off; off += mat;
  w.wmat = off; off += mat;
  w.da = off; off += vec;
  w.v = off; off += vec;
  w.f = off; off += vec;
  w.r = off; off += vec;
  w.vt = off; off += vec;
  w.ft = off; off += vec;
  w.rt = off; off += vec;
  w.vb = off; off += vec;
  w.rb = off; off += vec;
  w.x = off; off += align_up((size_t)n * 4);
  w.y = off; off += align_up((size_t)n * 4);
  w.ediag = off; off += align_up((size_t)n * 4);
  w.mlp = off; off += hidden > 0 ? align_up(mixer_scratch_floats(n, window, hidden, 1) * 4) : 0;
  w.dv = off; off += (size_t)depth * vec;
  w.dr = off; off += (size_t)depth * vec;
  w.tab = off; off += align_up((size_t)2 * (2 + 2 * 16) * sizeof(void*));
  w.coef = off; off += align_up((size_t)(2 + 2 * 16) * 8);
  w.dot = off; off += align_up((size_t)(16 * 16 + 32) * 8);
  w.total = off;
  return w;
}

static dmpt_status scf_check(const dmpt_opts* opts, const dmpt_scf_opts* scf, Opts* o, dmpt_opts* o2, size_t* run_bytes) {
  dmpt_status st = normalise(opts, o);
  if (st != DMPT_OK) return st;
  if (!scf) return fail(DMPT_ERR_ARG, "scf options are NULL");
  if (scf->max_iter < 1 || scf->max_iter > DMPT_MAX_SCF)
    return fail(DMPT_ERR_ARG, "scf max_iter out of range [1, %d]", DMPT_MAX_SCF);
  if (!(scf->mix > 0 && scf->mix <= 1)) return fail(DMPT_ERR_ARG, "scf mix must be in (0, 1]");
  if (!(scf->tol > 0)) return fail(DMPT_ERR_ARG, "scf tol must be > 0");
  if (scf->mixer < DMPT_MIX_LINEAR || scf->mixer > DMPT_MIX_LEARNED_ANDERSON)
    return fail(DMPT_ERR_ARG, "unknown mixer %d", scf->mixer);
  const bool anderson = scf->mixer == DMPT_MIX_ANDERSON || scf->mixer == DMPT_MIX_LEARNED_ANDERSON;
  const bool learned = scf->mixer == DMPT_MIX_LEARNED || scf->mixer == DMPT_MIX_LEARNED_ANDERSON;
  if (anderson && (scf->anderson_depth < 1 || scf->anderson_depth > 16))
    return fail(DMPT_ERR_ARG, "anderson_depth out of range [1, 16]");
  if (learned &&
      (!scf->mlp_params || !mixer_sizes_ok(o->n, scf->mlp_window, scf->mlp_hidden, 1)))
    return fail(DMPT_ERR_ARG, "the learned mixer needs mlp_params and a valid mlp_window / mlp_hidden");
  if (scf->reserved != 0) return fail(DMPT_ERR_ARG, "scf reserved must be 0");
  if (o->refine) return fail(DMPT_ERR_UNSUPPORTED, "refine applies to the forward sweep, not the self-consistent loop");
  *o2 = *opts;
  o2->sweep = DMPT_SWEEP_ADJOINT;
  o2->spin = 1.0;
  Opts oo;
  normalise(o2, &oo);
  Plan p;
  make_plan(oo, 1, &p);
  *run_bytes = p.total;
  return DMPT_OK;
}

// Solve the k x k system (g + lambda I) x = b by Gaussian elimination with
// partial pivoting (k <= 16).
static void small_solve(std::vector<double> g, std::vector<double> b, int k, std::vector<double>* x) {
  double tr = 0.0;
  for (int i = 0; i < k; ++i) tr += g[i * k + i];
  const double lambda = 1e-12 * (tr > 0 ? tr / k : 1.0);
  for (int i = 0; i < k; ++i) g[i * k + i] += lambda;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(g[r * k + c]) > std::fabs(g[piv * k + c])) piv = r;
    if (piv != c) {
      for (int j = 0; j < k; ++j) std::swap(g[c * k + j], g[piv * k + j]);
      std::swap(b[c], b[piv]);
    }
    const double d = g[c * k + c];
    if (d == 0.0) continue;
    for (int r = c + 1; r < k; ++r) {
      const double f = g[r * k + c] / d;
      for (int j = c; j < k; ++j) g[r * k + j] -= f * g[c * k + j];
      b[r] -= f * b[c];
    }
  }
  x->assign(k, 0.0);
  for (int c = k - 1; c >= 0; --c) {
    double t = b[c];
    for (int j = c + 1; j < k; ++j) t -= g[c * k + j] * (*x)[j];
    (*x)[c] = g[c * k + c] != 0.0 ? t / g[c * k + c] : 0.0;
  }
}

}  // namespace
}  // namespace dmpt

size_t dmpt_mixer_param_count(int32_t window, int32_t hidden) {
  if (!mixer_sizes_ok(1, window, hidden, 1)) return 0;
  return mixer_param_count(window, hidden);
}

size_t dmpt_mixer_workspace_bytes(int32_t n, int32_t window, int32_t hidden, int32_t batch) {
  if (!mixer_sizes_ok(n, window, hidden, batch)) {
    fail(DMPT_ERR_ARG, "mixer sizes out of range (n %d, window %d, hidden %d, batch %d)", n, window, hidden, batch);
    return 0;
  }
  return mixer_ws(n, window, hidden, batch).total;
}

dmpt_status dmpt_mixer_init(float* master, uint16_t* params, int32_t window, int32_t hidden, uint64_t seed,
                            void* stream) {
  if (!master || !params) return fail(DMPT_ERR_ARG, "master and params must not be NULL");
  if (!mixer_sizes_ok(1, window, hidden, 1)) return fail(DMPT_ERR_ARG, "mixer sizes out of range");
  hipStream_t s = (hipStream_t)stream;
  DMPT_HIP(mixer_init(master, params, window, hidden, seed, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

dmpt_status dmpt_mixer_forward(const uint16_t* params, int32_t window, int32_t hidden, const float* U, const float* E,
                               int32_t n,
                               const float* x, int32_t batch, float* y, void* stream, void* workspace,
                               size_t workspace_bytes) {
  if (!params || !U || !E || !x || !y) return fail(DMPT_ERR_ARG, "params, U, E, x and y must not be NULL");
  MixWS m;
  dmpt_status st = mixer_check(n, window, hidden, batch, workspace, workspace_bytes, &m);
  if (st != DMPT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  DMPT_HIP(mixer_forward(params, window, hidden, U, E, n, x, batch, y, (float*)(ws + m.scratch), s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

dmpt_status dmpt_mixer_loss_grad(const uint16_t* params, int32_t window, int32_t hidden, const float* U, const float* E,
                                 int32_t n,
                                 const float* x, const float* t, int32_t batch, float* grad, double* loss,
                                 void* stream, void* workspace, size_t workspace_bytes) {
  if (!params || !U || !E || !x || !t || !grad || !loss) return fail(DMPT_ERR_ARG, "NULL argument");
  MixWS m;
  dmpt_status st = mixer_check(n, window, hidden, batch, workspace, workspace_bytes, &m);
  if (st != DMPT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  double* ld = (double*)(ws + m.loss);
  DMPT_HIP(mixer_loss_grad(params, window, hidden, U, E, n, x, t, batch, (float*)(ws + m.scratch),
                           (double*)(ws + m.part), grad, ld, 0, s));
  DMPT_HIP(hipMemcpyAsync(loss, ld, sizeof(double), hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

dmpt_status dmpt_mixer_train(float* master, uint16_t* params, float* adam_m, float* adam_v, int32_t window,
                             int32_t hidden, const float* U, const float* E, int32_t n, const float* x, const float* t,
                             int32_t npairs, int32_t batch, int32_t steps, double lr, double* loss_history,
                             void* stream, void* workspace, size_t workspace_bytes) {
  if (!master || !params || !adam_m || !adam_v || !U || !E || !x || !t) return fail(DMPT_ERR_ARG, "NULL argument");
  if (npairs < batch || steps < 1 || steps > kMixerMaxSteps || !(lr > 0))
    return fail(DMPT_ERR_ARG, "need npairs >= batch, 1 <= steps <= %d, lr > 0", kMixerMaxSteps);
  MixWS m;
  dmpt_status st = mixer_check(n, window, hidden, batch, workspace, workspace_bytes, &m);
  if (st != DMPT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  double* ld = (double*)(ws + m.loss);
  const size_t np = mixer_param_count(window, hidden);
  for (int k = 1; k <= steps; ++k) {
    size_t start = ((size_t)(k - 1) * batch) % (size_t)npairs;
    if (start + batch > (size_t)npairs) start = (size_t)npairs - batch;
    DMPT_HIP(mixer_loss_grad(params, window, hidden, U, E, n, x + start * n, t + start * n, batch,
                             (float*)(ws + m.scratch), (double*)(ws + m.part), (float*)(ws + m.grad), ld, k - 1, s));
    DMPT_HIP(mixer_adam(master, params, adam_m, adam_v, (const float*)(ws + m.grad), np, (float)lr, k, s));
  }
  if (loss_history) DMPT_HIP(hipMemcpyAsync(loss_history, ld, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

size_t dmpt_mixer_rows_workspace_bytes(int32_t rows) {
  if (rows < 1 || rows > (1 << 24)) {
    fail(DMPT_ERR_ARG, "rows = %d out of range [1, 2^24]", rows);
    return 0;
  }
  return align_up(sizeof(int32_t) * (size_t)rows);
}

dmpt_status dmpt_mixer_pairs(const float* v, const float* r, const double* residual, int32_t k, int32_t n,
                             const float* vstar, double mix, double min_residual, int32_t drop_last,
                             float* x_out, float* t_out, int32_t capacity, int32_t* count, void* stream,
                             void* workspace, size_t workspace_bytes) {
  if (!v || !r || !residual || !vstar || !x_out || !t_out || !count) return fail(DMPT_ERR_ARG, "NULL argument");
  if (k < 1 || k > (1 << 24) || n < 1 || n > 65536) return fail(DMPT_ERR_ARG, "k = %d or n = %d out of range", k, n);
  if (drop_last != 0 && drop_last != 1) return fail(DMPT_ERR_ARG, "drop_last must be 0 or 1");
  if (!std::isfinite(mix) || !std::isfinite(min_residual)) return fail(DMPT_ERR_ARG, "mix and min_residual must be finite");
  if (!workspace || workspace_bytes < align_up(sizeof(int32_t) * (size_t)k))
    return fail(DMPT_ERR_WORKSPACE, "workspace needs %zu bytes", align_up(sizeof(int32_t) * (size_t)k));
  std::vector<int32_t> rows;
  for (int j = 0; j < k; ++j)
    if (residual[j] >= min_residual && !(drop_last && j == k - 1)) rows.push_back(j);
  if ((int)rows.size() > capacity) return fail(DMPT_ERR_ARG, "%zu pairs exceed capacity %d", rows.size(), capacity);
  *count = (int32_t)rows.size();
  if (rows.empty()) return DMPT_OK;
  hipStream_t s = (hipStream_t)stream;
  int* d_rows = (int*)workspace;
  DMPT_HIP(hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, s));
  DMPT_HIP(mixer_pairs(v, r, vstar, d_rows, (int)rows.size(), n, (float)mix, x_out, t_out, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

dmpt_status dmpt_mixer_shuffle(const float* x, const float* t, int32_t npairs, int32_t n, uint64_t seed,
                               float* x_out, float* t_out, void* stream, void* workspace, size_t workspace_bytes) {
  if (!x || !t || !x_out || !t_out) return fail(DMPT_ERR_ARG, "NULL argument");
  if (npairs < 1 || npairs > (1 << 24) || n < 1 || n > 65536)
    return fail(DMPT_ERR_ARG, "npairs = %d or n = %d out of range", npairs, n);
  if (x_out == x || t_out == t) return fail(DMPT_ERR_ARG, "the shuffle does not run in place");
  if (!workspace || workspace_bytes < align_up(sizeof(int32_t) * (size_t)npairs))
    return fail(DMPT_ERR_WORKSPACE, "workspace needs %zu bytes", align_up(sizeof(int32_t) * (size_t)npairs));
  // Fisher-Yates with splitmix64 draws (counter = seed + step), index by
  // the high half of a 64 x 64-bit product (Lemire's bounded integers).
  std::vector<int32_t> perm(npairs);
  for (int i = 0; i < npairs; ++i) perm[i] = i;
  for (int i = npairs - 1; i > 0; --i) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(npairs - i);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int j = (int)(((unsigned __int128)z * (uint64_t)(i + 1)) >> 64);
    std::swap(perm[i], perm[j]);
  }
  hipStream_t s = (hipStream_t)stream;
  int* d_perm = (int*)workspace;
  DMPT_HIP(hipMemcpyAsync(d_perm, perm.data(), sizeof(int32_t) * npairs, hipMemcpyHostToDevice, s));
  DMPT_HIP(mixer_gather_rows(x, d_perm, npairs, n, x_out, s));
  DMPT_HIP(mixer_gather_rows(t, d_perm, npairs, n, t_out, s));
  DMPT_HIP(hipStreamSynchronize(s));
  return DMPT_OK;
}

size_t dmpt_scf_workspace_bytes(const dmpt_opts* opts, const dmpt_scf_opts* scf) {
  Opts o;
  dmpt_opts o2;
  size_t run_bytes = 0;
  if (scf_check(opts, scf, &o, &o2, &run_bytes) != DMPT_OK) return 0;
  return scf_ws(run_bytes, o.n, scf_depth(scf), scf->mlp_window, scf_hidden(scf)).total;
}

dmpt_status dmpt_scf_response(const float* H0, const float* U, const float* A, float* chi,
                              const dmpt_scf_opts* scf, const dmpt_opts* opts, dmpt_info* info,
                              dmpt_scf_info* sinfo) {
  Opts o;
  dmpt_opts o2;
  size_t run_bytes = 0;
  dmpt_status st = scf_check(opts, scf, &o, &o2, &run_bytes);
  if (st != DMPT_OK) return st;
  if (!H0 || !U || !A || !chi) return fail(DMPT_ERR_ARG, "H0, U, A and chi must not be NULL");
  const int n = o.n;
  const int depth = scf_depth(scf);
  const ScfWS w = scf_ws(run_bytes, n, depth, scf->mlp_window, scf_hidden(scf));
  if (!o.ws) return fail(DMPT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", w.total);
  if (o.ws_bytes < w.total) return fail(DMPT_ERR_WORKSPACE, "workspace has %zu bytes, need %zu", o.ws_bytes, w.total);
  if (sinfo) std::memset(sinfo, 0, sizeof(*sinfo));
  hipStream_t s = o.stream;
  char* ws = o.ws;
  o2.workspace = ws;
  o2.workspace_bytes = w.run_bytes;
  float* ca = (float*)(ws + w.ca);
  float* cw[2] = {(float*)(ws + w.cw[0]), (float*)(ws + w.cw[1])};
  float* wmat = (float*)(ws + w.wmat);
  double* da = (double*)(ws + w.da);
  double *v = (double*)(ws + w.v), *f = (double*)(ws + w.f), *r = (double*)(ws + w.r);
  double *vt = (double*)(ws + w.vt), *ft = (double*)(ws + w.ft), *rt = (double*)(ws + w.rt);
  float* xf = (float*)(ws + w.x);
  float* yf = (float*)(ws + w.y);
  float* ediag = (float*)(ws + w.ediag);   // on-site energies of H0 (learned mixer input)
  const void** tab = (const void**)(ws + w.tab);
  double* coef = (double*)(ws + w.coef);
  double* dot = (double*)(ws + w.dot);
  const double spin = o.spin;

  // chi'_A = L[A]: the SP2 recursion of H0 (X_n kept) and one backward sweep
  st = run(H0, A, 1, ca, nullptr, nullptr, &o2, info, false);
  if (st != DMPT_OK) return st;
  DMPT_HIP(scf_get_diag(ca, n, da, s));
  if (scf_hidden(scf) > 0) DMPT_HIP(mixer_diag(H0, n, ediag, s));
  DMPT_HIP(hipMemsetAsync(v, 0, (size_t)n * 8, s));
  DMPT_HIP(hipMemcpyAsync(f, da, (size_t)n * 8, hipMemcpyDeviceToDevice, s));

  // host-side helpers: norms of r and f; F at a trial state
  std::vector<const void*> htab(2 * (2 + 2 * 16));
  auto norms = [&](const double* rr, const double* ff, double* rn, double* fn) -> dmpt_status {
    htab[0] = rr; htab[1] = ff; htab[2] = rr; htab[3] = ff;
    DMPT_HIP(hipMemcpyAsync(tab, htab.data(), 4 * sizeof(void*), hipMemcpyHostToDevice, s));
    DMPT_HIP(scf_dots((const double* const*)tab, (const double* const*)(tab + 2), 2, n, dot, s));
    double h2[2];
    DMPT_HIP(hipMemcpyAsync(h2, dot, sizeof(h2), hipMemcpyDeviceToHost, s));
    DMPT_HIP(hipStreamSynchronize(s));
    *rn = std::sqrt(h2[0]);
    *fn = std::sqrt(h2[1]);
    return DMPT_OK;
  };
  int cur = 0;   // cw[cur] belongs to the accepted state (unused while v = 0)
  bool have_cw = false;
  auto evaluate = [&](const double* vv, double* ff, float* cwout) -> dmpt_status {
    DMPT_HIP(scf_set_diag(wmat, n, U, vv, spin, s));
    dmpt_status e = run(H0, wmat, 1, cwout, nullptr, nullptr, &o2, nullptr, true);
    if (e != DMPT_OK) return e;
    DMPT_HIP(scf_fvec(ff, da, cwout, n, s));
    return DMPT_OK;
  };

  int evals = 1, rejected = 0, converged = 0, hist = 0, hhead = 0, accepted = 0;
  double rn = 0, fn = 0;
  DMPT_HIP(scf_residual(r, f, v, n, scf->record_v, scf->record_r, s));
  st = norms(r, f, &rn, &fn);
  if (st != DMPT_OK) return st;
  double res = fn > 0 ? rn / fn : 0.0;
  if (sinfo) sinfo->residual[0] = res;
  converged = res <= scf->tol;
  while (!converged && evals < scf->max_iter) {
    // proposal
    bool special = false;
    const bool learned = scf->mixer == DMPT_MIX_LEARNED || scf->mixer == DMPT_MIX_LEARNED_ANDERSON;
    const bool anderson = scf->mixer == DMPT_MIX_ANDERSON || scf->mixer == DMPT_MIX_LEARNED_ANDERSON;
    // the learned step from (vv, rr) with ||rr|| = rrn:
    // vt = vv + mix rr + (rrn / sqrt(n)) net(sqrt(n) rr / rrn)
    auto learned_step = [&](const double* vv, const double* rr, double rrn) -> dmpt_status {
      const double sq = std::sqrt((double)n);
      DMPT_HIP(scf_to_float(xf, rr, sq / rrn, n, s));
      DMPT_HIP(mixer_forward(scf->mlp_params, scf->mlp_window, scf->mlp_hidden, U, ediag, n, xf, 1, yf,
                             (float*)(ws + w.mlp), s));
      DMPT_HIP(scf_step(vt, vv, rr, scf->mix, yf, rrn / sq, n, s));
      return DMPT_OK;
    };
    auto dr = [&](int i) { return (const double*)(ws + w.dr) + (size_t)i * n; };
    auto dv = [&](int i) { return (const double*)(ws + w.dv) + (size_t)i * n; };
    // gamma = argmin || r - sum_j gamma_j dR_j || over the history
    auto anderson_gamma = [&](std::vector<double>* gamma) -> dmpt_status {
      const int k = hist;
      std::vector<std::pair<int, int>> pairs;
      for (int i = 0; i < k; ++i)
        for (int j = i; j < k; ++j) pairs.emplace_back(i, j);
      // the Gram matrix dR^T dR and dR^T r, 16 dot products per pass
      std::vector<double> g(k * k), b(k);
      for (size_t base = 0; base < pairs.size() + k; base += 16) {
        std::vector<const void*> xs, ys;
        for (size_t e = base; e < std::min(pairs.size() + k, base + 16); ++e) {
          if (e < pairs.size()) {
            xs.push_back(dr(pairs[e].first));
            ys.push_back(dr(pairs[e].second));
          } else {
            xs.push_back(dr((int)(e - pairs.size())));
            ys.push_back(r);
          }
        }
        const int cnt = (int)xs.size();
        std::vector<const void*> both(xs);
        both.insert(both.end(), ys.begin(), ys.end());
        DMPT_HIP(hipMemcpyAsync(tab, both.data(), both.size() * sizeof(void*), hipMemcpyHostToDevice, s));
        DMPT_HIP(scf_dots((const double* const*)tab, (const double* const*)(tab + cnt), cnt, n, dot, s));
        std::vector<double> out(cnt);
        DMPT_HIP(hipMemcpyAsync(out.data(), dot, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        DMPT_HIP(hipStreamSynchronize(s));
        for (int e = 0; e < cnt; ++e) {
          const size_t idx = base + e;
          if (idx < pairs.size()) {
            g[pairs[idx].first * k + pairs[idx].second] = out[e];
            g[pairs[idx].second * k + pairs[idx].first] = out[e];
          } else {
            b[idx - pairs.size()] = out[e];
          }
        }
      }
      small_solve(g, b, k, gamma);
      return DMPT_OK;
    };
    // out = sum_q c_q x_q (device vectors), synchronised
    auto lincomb = [&](double* out, const std::vector<const void*>& vecs, const std::vector<double>& cs) -> dmpt_status {
      DMPT_HIP(hipMemcpyAsync(tab, vecs.data(), vecs.size() * sizeof(void*), hipMemcpyHostToDevice, s));
      DMPT_HIP(hipMemcpyAsync(coef, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice, s));
      DMPT_HIP(scf_lincomb(out, (const double* const*)tab, coef, (int)vecs.size(), n, s));
      DMPT_HIP(hipStreamSynchronize(s));
      return DMPT_OK;
    };
    if (anderson && hist > 0) {
      std::vector<double> gamma;
      if ((st = anderson_gamma(&gamma)) != DMPT_OK) return st;
      if (!learned) {
        // v' = v + mix r - sum_j gamma_j (dV_j + mix dR_j)
        std::vector<const void*> vecs = {v, r};
        std::vector<double> cs = {1.0, scf->mix};
        for (int j = 0; j < hist; ++j) {
          vecs.push_back(dv(j));
          cs.push_back(-gamma[j]);
          vecs.push_back(dr(j));
          cs.push_back(-scf->mix * gamma[j]);
        }
        if ((st = lincomb(vt, vecs, cs)) != DMPT_OK) return st;
        special = true;
      } else {
        // the learned step from the extrapolated state and residual
        // vb = v - sum_j gamma_j dV_j, rb = r - sum_j gamma_j dR_j
        std::vector<const void*> vv = {v}, rr = {r};
        std::vector<double> cv = {1.0}, cr = {1.0};
        for (int j = 0; j < hist; ++j) {
          vv.push_back(dv(j));
          cv.push_back(-gamma[j]);
          rr.push_back(dr(j));
          cr.push_back(-gamma[j]);
        }
        double* vb = (double*)(ws + w.vb);
        double* rb = (double*)(ws + w.rb);
        if ((st = lincomb(vb, vv, cv)) != DMPT_OK) return st;
        if ((st = lincomb(rb, rr, cr)) != DMPT_OK) return st;
        double rbn = 0, unused = 0;
        if ((st = norms(rb, rb, &rbn, &unused)) != DMPT_OK) return st;
        if (rbn > 0) {
          if ((st = learned_step(vb, rb, rbn)) != DMPT_OK) return st;
          special = true;
        } else {
          DMPT_HIP(scf_step(vt, v, r, scf->mix, nullptr, 0.0, n, s));
        }
      }
    } else if (learned && rn > 0) {
      if ((st = learned_step(v, r, rn)) != DMPT_OK) return st;
      special = true;
    } else {
      DMPT_HIP(scf_step(vt, v, r, scf->mix, nullptr, 0.0, n, s));
    }
    // evaluate the proposal
    st = evaluate(vt, ft, cw[cur ^ 1]);
    if (st != DMPT_OK) return st;
    ++evals;
    DMPT_HIP(scf_residual(rt, ft, vt, n, nullptr, nullptr, s));
    double rn2 = 0, fn2 = 0;
    st = norms(rt, ft, &rn2, &fn2);
    if (st != DMPT_OK) return st;
    if (special && rn2 > rn && evals < scf->max_iter) {
      // rejected: fall back to the linear step from the current state
      ++rejected;
      DMPT_HIP(scf_step(vt, v, r, scf->mix, nullptr, 0.0, n, s));
      st = evaluate(vt, ft, cw[cur ^ 1]);
      if (st != DMPT_OK) return st;
      ++evals;
      DMPT_HIP(scf_residual(rt, ft, vt, n, nullptr, nullptr, s));
      st = norms(rt, ft, &rn2, &fn2);
      if (st != DMPT_OK) return st;
    }
    // accept: history (Anderson), swap state
    if (depth > 0) {
      double* dvj = (double*)(ws + w.dv) + (size_t)hhead * n;
      double* drj = (double*)(ws + w.dr) + (size_t)hhead * n;
      std::vector<const void*> vecs = {vt, v, rt, r};
      DMPT_HIP(hipMemcpyAsync(tab, vecs.data(), 4 * sizeof(void*), hipMemcpyHostToDevice, s));
      const double cs[4] = {1.0, -1.0, 1.0, -1.0};
      DMPT_HIP(hipMemcpyAsync(coef, cs, sizeof(cs), hipMemcpyHostToDevice, s));
      DMPT_HIP(scf_lincomb(dvj, (const double* const*)tab, coef, 2, n, s));
      DMPT_HIP(scf_lincomb(drj, (const double* const*)(tab + 2), coef + 2, 2, n, s));
      DMPT_HIP(hipStreamSynchronize(s));
      hhead = (hhead + 1) % depth;
      hist = std::min(hist + 1, depth);
    }
    std::swap(v, vt);
    std::swap(f, ft);
    std::swap(r, rt);
    cur ^= 1;
    have_cw = true;
    rn = rn2;
    fn = fn2;
    res = fn > 0 ? rn / fn : 0.0;
    ++accepted;   // accepted states are numbered 0 (v = 0), 1, 2, ... (<= evals - 1 < max_iter)
    if (scf->record_v || scf->record_r) {
      const size_t slot = (size_t)accepted * n;
      DMPT_HIP(scf_residual(rt, f, v, n, scf->record_v ? scf->record_v + slot : nullptr,
                            scf->record_r ? scf->record_r + slot : nullptr, s));
    }
    if (sinfo) sinfo->residual[accepted] = res;
    converged = res <= scf->tol;
  }
  // chi = s (L[A] + L[diag(U s v)]) at the last accepted state
  DMPT_HIP(scf_combine(chi, ca, have_cw ? cw[cur] : nullptr, spin, (size_t)n * n, s));
  DMPT_HIP(hipStreamSynchronize(s));
  if (sinfo) {
    sinfo->iters = evals;
    sinfo->converged = converged;
    sinfo->rejected = rejected;
    sinfo->states = accepted + 1;
  }
  if (!converged) return fail(DMPT_ERR_NOT_CONVERGED, "self-consistent loop did not converge in %d evaluations", evals);
  return DMPT_OK;
}

int32_t dmpt_sp2_decide(double tr, double sq, double eps, double eps_prev1, double eps_prev2, double eps_prev3,
                        int32_t steps, int32_t n, double nocc, int32_t min_iter, double idem_tol,
                        int32_t precision) {
  return sp2_decide(tr, sq, eps, eps_prev1, eps_prev2, eps_prev3, steps, n, nocc, min_iter, idem_tol, precision);
}

const char* dmpt_status_string(dmpt_status st) {
  switch (st) {
    case DMPT_OK: return "DMPT_OK";
    case DMPT_ERR_ARG: return "DMPT_ERR_ARG";
    case DMPT_ERR_NONFINITE: return "DMPT_ERR_NONFINITE";
    case DMPT_ERR_NOT_CONVERGED: return "DMPT_ERR_NOT_CONVERGED";
    case DMPT_ERR_BOUNDS: return "DMPT_ERR_BOUNDS";
    case DMPT_ERR_DEVICE: return "DMPT_ERR_DEVICE";
    case DMPT_ERR_WORKSPACE: return "DMPT_ERR_WORKSPACE";
    case DMPT_ERR_UNSUPPORTED: return "DMPT_ERR_UNSUPPORTED";
  }
  return "unknown dmpt_status";
}

const char* dmpt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
