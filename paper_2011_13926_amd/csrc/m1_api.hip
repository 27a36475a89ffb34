// C ABI of the implicit M1 step: context management, argument validation, the
// Newton loop (Sect. 3.3.1) and the restarted GMRES driver (one host read-back
// per GMRES cycle; everything else stays on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/m1.h"
#include "m1_internal.h"
#include "m1_nn.h"

using namespace m1;

namespace {

const char* kClassNames[KC_COUNT] = {"setup",   "setup_bj", "residual",   "apply",         "block_jacobi",
                                     "arnoldi_dot", "arnoldi_scalar", "arnoldi_update", "x_update",
                                     "true_residual", "newton_update", "norm", "convert", "learned_pc", "apply_bj_fused",
                                     "time_step", "velocity_sources", "mg_setup", "mg_fine", "mg_smooth",
                                     "mg_down", "mg_coarse_solve"};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  // iter >= 0: a launch inside a GMRES cycle that may have returned at once after
  // the cycle converged; resolved against the cycle's column count (prof_resolve).
  // phase 0: before the Hessenberg step of iteration `iter`, 1: after it, 2: final step.
  // n: launches the record spans (consecutive launches of one multigrid class share
  // one event pair; see timed)
  struct Rec { int kc; hipEvent_t a, b; double bytes; int iter; int phase; bool valid; int n; };
  std::vector<Rec> pending;
  int open = -1;   // index in pending of a record whose end event is not yet recorded
  int64_t seen[KC_COUNT] = {};   // launches issued while profiling, sampled or not
  int64_t launches[KC_COUNT] = {};
  double ms[KC_COUNT] = {};
  double bytes[KC_COUNT] = {};
};

}  // namespace

struct m1_ctx {
  m1_config cfg;
  int nd = 2, nu = 3, nrad = 3, njac = 9, m = 30;
  bool cpl = false;
  Geom g;
  Scheme sc;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  bool linearized = false;
  bool bj_ready = false;     // block-Jacobi inverse (and FP32 shadow) match the coefficients and sc.psi
  double bj_psi = 0.0;       // shift the block-Jacobi inverse was built with
  double lin_rtol = -1.0;    // >= 0: linear tolerance of the current Newton solve (else cfg.rtol)
  // boundary copies
  double* plane[6] = {};
  double* mask[6] = {};
  // states
  double* Uk = nullptr;
  double* Un = nullptr;
  double* Uprev = nullptr;   // Newton line search: the iterate before the step
  double* fn = nullptr;
  // coefficients
  double* coef64 = nullptr;
  float* coef32 = nullptr;
  int64_t coef_len = 0;
  Coefs<double> cf64;
  Coefs<float> cf32;
  // Krylov workspace
  void* V = nullptr;
  int64_t n = 0;        // vector length n_u*N
  int64_t vs = 0;       // stride between basis vectors: n rounded up to 64 elements (aligned quads)
  double* b = nullptr;
  double* x = nullptr;
  void* u[2] = {};
  void* p = nullptr;
  void* z = nullptr;
  double* part = nullptr;
  int nb = 1;
  GmresState* gs = nullptr;
  double* dscal = nullptr;
  unsigned long long* dcount = nullptr;
  // flexible GMRES (learned preconditioner)
  m1nn* net = nullptr;
  void* Z = nullptr;
  int use_learned = 0;   // 1 while the current solve uses the network
  // aggregation multigrid (pc = M1_PC_MULTIGRID)
  MgHierarchy mg;
  double* xw = nullptr;  // V y before the preconditioner at the end of a cycle
  // pinned host read-back
  double* hscal = nullptr;
  Profiler prof;
};

namespace {

bool hip_ok(m1_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

#define HIPCHK(ctx, call)                                   \
  do {                                                      \
    if (!hip_ok((ctx), (call), #call)) return M1_ERR_HIP;   \
  } while (0)

hipEvent_t prof_event(m1_ctx* c) {
  Profiler& p = c->prof;
  if (p.used == p.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.pool.push_back(e);
  }
  return p.pool[p.used++];
}

// Kernel classes launched once per Krylov iteration are timed on every 13th
// launch only (13 is prime to the restart lengths, so every Arnoldi step j is
// sampled over a solve); an event pair per launch would cost about a third of
// the solver's run time at 512^2.  Other classes are timed on every launch.
bool per_iteration_class(int kc) {
  return kc == KC_APPLY || kc == KC_BJ || kc == KC_DOT || kc == KC_SCALAR || kc == KC_UPDATE || kc == KC_NN ||
         kc == KC_APPLY_PC || kc == KC_MG_FINE || kc == KC_MG_SMOOTH || kc == KC_MG_DOWN || kc == KC_MG_COARSE;
}

// The multigrid classes come in runs of consecutive launches (a cycle's finest-level
// sweeps of one leg, its restrictions, its prolongations): a sampled launch of such a
// class keeps its interval open, and the following launches of the same class join it
// until another launch or prof_close ends it.  One event pair then spans several
// kernels, so the dispatch that the events add is spread over them instead of being
// charged to each.
bool grouped_class(int kc) {
  return kc == KC_MG_FINE || kc == KC_MG_SMOOTH || kc == KC_MG_DOWN || kc == KC_MG_COARSE;
}

// end an open interval (before any stream work that is not launched through timed)
void prof_close(m1_ctx* c) {
  Profiler& p = c->prof;
  if (p.open < 0) return;
  hipEventRecord(p.pending[p.open].b, c->stream);
  p.open = -1;
}

// Launch with optional HIP-event timing; `bytes` is the launch's algorithmic
// HBM traffic (each array element the kernel must read or write, once).
template <typename F>
void timed(m1_ctx* c, int kc, double bytes, F&& launch, int iter = -1, int phase = 0) {
  if (!c->prof.on) {
    launch();
    return;
  }
  Profiler& p = c->prof;
  if (p.open >= 0) {
    Profiler::Rec& r = p.pending[p.open];
    if (r.kc == kc && r.iter == iter && r.phase == phase) {
      p.seen[kc]++;
      launch();
      r.bytes += bytes;
      r.n += 1;
      return;
    }
    prof_close(c);
  }
  const int64_t seq = p.seen[kc]++;
  if (per_iteration_class(kc) && seq % 13 != 0) {
    launch();
    return;
  }
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (a) hipEventRecord(a, c->stream);
  launch();
  if (!(a && b)) return;
  p.pending.push_back({kc, a, b, bytes, iter, phase, true, 1});
  if (grouped_class(kc)) p.open = (int)p.pending.size() - 1;
  else hipEventRecord(b, c->stream);
}

// Drop the records of launches that returned at once because the cycle had
// already finished: k columns were used out of `steps`.
void prof_resolve(m1_ctx* c, int k, int steps) {
  for (auto& r : c->prof.pending) {
    if (r.iter < 0) continue;
    r.valid = r.phase == 0 ? r.iter <= k : (r.phase == 1 ? r.iter < k : k == steps);
    r.iter = -1;
  }
}

void prof_collect(m1_ctx* c) {
  Profiler& p = c->prof;
  prof_close(c);   // normally closed before the synchronisation that precedes this
  if (p.pending.empty()) return;
  hipEventSynchronize(p.pending.back().b);
  for (auto& r : p.pending) {
    float ms = 0.f;
    if (r.valid && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p.launches[r.kc] += r.n;
      p.ms[r.kc] += ms;
      p.bytes[r.kc] += r.bytes;
    }
  }
  p.pending.clear();
  p.used = 0;
}

int nu_of(const m1_config& c) { return 1 + c.ndim + (c.source == M1_SRC_COUPLED_T ? 1 : 0); }

bool finite(double v) { return std::isfinite(v); }

// M1_VERBOSE=1: one line per Newton iteration on stderr; 2: also every GMRES
// cycle and every line-search trial
int verbose() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("M1_VERBOSE");
    v = (e && e[0] >= '1' && e[0] <= '9') ? e[0] - '0' : 0;
  }
  return v;
}

m1_status validate_config(const m1_config* c, std::string& err) {
  if (!c) { err = "cfg is NULL"; return M1_ERR_INVALID_ARG; }
  if (c->ndim != 2 && c->ndim != 3) { err = "ndim must be 2 or 3"; return M1_ERR_INVALID_ARG; }
  int64_t N = 1;
  for (int d = 0; d < c->ndim; ++d) {
    if (c->n[d] < 1 || c->n[d] > (1 << 20)) { err = "grid size out of range"; return M1_ERR_INVALID_ARG; }
    N *= c->n[d];
  }
  if (N > (int64_t)1 << 31) { err = "too many cells (max 2^31)"; return M1_ERR_INVALID_ARG; }
  if (!(finite(c->dx) && c->dx > 0) || !(finite(c->c) && c->c > 0) || !(finite(c->a_r) && c->a_r > 0)) {
    err = "dx, c and a_r must be finite and > 0";
    return M1_ERR_INVALID_ARG;
  }
  if (c->source < 0 || c->source > 2 || c->flux_source < 0 || c->flux_source > 1 || c->closure < 0 ||
      c->closure > 1 || c->linearization < 0 || c->linearization > 1 || c->precision < 0 || c->precision > 1 ||
      c->pc < 0 || c->pc > 3) {
    err = "enum value out of range";
    return M1_ERR_INVALID_ARG;
  }
  if (c->pc == M1_PC_LEARNED && (c->ndim != 2 || c->source == M1_SRC_COUPLED_T)) {
    err = "the learned preconditioner is for 2D radiation-only problems";
    return M1_ERR_INVALID_ARG;
  }
  if (c->pc == M1_PC_MULTIGRID) {
    if (!(finite(c->mg_omega) && c->mg_omega > 0 && c->mg_omega < 2)) { err = "mg_omega must be in (0, 2)"; return M1_ERR_INVALID_ARG; }
    if (c->mg_nu1 < 0 || c->mg_nu1 > 16 || c->mg_nu2 < 0 || c->mg_nu2 > 16) { err = "mg_nu1 and mg_nu2 must be in 0..16"; return M1_ERR_INVALID_ARG; }
    if (c->mg_nu1_coarse < -1 || c->mg_nu1_coarse > 4 || c->mg_nu2_coarse < -1 || c->mg_nu2_coarse > 4) {
      err = "mg_nu1_coarse and mg_nu2_coarse must be in -1..4";
      return M1_ERR_INVALID_ARG;
    }
    if (c->mg_nmin != 0 && c->mg_nmin < 2) { err = "mg_nmin must be 0 or >= 2"; return M1_ERR_INVALID_ARG; }
  }
  if (c->wb_boundary != 0 && c->wb_boundary != 1) { err = "wb_boundary must be 0 or 1"; return M1_ERR_INVALID_ARG; }
  if (c->wb_boundary && c->flux_source != M1_FSRC_WELL_BALANCED) {
    err = "wb_boundary needs the well-balanced flux source";
    return M1_ERR_INVALID_ARG;
  }
  if (c->newton_flags & ~3) { err = "newton_flags: only bits 0 and 1 are defined"; return M1_ERR_INVALID_ARG; }
  if (!(finite(c->lambda_floor) && c->lambda_floor >= 0)) { err = "lambda_floor must be >= 0"; return M1_ERR_INVALID_ARG; }
  for (int f = 0; f < 2 * c->ndim; ++f) {
    if (c->bc[f] < 0 || c->bc[f] > 3) { err = "bc value out of range"; return M1_ERR_INVALID_ARG; }
  }
  for (int d = 0; d < c->ndim; ++d) {
    if ((c->bc[2 * d] == M1_BC_PERIODIC) != (c->bc[2 * d + 1] == M1_BC_PERIODIC)) {
      err = "periodic must be set on both faces of a direction";
      return M1_ERR_INVALID_ARG;
    }
  }
  if (c->restart < 1 || c->restart > kMaxRestart) { err = "restart must be in 1..48"; return M1_ERR_INVALID_ARG; }
  if (c->max_iters < 1 || c->newton_max < 1 || c->fixed_iters < 0) {
    err = "max_iters and newton_max must be >= 1, fixed_iters >= 0";
    return M1_ERR_INVALID_ARG;
  }
  if (!(finite(c->rtol) && c->rtol >= 0) || !(finite(c->newton_rtol) && c->newton_rtol >= 0) ||
      !(finite(c->inner_rtol) && c->inner_rtol >= 0 && c->inner_rtol < 1)) {
    err = "tolerances must be finite, >= 0 (inner_rtol < 1)";
    return M1_ERR_INVALID_ARG;
  }
  if (!(finite(c->ptc_psi0) && c->ptc_psi0 >= 0) || !(finite(c->ptc_rtol) && c->ptc_rtol >= 0 && c->ptc_rtol < 1) ||
      !(finite(c->positivity_clip) && c->positivity_clip >= 0 && c->positivity_clip < 1) ||
      !(finite(c->newton_forcing) && c->newton_forcing >= 0)) {
    err = "ptc_psi0 and newton_forcing must be finite and >= 0; ptc_rtol and positivity_clip in [0, 1)";
    return M1_ERR_INVALID_ARG;
  }
  return M1_OK;
}

__global__ void k_check(const double* a, int64_t n, int positive, unsigned long long* bad) {
  bool b = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = a[i];
    b = b || !isfinite(v) || (positive == 1 && !(v > 0.0)) || (positive == 2 && !(v >= 0.0)) ||
        (positive == 3 && !(v == 0.0 || v == 1.0));
  }
  const unsigned long long ballot = __ballot(b);
  if ((threadIdx.x & 63) == 0 && ballot) atomicAdd(bad, 1ull);
}

// Number of entries with !(a > 0) (E <= 0 or NaN) into cnt[0].
__global__ void k_count_nonpos(const double* a, int64_t n, unsigned long long* cnt) {
  unsigned long long local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    local += !(a[i] > 0.0) ? 1ull : 0ull;
  for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off, 64);
  if ((threadIdx.x & 63) == 0 && local) atomicAdd(cnt, local);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) p[0] = 0ull;
}

// Count entries that are non-finite (positive = 0), or also <= 0 (1), or < 0 (2),
// or other than 0 and 1 (3).
m1_status check_array(m1_ctx* c, const double* a, int64_t n, int positive, const char* name, m1_status code) {
  k_zero_u64<<<1, 64, 0, c->stream>>>(c->dcount);
  const int64_t grd = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
  k_check<<<grd, 256, 0, c->stream>>>(a, n, positive, c->dcount);
  unsigned long long bad = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, c->dcount, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) {
    c->err = std::string(name) + (positive == 1 ? " has non-finite or non-positive entries"
                                                : positive == 2 ? " has non-finite or negative entries"
                                                                : " has non-finite entries");
    return code;
  }
  return M1_OK;
}

template <typename T>
m1_status dalloc(m1_ctx* c, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return M1_OK;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
  if (e != hipSuccess) {
    c->err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
    *p = nullptr;
    return e == hipErrorOutOfMemory ? M1_ERR_OUT_OF_MEMORY : M1_ERR_HIP;
  }
  return M1_OK;
}

void free_all(m1_ctx* c) {
  for (int f = 0; f < 6; ++f) {
    if (c->plane[f]) hipFree(c->plane[f]);
    if (c->mask[f]) hipFree(c->mask[f]);
  }
  void* bufs[] = {c->Uk, c->Un, c->Uprev, c->fn, c->coef64, c->coef32, c->V, c->b, c->x, c->u[0], c->u[1],
                  c->p, c->z, c->part, c->gs, c->dscal, c->dcount, c->Z, c->xw,
                  c->mg.Ainv64, c->mg.Ainv32, c->mg.work, c->mg.bad};
  for (void* b : bufs)
    if (b) hipFree(b);
  for (int l = 0; l < c->mg.nlev; ++l) {
    MgLevel& L = c->mg.lev[l];
    void* lb[] = {L.S64, L.S32, L.Dinv64, L.Dinv32, L.b, L.z, L.w, L.t};
    for (void* b : lb)
      if (b) hipFree(b);
  }
  if (c->hscal) hipHostFree(c->hscal);
  for (auto e : c->prof.pool) hipEventDestroy(e);
}

bool mixed(const m1_ctx* c) { return c->cfg.precision == M1_MIXED; }
bool basis32(const m1_ctx* c) { return mixed(c) && c->cfg.basis_fp32; }

template <typename R> void layout(m1_ctx* c, R* base, Coefs<R>& cf) {
  const int64_t N = c->g.N;
  int64_t off = 0;
  cf.jac = base + off; off += (int64_t)c->njac * N;
  cf.face = base + off; off += (int64_t)3 * c->nd * N;
  cf.lowface = base;
  for (int d = 0; d < c->nd; ++d) { cf.lowoff[d] = off; off += (int64_t)3 * c->g.plane_n[d]; }
  cf.gjac = base;
  for (int f = 0; f < 6; ++f) {
    cf.gjoff[f] = off;
    if (f < 2 * c->nd) off += (int64_t)c->njac * c->g.plane_n[f / 2];
  }
  cf.sigma = base + off; off += N;
  cf.kap = base + off; off += c->cpl ? N : 0;
  cf.rcv = base + off; off += c->cpl ? N : 0;
  cf.bjinv = base + off; off += (int64_t)c->nu * c->nu * N;
  c->coef_len = off;
}

// ---- algorithmic bytes per launch (per cell: every array element touched once) ----
double cells(const m1_ctx* c) { return (double)c->g.N; }
double bytes_apply(const m1_ctx* c, size_t rs, size_t vin, size_t vout, bool with_b) {
  const double per = c->nu * (double)(vin + vout) + (c->njac + 3.0 * c->nd + 1.0 + (c->cpl ? 2.0 : 0.0)) * rs +
                     (with_b ? c->nu * 8.0 : 0.0);
  return per * cells(c);
}
double bytes_bj(const m1_ctx* c, size_t rs, size_t vin, size_t vout) {
  return (c->nu * (double)(vin + vout) + (double)c->nu * c->nu * rs) * cells(c);
}
double bytes_setup(const m1_ctx* c) {
  return ((c->nrad + 2.0 + (c->cpl ? 1.0 : 0.0)) + (c->njac + 3.0 * c->nd + (c->cpl ? 1.0 : 0.0))) * 8.0 * cells(c);
}
double bytes_setup_bj(const m1_ctx* c) {
  return ((c->njac + 3.0 * c->nd + 1.0 + (c->cpl ? 2.0 : 0.0)) + (double)c->nu * c->nu) * 8.0 * cells(c);
}
double bytes_residual(const m1_ctx* c) {
  return (3.0 * c->nu + 3.0 * c->nd + 1.0 + (c->cpl ? 1.0 : 0.0)) * 8.0 * cells(c);
}

Bdry bdry(const m1_ctx* c) {
  Bdry b;
  for (int f = 0; f < 6; ++f) {
    b.plane[f] = c->plane[f];
    b.mask[f] = c->mask[f];
  }
  return b;
}

// grid sizes, strides, boundary kinds and plane sizes of a validated configuration
void fill_geom(const m1_config& cfg, Geom& g) {
  const int nd = cfg.ndim;
  g.n[0] = (int)cfg.n[0];
  g.n[1] = (int)cfg.n[1];
  g.n[2] = nd == 3 ? (int)cfg.n[2] : 1;
  g.rows = g.n[1] * g.n[2];
  g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
  g.stride[0] = 1;
  g.stride[1] = g.n[0];
  g.stride[2] = (int64_t)g.n[0] * g.n[1];
  for (int f = 0; f < 6; ++f) g.bc[f] = f < 2 * nd ? cfg.bc[f] : M1_BC_PERIODIC;
  g.plane_n[0] = g.n[1] * g.n[2];
  g.plane_n[1] = g.n[0] * g.n[2];
  g.plane_n[2] = g.n[0] * g.n[1];
  g.order3d = 0;
}

// scheme constants of a validated configuration (dt-derived ones left to set_dt)
void fill_scheme(const m1_config& cfg, Scheme& sc) {
  sc.c = cfg.c;
  sc.c2 = cfg.c * cfg.c;
  sc.a_r = cfg.a_r;
  sc.dx = cfg.dx;
  sc.dx_c = cfg.dx / cfg.c;
  sc.lambda_floor = cfg.lambda_floor;
  sc.src = cfg.source;
  sc.wb = cfg.flux_source == M1_FSRC_WELL_BALANCED;
  sc.ap = cfg.ap_correction != 0;
  sc.p1 = cfg.closure == M1_CLOSURE_P1;
  sc.newton = cfg.linearization == M1_LIN_NEWTON;
  sc.psi = 0.0;
  sc.wbb = cfg.wb_boundary;
  sc.inv_cdx = 1.0 / (cfg.c * cfg.dx);
}

void set_dt(m1_ctx* c, double dt) {
  c->sc.dt = dt;
  c->sc.s = dt / c->cfg.dx;
  c->sc.cdt = c->cfg.c * dt;
}

m1_status copy_state_in(m1_ctx* c, const m1_state* U, double* dst) {
  const size_t bytes = sizeof(double) * (size_t)c->g.N;
  if (!U || !U->E) { c->err = "state E is NULL"; return M1_ERR_INVALID_ARG; }
  for (int d = 0; d < c->nd; ++d)
    if (!U->F[d]) { c->err = "state F[d] is NULL"; return M1_ERR_INVALID_ARG; }
  if (c->cpl && !U->T) { c->err = "state T is NULL (coupled source)"; return M1_ERR_INVALID_ARG; }
  HIPCHK(c, hipMemcpyAsync(dst, U->E, bytes, hipMemcpyDeviceToDevice, c->stream));
  for (int d = 0; d < c->nd; ++d)
    HIPCHK(c, hipMemcpyAsync(dst + (1 + d) * c->g.N, U->F[d], bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->cpl) HIPCHK(c, hipMemcpyAsync(dst + (1 + c->nd) * c->g.N, U->T, bytes, hipMemcpyDeviceToDevice, c->stream));
  return M1_OK;
}

m1_status copy_state_out(m1_ctx* c, const double* src, m1_state* U) {
  const size_t bytes = sizeof(double) * (size_t)c->g.N;
  HIPCHK(c, hipMemcpyAsync(U->E, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  for (int d = 0; d < c->nd; ++d)
    HIPCHK(c, hipMemcpyAsync(U->F[d], src + (1 + d) * c->g.N, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->cpl) HIPCHK(c, hipMemcpyAsync(U->T, src + (1 + c->nd) * c->g.N, bytes, hipMemcpyDeviceToDevice, c->stream));
  return M1_OK;
}

// ---- aggregation multigrid: hierarchy sizes, algorithmic bytes, finest-level operator ----
int mg_default_nmin(int nd) { return nd == 2 ? 8 : 4; }

// level extents: halve (rounding up) until every extent is <= nmin
void mg_levels(const m1_ctx* c, MgHierarchy& h) {
  const int nmin = c->cfg.mg_nmin > 0 ? c->cfg.mg_nmin : mg_default_nmin(c->nd);
  MgGeom g{};
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c->g.n[d];
    g.per[d] = d < c->nd && c->g.bc[2 * d] == M1_BC_PERIODIC;
  }
  h.nlev = 0;
  while (true) {
    g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    h.lev[h.nlev++].g = g;
    if (std::max(g.n[0], std::max(g.n[1], g.n[2])) <= nmin || h.nlev == kMgMaxLevels) break;
    for (int d = 0; d < 3; ++d) g.n[d] = (g.n[d] + 1) / 2;
  }
}

double mg_setup_bytes(const m1_ctx* c) {
  const MgHierarchy& h = c->mg;
  const double nu = c->nu, nb = 1 + 2 * c->nd;
  double b = bytes_setup_bj(c) + nb * nu * nu * 8.0 * cells(c);
  for (int l = 1; l < h.nlev; ++l) b += (nb * nu * nu + nu * nu) * 8.0 * (double)h.lev[l].g.N;
  return b;
}

template <typename R> const Coefs<R>& coefs_of(const m1_ctx* c);
template <> const Coefs<double>& coefs_of<double>(const m1_ctx* c) { return c->cf64; }
template <> const Coefs<float>& coefs_of<float>(const m1_ctx* c) { return c->cf32; }

template <typename R>
void mg_fine_apply(const void* self, const R* x, R* y, hipStream_t s, const int* skip) {
  const m1_ctx* c = (const m1_ctx*)self;
  launch_apply<R, R, R>(c->nd, c->cpl, 0, c->g, c->sc, coefs_of<R>(c), bdry(c), x, nullptr, y, s, skip);
}

template <typename R>
bool mg_fine_sweep(const void* self, int op, int xin, int ns, const void* r, int r_fp64, const R* zin, const R* zc,
                   R omega, R* out, const R* dinv1, int sm, R* b1, R* z1, hipStream_t s, const int* skip) {
  const m1_ctx* c = (const m1_ctx*)self;
  if (r_fp64)
    return launch_mg_sweep2d<R, double>(c->nd, c->cpl, op, xin, ns, c->g, c->sc, coefs_of<R>(c), bdry(c),
                                        (const double*)r, zin, zc, omega, out, dinv1, sm, b1, z1, s, skip);
  if constexpr (std::is_same<R, float>::value)
    return launch_mg_sweep2d<float, float>(c->nd, c->cpl, op, xin, ns, c->g, c->sc, coefs_of<float>(c), bdry(c),
                                           (const float*)r, zin, zc, omega, out, dinv1, sm, b1, z1, s, skip);
  return false;
}

template <typename R> MgFine<R> mg_fine(const m1_ctx* c) {
  MgFine<R> f;
  f.nd = c->nd;
  f.nu = c->nu;
  f.apply_bytes = bytes_apply(c, sizeof(R), sizeof(R), sizeof(R), false);
  f.coef_bytes = bytes_apply(c, sizeof(R), 0, 0, false);
  f.bjinv = coefs_of<R>(c).bjinv;
  f.apply = &mg_fine_apply<R>;
  f.sweep = fused_apply_available(c->nd) ? &mg_fine_sweep<R> : nullptr;
  f.self = c;
  return f;
}

// Linearise at c->Uk with time-level state c->Un (|f^n| already in c->fn).
// block-Jacobi inverses of the current coefficients with the current shift
// sc.psi, then the FP32 shadow of the whole slab (mixed precision)
m1_status build_bj(m1_ctx* c) {
  const Bdry bd = bdry(c);
  timed(c, KC_SETUP_BJ, bytes_setup_bj(c), [&] { launch_setup_bj(c->nd, c->cpl, c->g, c->sc, c->cf64, bd, c->stream); });
  if (mixed(c)) timed(c, KC_CONVERT, 12.0 * c->coef_len, [&] { launch_convert(c->coef64, c->coef32, c->coef_len, c->stream); });
  if (c->cfg.pc == M1_PC_MULTIGRID) {
    MgHierarchy& h = c->mg;
    const int nb = 1 + 2 * c->nd, bs = c->nu * c->nu;
    timed(c, KC_MG_SETUP, mg_setup_bytes(c), [&] {
      launch_fine_stencil(c->nd, c->cpl, c->g, c->sc, c->cf64, bd, h.lev[0].S64, c->stream);
      mg_build(h, c->nd, c->nu, c->stream);
      if (mixed(c)) {
        for (int l = 1; l < h.nlev; ++l) {
          launch_convert(h.lev[l].S64, h.lev[l].S32, (int64_t)nb * bs * h.lev[l].g.N, c->stream);
          if (h.lev[l].Dinv64) launch_convert(h.lev[l].Dinv64, h.lev[l].Dinv32, (int64_t)bs * h.lev[l].g.N, c->stream);
        }
        const int64_t nc = (int64_t)c->nu * h.lev[h.nlev - 1].g.N;
        launch_convert(h.Ainv64, h.Ainv32, nc * nc, c->stream);
      }
    });
  }
  HIPCHK(c, hipGetLastError());
  c->bj_ready = true;
  c->bj_psi = c->sc.psi;
  return M1_OK;
}

m1_status ensure_bj(m1_ctx* c) {
  if (c->bj_ready && c->bj_psi == c->sc.psi) return M1_OK;
  return build_bj(c);
}

// closure and face coefficients at c->Uk (a1); with_bj also builds the
// block-Jacobi inverses (else they are built on first use)
m1_status linearize_internal(m1_ctx* c, bool with_bj = true) {
  const Bdry bd = bdry(c);
  timed(c, KC_SETUP, bytes_setup(c), [&] { launch_setup(c->nd, c->cpl, c->g, c->sc, c->cf64, bd, c->Uk, c->Un, c->fn, c->stream); });
  HIPCHK(c, hipGetLastError());
  c->linearized = true;
  c->bj_ready = false;
  if (with_bj) return build_bj(c);
  return M1_OK;
}

// ||v||^2 of an FP64 vector into c->dscal[slot] (device)
void norm2_into(m1_ctx* c, const double* v, int slot) {
  timed(c, KC_NORM, 8.0 * c->n, [&] {
    launch_dot<double>(0, nullptr, 0, v, nullptr, c->n, c->part, c->nb, nullptr, c->stream);
    launch_reduce(c->part, 1, c->nb, c->dscal + slot, c->stream);
  });
}

struct SolveResult {
  int iters = 0, restarts = 0;
  double rel = 0.0;
  bool converged = false;
  bool nonfinite = false;
};

// GMRES(m) on A x = b (b = c->b, x = c->x), x0 = 0.  TV: basis storage; R: type of
// the preconditioner and of the operator inside the Arnoldi process.
template <typename TV, typename R>
m1_status gmres(m1_ctx* c, double bnorm, SolveResult& res, const Coefs<R>& cfi) {
  const Bdry bd = bdry(c);
  const int64_t n = c->n;
  const int64_t vs = c->vs;
  TV* V = (TV*)c->V;
  TV* u[2] = {(TV*)c->u[0], (TV*)c->u[1]};
  TV* p = (TV*)c->p;
  R* z = (R*)c->z;
  const bool fixed = c->cfg.fixed_iters > 0;
  const int budget = fixed ? c->cfg.fixed_iters : c->cfg.max_iters;
  const double rtol = c->lin_rtol >= 0 ? c->lin_rtol : c->cfg.rtol;
  const double tol_rel = (mixed(c) && !fixed) ? c->cfg.inner_rtol : 0.0;
  const bool learned = c->use_learned && c->net;
  const int use_pc = !learned && c->cfg.pc != M1_PC_NONE;
  const bool use_mg = use_pc && c->cfg.pc == M1_PC_MULTIGRID;
  const bool fused = use_pc && !use_mg && fused_apply_available(c->nd);
  const MgFine<R> mgf = mg_fine<R>(c);
  R* Z = (R*)c->Z;
  HIPCHK(c, hipMemsetAsync(c->x, 0, sizeof(double) * n, c->stream));
  // r = b
  launch_copy_cast<double, TV>(c->b, u[0], n, c->stream);
  double beta = bnorm;
  // device copy of beta^2 for the cycle's relative tolerance
  HIPCHK(c, hipMemcpyAsync(c->dscal + 1, c->dscal + 0, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  int total = 0, cycles = 0;
  res = SolveResult();
  while (true) {
    if (!fixed && beta <= rtol * bnorm) { res.converged = true; break; }
    if (total >= budget) { res.converged = fixed || beta <= rtol * bnorm; break; }
    ++cycles;
    const int steps = std::min(c->m, budget - total);
    launch_cycle_init(c->gs, c->dscal + 1, fixed ? 0.0 : rtol * bnorm, tol_rel, c->stream);
    if (learned) {
      // Flexible GMRES in the standard Arnoldi order: the network is nonlinear, so it
      // is applied to the orthonormal v_j (the delayed one-reduction form applies the
      // preconditioner before orthogonalisation and would scale the network's
      // nonlinear part by ||u_j||/nu).  V_0 = r/beta, then per iteration: z_j = P(v_j)
      // stored as Z_j, w = A z_j, one reduction over [V_0..V_j, w], the Hessenberg
      // column, and v_{j+1} = (w - V s)/nu.
      timed(c, KC_DOT, 1.0 * n * sizeof(TV), [&] { launch_dot<TV>(0, V, vs, u[0], nullptr, n, c->part, c->nb, c->gs, c->stream); }, 0, 0);
      timed(c, KC_SCALAR, c->nb * 8.0, [&] { launch_scalar(0, 0, c->part, c->nb, c->gs, c->stream, 1); }, 0, 0);
      timed(c, KC_UPDATE, 4.0 * n * sizeof(TV), [&] { launch_update<TV>(0, V, vs, u[0], u[0], u[1], n, c->gs, c->stream); }, 0, 1);
      for (int j = 0; j < steps; ++j) {
        TV* vj = V + (int64_t)j * vs;
        R* zj = Z + (int64_t)j * vs;
        // the network on the cycle's first direction (the normalised restart residual,
        // the kind of input it is trained on), block-Jacobi on the Krylov directions
        if (j > 0) {
          timed(c, KC_BJ, bytes_bj(c, sizeof(R), sizeof(TV), sizeof(R)), [&] { launch_bj<R, TV, R>(c->nd, c->cpl, c->g, cfi, vj, zj, c->stream, &c->gs->done); }, j, 0);
        } else timed(c, KC_NN, 0.0, [&] {
          launch_dot<TV>(0, nullptr, 0, vj, nullptr, n, c->part, c->nb, c->gs, c->stream);
          launch_reduce(c->part, 1, c->nb, c->dscal + 2, c->stream);
          launch_nn_features<TV>(c->g.N, vj, c->dscal + 2, c->cf64.bjinv, c->Uk, c->cf64.sigma, c->cfg.c, c->sc.cdt,
                                 nn_cin_pad(c->net), nn_input(c->net), nullptr, c->stream, &c->gs->done);
          nn_run(c->net, c->g.n[1], c->g.n[0], c->stream, &c->gs->done);
          launch_nn_combine<TV, R>(c->g.N, vj, c->dscal + 2, c->cf64.bjinv, nn_output(c->net), zj, c->stream,
                                   &c->gs->done);
        }, j, 0);
        timed(c, KC_APPLY, bytes_apply(c, sizeof(R), sizeof(R), sizeof(TV), false), [&] { launch_apply<R, R, TV>(c->nd, c->cpl, 0, c->g, c->sc, cfi, bd, zj, nullptr, p, c->stream, &c->gs->done); }, j, 0);
        timed(c, KC_DOT, (j + 2.0) * n * sizeof(TV), [&] { launch_dot<TV>(j + 1, V, vs, p, nullptr, n, c->part, c->nb, c->gs, c->stream); }, j, 0);
        timed(c, KC_SCALAR, (j + 2.0) * c->nb * 8.0, [&] { launch_scalar(j + 1, j == steps - 1 ? 1 : 0, c->part, c->nb, c->gs, c->stream, 1); }, j, 0);
        if (j < steps - 1)
          timed(c, KC_UPDATE, (j + 4.0) * n * sizeof(TV), [&] { launch_update<TV>(j + 1, V, vs, p, p, u[1], n, c->gs, c->stream); }, j, 1);
      }
    }
    for (int j = 0; j < (learned ? 0 : steps); ++j) {
      TV* uj = u[j & 1];
      TV* un = u[(j + 1) & 1];
      if (fused) {
        // fused: p = A M^{-1} u_j (block-Jacobi applied while staging the halo tile)
        timed(c, KC_APPLY_PC, bytes_apply(c, sizeof(R), sizeof(TV), sizeof(TV), false) +
                                  (double)c->nu * c->nu * sizeof(R) * cells(c), [&] {
          launch_apply_pre<R, TV, TV>(c->nd, c->cpl, c->g, c->sc, cfi, bd, uj, p, c->stream, &c->gs->done);
        }, j, 0);
      } else if (use_mg) {
        const MgWrap wrap = [&](int kc, double bytes, const std::function<void()>& launch) { timed(c, kc, bytes, launch, j, 0); };
        mg_vcycle<R, TV>(c->mg, mgf, uj, z, c->stream, &c->gs->done, c->prof.on ? &wrap : nullptr);
        timed(c, KC_APPLY, bytes_apply(c, sizeof(R), sizeof(R), sizeof(TV), false), [&] { launch_apply<R, R, TV>(c->nd, c->cpl, 0, c->g, c->sc, cfi, bd, z, nullptr, p, c->stream, &c->gs->done); }, j, 0);
      } else if (use_pc) {
        timed(c, KC_BJ, bytes_bj(c, sizeof(R), sizeof(TV), sizeof(R)), [&] { launch_bj<R, TV, R>(c->nd, c->cpl, c->g, cfi, uj, z, c->stream, &c->gs->done); }, j, 0);
        timed(c, KC_APPLY, bytes_apply(c, sizeof(R), sizeof(R), sizeof(TV), false), [&] { launch_apply<R, R, TV>(c->nd, c->cpl, 0, c->g, c->sc, cfi, bd, z, nullptr, p, c->stream, &c->gs->done); }, j, 0);
      } else {
        timed(c, KC_APPLY, bytes_apply(c, sizeof(R), sizeof(TV), sizeof(TV), false), [&] { launch_apply<R, TV, TV>(c->nd, c->cpl, 0, c->g, c->sc, cfi, bd, uj, nullptr, p, c->stream, &c->gs->done); }, j, 0);
      }
      timed(c, KC_DOT, (j + 2.0) * n * sizeof(TV), [&] { launch_dot<TV>(j, V, vs, uj, p, n, c->part, c->nb, c->gs, c->stream); }, j, 0);
      timed(c, KC_SCALAR, (2.0 * j + 2.0) * c->nb * 8.0, [&] { launch_scalar(j, 0, c->part, c->nb, c->gs, c->stream); }, j, 0);
      timed(c, KC_UPDATE, (j + 4.0) * n * sizeof(TV), [&] { launch_update<TV>(j, V, vs, uj, p, un, n, c->gs, c->stream); }, j, 1);
    }
    if (!learned) {
      timed(c, KC_DOT, (steps + 1.0) * n * sizeof(TV), [&] { launch_dot<TV>(steps, V, vs, u[steps & 1], nullptr, n, c->part, c->nb, c->gs, c->stream); }, steps, 2);
      timed(c, KC_SCALAR, (steps + 1.0) * c->nb * 8.0, [&] { launch_scalar(steps, 1, c->part, c->nb, c->gs, c->stream); }, steps, 2);
    }
    if (learned) {
      timed(c, KC_XUPDATE, (double)steps * n * sizeof(R) + 16.0 * n, [&] { launch_xupdate<R, R>(c->nd, c->cpl, c->g, cfi, Z, vs, c->gs, c->x, 0, c->stream); });
    } else if (use_mg) {
      // x += M^{-1} (V y): V y into xw, one cycle, then the FP64 update
      HIPCHK(c, hipMemsetAsync(c->xw, 0, sizeof(double) * n, c->stream));
      timed(c, KC_XUPDATE, (double)steps * n * sizeof(TV) + 16.0 * n, [&] { launch_xupdate<R, TV>(c->nd, c->cpl, c->g, cfi, V, vs, c->gs, c->xw, 0, c->stream); });
      {
        const MgWrap wrap = [&](int kc, double bytes, const std::function<void()>& launch) { timed(c, kc, bytes, launch); };
        mg_vcycle<R, double>(c->mg, mgf, c->xw, z, c->stream, nullptr, c->prof.on ? &wrap : nullptr);
        prof_close(c);
      }
      mg_axpy<R>(z, c->x, n, c->stream);
    } else {
      timed(c, KC_XUPDATE, (double)steps * n * sizeof(TV) + 16.0 * n + (use_pc ? (double)c->nu * c->nu * sizeof(R) * cells(c) : 0.0), [&] { launch_xupdate<R, TV>(c->nd, c->cpl, c->g, cfi, V, vs, c->gs, c->x, use_pc, c->stream); });
    }
    // true residual in FP64: r = b - A x, stored as the next cycle's u_0
    timed(c, KC_TRUE_RESID, bytes_apply(c, 8, 8, sizeof(TV), true), [&] {
      launch_apply<double, double, TV>(c->nd, c->cpl, 1, c->g, c->sc, c->cf64, bd, c->x, c->b, u[0], c->stream);
    });
    timed(c, KC_NORM, (double)n * sizeof(TV), [&] {
      launch_dot<TV>(0, nullptr, 0, u[0], nullptr, n, c->part, c->nb, nullptr, c->stream);
      launch_reduce(c->part, 1, c->nb, c->dscal + 1, c->stream);
    });
    HIPCHK(c, hipGetLastError());
    prof_close(c);
    HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int hk[4];
    HIPCHK(c, hipMemcpyAsync(hk, c->gs, sizeof(int) * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int k = hk[1];
    prof_resolve(c, k, steps);
    prof_collect(c);
    total += fixed ? steps : std::max(k, 1);
    beta = std::sqrt(std::max(c->hscal[0], 0.0));
    if (verbose() > 1)
      std::fprintf(stderr, "[m1]     cycle %d: k=%d true |r|/|b|=%.3e done=%d breakdown=%d nonfinite=%d\n", cycles, k,
                   bnorm > 0 ? beta / bnorm : 0.0, hk[0], hk[2], hk[3]);
    if (!std::isfinite(beta) || hk[3]) { res.nonfinite = true; break; }
  }
  res.iters = total;
  res.restarts = std::max(cycles - 1, 0);
  res.rel = bnorm > 0 ? beta / bnorm : 0.0;
  return M1_OK;
}

m1_status solve_once(m1_ctx* c, double bnorm, SolveResult& res) {
  if (!mixed(c)) return gmres<double, double>(c, bnorm, res, c->cf64);
  if (basis32(c)) return gmres<float, float>(c, bnorm, res, c->cf32);
  return gmres<double, float>(c, bnorm, res, c->cf32);
}

// The learned preconditioner runs first when attached; if its solve fails
// (iteration cap or non-finite values) block-Jacobi redoes the solve.
m1_status solve(m1_ctx* c, double bnorm, SolveResult& res, int& fell_back) {
  c->use_learned = (c->cfg.pc == M1_PC_LEARNED && c->net) ? 1 : 0;
  m1_status st = solve_once(c, bnorm, res);
  if (st != M1_OK) return st;
  if (c->use_learned && (!res.converged || res.nonfinite)) {
    const int it = res.iters;
    c->use_learned = 0;
    st = solve_once(c, bnorm, res);
    res.iters += it;
    fell_back = 1;
  }
  c->use_learned = 0;
  return st;
}

}  // namespace

// nsteps explicit (semi = false) or semi-implicit steps, one fused kernel each
// (a1, a2 and the update), ping-ponging between the context's two work vectors
// b and x, so the linearisation held in Uk, Un and the coefficient slab stays.
m1_status time_steps(m1_ctx* c, m1_state* U, double dt, int32_t nsteps, m1_stats* stats, bool semi) {
  if (!c) return M1_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  if (!(std::isfinite(dt) && dt > 0)) { c->err = "dt must be finite and > 0"; return M1_ERR_INVALID_ARG; }
  if (nsteps < 1) { c->err = "nsteps must be >= 1"; return M1_ERR_INVALID_ARG; }
  if (semi && c->cfg.flux_source != M1_FSRC_CENTERED) {
    c->err = "the semi-implicit step needs the centred flux source (the well-balanced source couples cells)";
    return M1_ERR_INVALID_ARG;
  }
  if (c->cfg.wb_boundary) {
    c->err = "the explicit steps do not implement the boundary closure (wb_boundary)";
    return M1_ERR_INVALID_ARG;
  }
  m1_status st;
  double* src = c->b;
  double* dst = c->x;
  if ((st = copy_state_in(c, U, src)) != M1_OK) return st;
  if ((st = check_array(c, src, c->n, 0, "U", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = check_array(c, src, c->g.N, 1, "U.E", M1_ERR_INVALID_ARG)) != M1_OK) return st;
  // the step kernels read only dt-derived scalars of the scheme; the context's own are kept
  Scheme sc = c->sc;
  sc.dt = dt;
  sc.s = dt / c->cfg.dx;
  sc.cdt = c->cfg.c * dt;
  sc.psi = 0.0;
  const Bdry bd = bdry(c);
  const double bytes = 8.0 * (2.0 * c->nu + 1.0 + (c->cpl ? 1.0 : 0.0)) * cells(c);
  for (int32_t k = 0; k < nsteps; ++k) {
    timed(c, KC_TIME_STEP, bytes, [&] { launch_time_step(c->nd, c->cpl, semi, c->g, sc, c->cf64, bd, src, dst, c->stream); });
    std::swap(src, dst);
  }
  HIPCHK(c, hipGetLastError());
  unsigned long long nf = 0;
  k_zero_u64<<<1, 64, 0, c->stream>>>(c->dcount);
  launch_count_f(c->nd, c->g, src, c->cfg.c, c->dcount, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(&nf, c->dcount, sizeof(nf), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  if ((st = check_array(c, src, c->n, 0, "U^(n+nsteps)", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = copy_state_out(c, src, U)) != M1_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (stats) {
    stats->newton_iters = 0;
    stats->krylov_iters = 0;
    stats->restarts = 0;
    stats->fell_back = 0;
    stats->rel_residual = 0.0;
    stats->nonlinear_residual = 0.0;
    stats->cells_f_gt_1 = (int64_t)nf;
    stats->cells_e_nonpos = 0;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return M1_OK;
}

// step 3 of the splitting: the velocity-dependent sources, explicitly, on the
// context's work vectors b (in) and x (out) so the linearisation stays
m1_status velocity_sources(m1_ctx* c, m1_state* U, const double* ux, const double* uy, const double* uz, double dt,
                           m1_stats* stats) {
  if (!c) return M1_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  if (!(std::isfinite(dt) && dt > 0)) { c->err = "dt must be finite and > 0"; return M1_ERR_INVALID_ARG; }
  const double* u[3] = {ux, uy, uz};
  for (int d = 0; d < c->nd; ++d)
    if (!u[d]) { c->err = "velocity component is NULL"; return M1_ERR_INVALID_ARG; }
  m1_status st;
  if ((st = copy_state_in(c, U, c->b)) != M1_OK) return st;
  if ((st = check_array(c, c->b, c->n, 0, "U", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = check_array(c, c->b, c->g.N, 1, "U.E", M1_ERR_INVALID_ARG)) != M1_OK) return st;
  for (int d = 0; d < c->nd; ++d)
    if ((st = check_array(c, u[d], c->g.N, 0, "u", M1_ERR_NONFINITE)) != M1_OK) return st;
  const double bytes = 8.0 * (2.0 * c->nu + 1.0 + c->nd) * cells(c);
  timed(c, KC_VELOCITY, bytes, [&] {
    launch_velocity_sources(c->nd, c->cpl, c->g, c->sc, c->cf64.sigma, c->b, u, dt, c->x, c->stream);
  });
  HIPCHK(c, hipGetLastError());
  unsigned long long nf = 0;
  k_zero_u64<<<1, 64, 0, c->stream>>>(c->dcount);
  launch_count_f(c->nd, c->g, c->x, c->cfg.c, c->dcount, c->stream);
  HIPCHK(c, hipMemcpyAsync(&nf, c->dcount, sizeof(nf), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  if ((st = check_array(c, c->x, c->n, 0, "U after the velocity sources", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = copy_state_out(c, c->x, U)) != M1_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (stats) {
    *stats = m1_stats{};
    stats->cells_f_gt_1 = (int64_t)nf;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return M1_OK;
}

// ============================================================================
// Explicit / semi-implicit steps that allocate nothing.  Their work memory (two
// state buffers for the ping-pong and a counter) is the file-scope array
// `scratch` below, whose device address is looked up once per device with
// hipGetSymbolAddress; host code only ever passes that address on (the array's
// name in host code is a host-side stand-in, not a device pointer).
// ============================================================================
constexpr int64_t kNoAllocMaxVector = int64_t(1) << 22;   // n_u * N <= 4 Mi doubles (32 MiB)
constexpr int64_t kNoAllocCounterOff = 2 * kNoAllocMaxVector;
constexpr int64_t kScratchDoubles = kNoAllocCounterOff + 32; // + 256 B for the counter
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
m1_status scratch_on_device(double** out, std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  if (dev < 0 || dev >= kMaxDevices) { err = "device index beyond the supported range"; return M1_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return M1_ERR_HIP;
    }
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return M1_OK;
}

// count of entries of a[0..n) failing k_check's `mode` test, through the scratch counter
m1_status noalloc_check(const double* a, int64_t n, int mode, unsigned long long* cnt, hipStream_t s,
                        unsigned long long& bad, std::string& err) {
  k_zero_u64<<<1, 64, 0, s>>>(cnt);
  const int64_t grd = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
  k_check<<<grd, 256, 0, s>>>(a, n, mode, cnt);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { err = std::string("check: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  return M1_OK;
}

m1_status time_steps_noalloc(const m1_config* cfg, const m1_fields* fields, m1_state* U, double dt,
                             int32_t nsteps, int32_t semi, void* hip_stream, m1_stats* stats, std::string& err) {
  const auto t0 = std::chrono::steady_clock::now();
  m1_status st = validate_config(cfg, err);
  if (st != M1_OK) return st;
  if (!fields || !fields->sigma) { err = "fields or fields->sigma is NULL"; return M1_ERR_INVALID_ARG; }
  const bool cpl = cfg->source == M1_SRC_COUPLED_T;
  if (cpl && !fields->rho_cv) { err = "rho_cv is NULL"; return M1_ERR_INVALID_ARG; }
  for (int f = 0; f < 2 * cfg->ndim; ++f)
    if (cfg->bc[f] == M1_BC_DIRICHLET && !fields->bc_ghost[f]) { err = "Dirichlet face without bc_ghost"; return M1_ERR_INVALID_ARG; }
  if (!(std::isfinite(dt) && dt > 0)) { err = "dt must be finite and > 0"; return M1_ERR_INVALID_ARG; }
  if (nsteps < 1) { err = "nsteps must be >= 1"; return M1_ERR_INVALID_ARG; }
  if (semi != 0 && semi != 1) { err = "semi must be 0 or 1"; return M1_ERR_INVALID_ARG; }
  if (semi && cfg->flux_source != M1_FSRC_CENTERED) {
    err = "the semi-implicit step needs the centred flux source (the well-balanced source couples cells)";
    return M1_ERR_INVALID_ARG;
  }
  if (cfg->wb_boundary) {
    err = "the explicit steps do not implement the boundary closure (wb_boundary)";
    return M1_ERR_INVALID_ARG;
  }
  const int nd = cfg->ndim;
  if (!U || !U->E) { err = "state E is NULL"; return M1_ERR_INVALID_ARG; }
  for (int d = 0; d < nd; ++d)
    if (!U->F[d]) { err = "state F[d] is NULL"; return M1_ERR_INVALID_ARG; }
  if (cpl && !U->T) { err = "state T is NULL (coupled source)"; return M1_ERR_INVALID_ARG; }
  Geom g;
  fill_geom(*cfg, g);
  const int nu = nu_of(*cfg);
  const int64_t N = g.N;
  const int64_t n = (int64_t)nu * N;
  if (n > kNoAllocMaxVector) {
    err = "n_u * N = " + std::to_string(n) + " exceeds the no-allocation limit of " +
          std::to_string(kNoAllocMaxVector) + " values";
    return M1_ERR_INVALID_ARG;
  }
  double* base = nullptr;
  if ((st = scratch_on_device(&base, err)) != M1_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  double* src = base;
  double* dst = base + kNoAllocMaxVector;
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + kNoAllocCounterOff);
  unsigned long long bad = 0;
  // the caller's fields are used in place: validate them as m1_setup does
  if ((st = noalloc_check(fields->sigma, N, 2, cnt, s, bad, err)) != M1_OK) return st;
  if (bad) { err = "sigma has non-finite or negative entries"; return M1_ERR_NONFINITE; }
  if (cpl) {
    if ((st = noalloc_check(fields->rho_cv, N, 1, cnt, s, bad, err)) != M1_OK) return st;
    if (bad) { err = "rho_cv has non-finite or non-positive entries"; return M1_ERR_NONFINITE; }
  }
  Bdry bd{};
  for (int f = 0; f < 2 * nd; ++f) {
    if (g.bc[f] != M1_BC_DIRICHLET) continue;
    const int64_t pn = g.plane_n[f / 2];
    if ((st = noalloc_check(fields->bc_ghost[f], (int64_t)(1 + nd) * pn, 0, cnt, s, bad, err)) != M1_OK) return st;
    if (bad) { err = "bc_ghost has non-finite entries"; return M1_ERR_NONFINITE; }
    bd.plane[f] = fields->bc_ghost[f];
    if (fields->bc_mask[f]) {
      if ((st = noalloc_check(fields->bc_mask[f], pn, 3, cnt, s, bad, err)) != M1_OK) return st;
      if (bad) { err = "bc_mask values must be 0 or 1"; return M1_ERR_INVALID_ARG; }
      bd.mask[f] = fields->bc_mask[f];
    }
  }
  // state in, checked as by m1_explicit_step
  const size_t bytes = sizeof(double) * (size_t)N;
  const double* comps[5] = {U->E, U->F[0], U->F[1], U->F[2], U->T};
  hipError_t e = hipSuccess;
  for (int k = 0; k < nu && e == hipSuccess; ++k) {
    const double* from = k == 0 ? comps[0] : (k <= nd ? comps[k] : comps[4]);
    e = hipMemcpyAsync(src + (int64_t)k * N, from, bytes, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) { err = std::string("copy in: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  if ((st = noalloc_check(src, n, 0, cnt, s, bad, err)) != M1_OK) return st;
  if (bad) { err = "U has non-finite entries"; return M1_ERR_NONFINITE; }
  if ((st = noalloc_check(src, N, 1, cnt, s, bad, err)) != M1_OK) return st;
  if (bad) { err = "U.E has non-finite or non-positive entries"; return M1_ERR_INVALID_ARG; }
  Scheme sc;
  fill_scheme(*cfg, sc);
  sc.dt = dt;
  sc.s = dt / cfg->dx;
  sc.cdt = cfg->c * dt;
  Coefs<double> cf{};
  cf.sigma = const_cast<double*>(fields->sigma);
  cf.rcv = cpl ? const_cast<double*>(fields->rho_cv) : nullptr;
  for (int32_t k = 0; k < nsteps; ++k) {
    launch_time_step(nd, cpl, semi != 0, g, sc, cf, bd, src, dst, s);
    std::swap(src, dst);
  }
  e = hipGetLastError();
  if (e != hipSuccess) { err = std::string("time step launch: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  unsigned long long nf = 0;
  k_zero_u64<<<1, 64, 0, s>>>(cnt);
  launch_count_f(nd, g, src, cfg->c, cnt, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&nf, cnt, sizeof(nf), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { err = std::string("count: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  if ((st = noalloc_check(src, n, 0, cnt, s, bad, err)) != M1_OK) return st;
  if (bad) { err = "U^(n+nsteps) has non-finite entries"; return M1_ERR_NONFINITE; }
  double* outs[5] = {U->E, U->F[0], U->F[1], U->F[2], U->T};
  for (int k = 0; k < nu && e == hipSuccess; ++k) {
    double* to = k == 0 ? outs[0] : (k <= nd ? outs[k] : outs[4]);
    e = hipMemcpyAsync(to, src + (int64_t)k * N, bytes, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { err = std::string("copy out: ") + hipGetErrorString(e); return M1_ERR_HIP; }
  if (stats) {
    *stats = m1_stats{};
    stats->cells_f_gt_1 = (int64_t)nf;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return M1_OK;
}

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

size_t m1_config_size(void) { return sizeof(m1_config); }
size_t m1_stats_size(void) { return sizeof(m1_stats); }

const char* m1_status_string(int32_t s) {
  switch (s) {
    case M1_OK: return "M1_OK";
    case M1_NOT_CONVERGED: return "M1_NOT_CONVERGED";
    case M1_ERR_INVALID_ARG: return "M1_ERR_INVALID_ARG";
    case M1_ERR_OUT_OF_MEMORY: return "M1_ERR_OUT_OF_MEMORY";
    case M1_ERR_HIP: return "M1_ERR_HIP";
    case M1_ERR_NONFINITE: return "M1_ERR_NONFINITE";
    case M1_NOT_ADMISSIBLE: return "M1_NOT_ADMISSIBLE";
    case M1_ERR_STATE: return "M1_ERR_STATE";
  }
  return "unknown status";
}

const char* m1_kernel_class_name(int32_t kc) { return (kc >= 0 && kc < KC_COUNT) ? kClassNames[kc] : ""; }
int32_t m1_kernel_class_count(void) { return KC_COUNT; }

static thread_local std::string g_setup_err;

m1_status m1_setup(const m1_config* cfg, const m1_fields* fields, const m1_state* U_lin, const m1_state* U_n,
                   double dt, void* hip_stream, m1_ctx** out) {
  if (!out) return M1_ERR_INVALID_ARG;
  *out = nullptr;
  std::string err;
  m1_status st = validate_config(cfg, err);
  if (st != M1_OK) { g_setup_err = err; return st; }
  if (!fields || !fields->sigma) { g_setup_err = "fields or fields->sigma is NULL"; return M1_ERR_INVALID_ARG; }
  if (cfg->source == M1_SRC_COUPLED_T && !fields->rho_cv) { g_setup_err = "rho_cv is NULL"; return M1_ERR_INVALID_ARG; }
  for (int f = 0; f < 2 * cfg->ndim; ++f)
    if (cfg->bc[f] == M1_BC_DIRICHLET && !fields->bc_ghost[f]) { g_setup_err = "Dirichlet face without bc_ghost"; return M1_ERR_INVALID_ARG; }
  if ((U_lin == nullptr) != (U_n == nullptr)) { g_setup_err = "U_lin and U_n must both be given or both NULL"; return M1_ERR_INVALID_ARG; }
  if (U_lin && !(std::isfinite(dt) && dt > 0)) { g_setup_err = "dt must be finite and > 0"; return M1_ERR_INVALID_ARG; }

  m1_ctx* c = new m1_ctx();
  c->cfg = *cfg;
  c->cfg.nn_weights_path = nullptr;
  c->nd = cfg->ndim;
  c->cpl = cfg->source == M1_SRC_COUPLED_T;
  c->nrad = 1 + c->nd;
  c->nu = nu_of(*cfg);
  c->njac = (c->nd * (c->nd + 1) / 2) * (1 + c->nd);
  c->m = cfg->restart;
  c->stream = (hipStream_t)hip_stream;
  hipGetDevice(&c->device);
  fill_geom(*cfg, c->g);
  fill_scheme(*cfg, c->sc);
  const Geom& g = c->g;
  set_dt(c, U_lin ? dt : 1.0);
  c->n = (int64_t)c->nu * g.N;
  c->vs = (c->n + 63) / 64 * 64;
  c->nb = dot_blocks(c->n);

  auto fail = [&](m1_status s) {
    g_setup_err = c->err;
    free_all(c);
    delete c;
    return s;
  };
  const int64_t N = g.N;
  // workspace
  layout<double>(c, nullptr, c->cf64);
  if ((st = dalloc(c, &c->coef64, c->coef_len)) != M1_OK) return fail(st);
  layout<double>(c, c->coef64, c->cf64);
  if (mixed(c)) {
    if ((st = dalloc(c, &c->coef32, c->coef_len)) != M1_OK) return fail(st);
    layout<float>(c, c->coef32, c->cf32);
  }
  if ((st = dalloc(c, &c->Uk, c->n)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->Un, c->n)) != M1_OK) return fail(st);
  if ((cfg->newton_flags & 1) && (st = dalloc(c, &c->Uprev, c->n)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->fn, N)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->b, c->n)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->x, c->n)) != M1_OK) return fail(st);
  const size_t tvs = basis32(c) ? sizeof(float) : sizeof(double);
  const size_t rs = mixed(c) ? sizeof(float) : sizeof(double);
  {
    char* v = nullptr;
    if ((st = dalloc(c, &v, (int64_t)(c->m + 1) * c->vs * (int64_t)tvs)) != M1_OK) return fail(st);
    c->V = v;
    char* a = nullptr;
    if ((st = dalloc(c, &a, c->n * (int64_t)tvs)) != M1_OK) return fail(st);
    c->u[0] = a;
    if ((st = dalloc(c, &a, c->n * (int64_t)tvs)) != M1_OK) return fail(st);
    c->u[1] = a;
    if ((st = dalloc(c, &a, c->n * (int64_t)tvs)) != M1_OK) return fail(st);
    c->p = a;
    if ((st = dalloc(c, &a, c->n * (int64_t)rs)) != M1_OK) return fail(st);
    c->z = a;
  }
  if (cfg->pc == M1_PC_LEARNED) {
    char* a = nullptr;
    if ((st = dalloc(c, &a, (int64_t)(c->m + 1) * c->vs * (int64_t)rs)) != M1_OK) return fail(st);
    c->Z = a;
  }
  if (cfg->pc == M1_PC_MULTIGRID) {
    MgHierarchy& h = c->mg;
    h.omega = cfg->mg_omega;
    h.nu1 = cfg->mg_nu1;
    h.nu2 = cfg->mg_nu2;
    h.nu1c = cfg->mg_nu1_coarse >= 0 ? cfg->mg_nu1_coarse : cfg->mg_nu1;
    h.nu2c = cfg->mg_nu2_coarse >= 0 ? cfg->mg_nu2_coarse : cfg->mg_nu2;
    mg_levels(c, h);
    const int64_t ncoarse = (int64_t)c->nu * h.lev[h.nlev - 1].g.N;
    if (ncoarse > kMgMaxCoarse) {
      c->err = "multigrid: the coarsest level has " + std::to_string(ncoarse) + " unknowns (at most " +
               std::to_string(kMgMaxCoarse) + "); lower mg_nmin";
      return fail(M1_ERR_INVALID_ARG);
    }
    const int64_t nbs = (int64_t)(1 + 2 * c->nd) * c->nu * c->nu;
    for (int l = 0; l < h.nlev; ++l) {
      MgLevel& L = h.lev[l];
      const int64_t Nl = L.g.N;
      const bool coarsest = l + 1 == h.nlev;
      if ((st = dalloc(c, &L.S64, nbs * Nl)) != M1_OK) return fail(st);
      if (l > 0 && mixed(c) && (st = dalloc(c, &L.S32, nbs * Nl)) != M1_OK) return fail(st);
      if (l > 0 && !coarsest) {
        if ((st = dalloc(c, &L.Dinv64, (int64_t)c->nu * c->nu * Nl)) != M1_OK) return fail(st);
        if (mixed(c) && (st = dalloc(c, &L.Dinv32, (int64_t)c->nu * c->nu * Nl)) != M1_OK) return fail(st);
      }
      double* v = nullptr;
      if ((st = dalloc(c, &v, (int64_t)c->nu * Nl)) != M1_OK) return fail(st);
      L.b = v;
      if ((st = dalloc(c, &v, (int64_t)c->nu * Nl)) != M1_OK) return fail(st);
      L.z = v;
      if ((st = dalloc(c, &v, (int64_t)c->nu * Nl)) != M1_OK) return fail(st);
      L.w = v;
      if (l == 0) {
        if ((st = dalloc(c, &v, (int64_t)c->nu * Nl)) != M1_OK) return fail(st);
        L.t = v;
      }
    }
    if ((st = dalloc(c, &h.Ainv64, ncoarse * ncoarse)) != M1_OK) return fail(st);
    if (mixed(c) && (st = dalloc(c, &h.Ainv32, ncoarse * ncoarse)) != M1_OK) return fail(st);
    if ((st = dalloc(c, &h.work, 2 * ncoarse * ncoarse)) != M1_OK) return fail(st);
    if ((st = dalloc(c, &h.bad, 1)) != M1_OK) return fail(st);
    if (!hip_ok(c, hipMemsetAsync(h.bad, 0, sizeof(int), c->stream), "memset")) return fail(M1_ERR_HIP);
    if ((st = dalloc(c, &c->xw, c->n)) != M1_OK) return fail(st);
  }
  if ((st = dalloc(c, &c->part, (int64_t)(2 * kMaxRestart + 2) * c->nb)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->gs, 1)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->dscal, 8)) != M1_OK) return fail(st);
  if ((st = dalloc(c, &c->dcount, 1)) != M1_OK) return fail(st);
  if (!hip_ok(c, hipHostMalloc((void**)&c->hscal, 8 * sizeof(double)), "hipHostMalloc")) return fail(M1_ERR_HIP);
  if (!hip_ok(c, hipMemsetAsync(c->gs, 0, sizeof(GmresState), c->stream), "memset")) return fail(M1_ERR_HIP);
  if (!hip_ok(c, hipMemsetAsync(c->coef64, 0, sizeof(double) * c->coef_len, c->stream), "memset")) return fail(M1_ERR_HIP);

  // field copies and their validation
  if (!hip_ok(c, hipMemcpyAsync(c->cf64.sigma, fields->sigma, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream), "copy sigma"))
    return fail(M1_ERR_HIP);
  if ((st = check_array(c, c->cf64.sigma, N, 2, "sigma", M1_ERR_NONFINITE)) != M1_OK) return fail(st);
  if (c->cpl) {
    if (!hip_ok(c, hipMemcpyAsync(c->cf64.rcv, fields->rho_cv, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream), "copy rho_cv"))
      return fail(M1_ERR_HIP);
    if ((st = check_array(c, c->cf64.rcv, N, 1, "rho_cv", M1_ERR_NONFINITE)) != M1_OK) return fail(st);
  }
  for (int f = 0; f < 2 * c->nd; ++f) {
    if (g.bc[f] != M1_BC_DIRICHLET) continue;
    const int64_t pn = g.plane_n[f / 2];
    if ((st = dalloc(c, &c->plane[f], (int64_t)c->nrad * pn)) != M1_OK) return fail(st);
    if (!hip_ok(c, hipMemcpyAsync(c->plane[f], fields->bc_ghost[f], sizeof(double) * c->nrad * pn, hipMemcpyDeviceToDevice, c->stream), "copy ghost"))
      return fail(M1_ERR_HIP);
    if ((st = check_array(c, c->plane[f], (int64_t)c->nrad * pn, 0, "bc_ghost", M1_ERR_NONFINITE)) != M1_OK) return fail(st);
    if (fields->bc_mask[f]) {
      if ((st = dalloc(c, &c->mask[f], pn)) != M1_OK) return fail(st);
      if (!hip_ok(c, hipMemcpyAsync(c->mask[f], fields->bc_mask[f], sizeof(double) * pn, hipMemcpyDeviceToDevice, c->stream), "copy mask"))
        return fail(M1_ERR_HIP);
      std::vector<double> hm(pn);
      if (!hip_ok(c, hipMemcpyAsync(hm.data(), c->mask[f], sizeof(double) * pn, hipMemcpyDeviceToHost, c->stream), "mask readback") ||
          !hip_ok(c, hipStreamSynchronize(c->stream), "sync"))
        return fail(M1_ERR_HIP);
      for (double v : hm)
        if (!(v == 0.0 || v == 1.0)) { c->err = "bc_mask values must be 0 or 1"; return fail(M1_ERR_INVALID_ARG); }
    }
  }
  if (U_lin) {
    if ((st = copy_state_in(c, U_lin, c->Uk)) != M1_OK) return fail(st);
    if ((st = copy_state_in(c, U_n, c->Un)) != M1_OK) return fail(st);
    if ((st = check_array(c, c->Uk, c->n, 0, "U_lin", M1_ERR_NONFINITE)) != M1_OK) return fail(st);
    if ((st = check_array(c, c->Un, c->n, 0, "U_n", M1_ERR_NONFINITE)) != M1_OK) return fail(st);
    launch_fn(c->nd, g, c->sc, c->Un, c->fn, c->stream);
    if ((st = linearize_internal(c)) != M1_OK) return fail(st);
  }
  if (!hip_ok(c, hipStreamSynchronize(c->stream), "setup sync")) return fail(M1_ERR_HIP);
  *out = c;
  return M1_OK;
}

m1_status m1_linearize(m1_ctx* c, const m1_state* U_lin, const m1_state* U_n, double dt) {
  if (!c) return M1_ERR_INVALID_ARG;
  if (!U_lin || !U_n || !(std::isfinite(dt) && dt > 0)) { c->err = "U_lin, U_n and dt > 0 are required"; return M1_ERR_INVALID_ARG; }
  m1_status st;
  if ((st = copy_state_in(c, U_lin, c->Uk)) != M1_OK) return st;
  if ((st = copy_state_in(c, U_n, c->Un)) != M1_OK) return st;
  if ((st = check_array(c, c->Uk, c->n, 0, "U_lin", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = check_array(c, c->Un, c->n, 0, "U_n", M1_ERR_NONFINITE)) != M1_OK) return st;
  set_dt(c, dt);
  launch_fn(c->nd, c->g, c->sc, c->Un, c->fn, c->stream);
  if ((st = linearize_internal(c)) != M1_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  return M1_OK;
}

m1_status m1_apply_operator(m1_ctx* c, const double* x, double* y) {
  if (!c) return M1_ERR_INVALID_ARG;
  if (!x || !y) { c->err = "x or y is NULL"; return M1_ERR_INVALID_ARG; }
  if (x == y) { c->err = "x and y must not overlap"; return M1_ERR_INVALID_ARG; }
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  timed(c, KC_APPLY, bytes_apply(c, 8, 8, 8, false), [&] {
    launch_apply<double, double, double>(c->nd, c->cpl, 0, c->g, c->sc, c->cf64, bdry(c), x, nullptr, y, c->stream);
  });
  HIPCHK(c, hipGetLastError());
  return M1_OK;
}

m1_status m1_precondition(m1_ctx* c, const double* r, double* z) {
  if (!c) return M1_ERR_INVALID_ARG;
  if (!r || !z) { c->err = "r or z is NULL"; return M1_ERR_INVALID_ARG; }
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  if (c->cfg.pc == M1_PC_NONE) {
    if (r != z) HIPCHK(c, hipMemcpyAsync(z, r, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
    return M1_OK;
  }
  m1_status st;
  if ((st = ensure_bj(c)) != M1_OK) return st;
  if (c->cfg.pc == M1_PC_MULTIGRID) {
    if (r == z) { c->err = "the multigrid preconditioner needs distinct r and z"; return M1_ERR_INVALID_ARG; }
    const MgFine<double> f = mg_fine<double>(c);
    const MgWrap wrap = [&](int kc, double bytes, const std::function<void()>& launch) { timed(c, kc, bytes, launch); };
    mg_vcycle<double, double>(c->mg, f, r, z, c->stream, nullptr, c->prof.on ? &wrap : nullptr);
    prof_close(c);
  } else {
    timed(c, KC_BJ, bytes_bj(c, 8, 8, 8), [&] { launch_bj<double, double, double>(c->nd, c->cpl, c->g, c->cf64, r, z, c->stream); });
  }
  HIPCHK(c, hipGetLastError());
  return M1_OK;
}

m1_status m1_residual(m1_ctx* c, double* R) {
  if (!c) return M1_ERR_INVALID_ARG;
  if (!R) { c->err = "R is NULL"; return M1_ERR_INVALID_ARG; }
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  timed(c, KC_RESIDUAL, bytes_residual(c), [&] { launch_residual(c->nd, c->cpl, c->g, c->sc, c->cf64, bdry(c), c->Uk, c->Un, R, c->stream); });
  // the residual kernel writes -R (the Newton right-hand side); flip the sign
  launch_scale(R, -1.0, c->n, c->stream);
  HIPCHK(c, hipGetLastError());
  return M1_OK;
}

m1_status m1_implicit_step(m1_ctx* c, m1_state* U, double dt, m1_stats* stats) {
  if (!c) return M1_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  if (!(std::isfinite(dt) && dt > 0)) { c->err = "dt must be finite and > 0"; return M1_ERR_INVALID_ARG; }
  m1_status st;
  if ((st = copy_state_in(c, U, c->Un)) != M1_OK) return st;
  if ((st = check_array(c, c->Un, c->n, 0, "U", M1_ERR_NONFINITE)) != M1_OK) return st;
  if ((st = check_array(c, c->Un, c->g.N, 1, "U.E", M1_ERR_INVALID_ARG)) != M1_OK) return st;
  HIPCHK(c, hipMemcpyAsync(c->Uk, c->Un, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
  set_dt(c, dt);
  launch_fn(c->nd, c->g, c->sc, c->Un, c->fn, c->stream);
  const bool fixed = c->cfg.fixed_iters > 0;
  double r0 = -1.0, rel = 1.0;
  int it = 0, kry = 0, rst = 0, fell_back = 0;
  bool converged = false, nonfinite = false;
  double lin_rel = 0.0;
  const double psi0 = c->cfg.ptc_psi0, clip = c->cfg.positivity_clip;
  double psi = psi0;
  // evaluate the scheme at the current iterate: coefficients, b = -R(U^k), ||R||
  auto evaluate = [&](double& rn_out) -> m1_status {
    m1_status s2;
    if ((s2 = linearize_internal(c, false)) != M1_OK) return s2;
    timed(c, KC_RESIDUAL, bytes_residual(c), [&] { launch_residual(c->nd, c->cpl, c->g, c->sc, c->cf64, bdry(c), c->Uk, c->Un, c->b, c->stream); });
    norm2_into(c, c->b, 0);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    rn_out = std::sqrt(std::max(c->hscal[0], 0.0));
    return M1_OK;
  };
  // U^k <- base + lam * delta (delta = c->x, energy step clipped at -clip E)
  auto update = [&](const double* base, double lam) {
    timed(c, KC_NEWTON_UPDATE, 24.0 * c->n, [&] {
      launch_newton_update(c->nd, c->g, c->Uk, base, c->x, lam, clip, c->nu, c->cfg.c, c->dcount, c->stream);
    });
  };
  auto finish = [&]() {
    c->sc.psi = 0.0;
    c->lin_rtol = -1.0;
  };
  const bool line_search = (c->cfg.newton_flags & 1) && !fixed && c->Uprev;
  double rn = 0.0;
  if ((st = evaluate(rn)) != M1_OK) { finish(); return st; }
  while (true) {
    if (r0 < 0) r0 = rn;
    rel = r0 > 0 ? rn / r0 : 0.0;
    if (fixed) {
      if (it >= c->cfg.newton_max) { converged = true; break; }
    } else if (rn == 0.0 || (it > 0 && rel <= c->cfg.newton_rtol)) {
      converged = true;
      break;
    } else if (it >= c->cfg.newton_max) {
      break;
    }
    if (!std::isfinite(rn)) {
      if (verbose()) std::fprintf(stderr, "[m1] newton %d: non-finite residual norm\n", it);
      nonfinite = true;
      break;
    }
    // pseudo-transient continuation: solve (A + psi M) delta = -R
    c->sc.psi = psi;
    // linear tolerance: rtol, loosened by the forcing term and by PTC (the looser applies)
    double eta = c->cfg.rtol;
    if (c->cfg.newton_forcing > 0) eta = std::max(eta, std::min(0.1, c->cfg.newton_forcing * rel));
    if (psi > 0 && c->cfg.ptc_rtol > 0) eta = std::max(eta, std::min(c->cfg.ptc_rtol, psi / psi0));
    c->lin_rtol = eta;
    if ((st = ensure_bj(c)) != M1_OK) { finish(); return st; }
    SolveResult sr;
    if ((st = solve(c, rn, sr, fell_back)) != M1_OK) { finish(); return st; }
    kry += sr.iters;
    rst += sr.restarts;
    lin_rel = sr.rel;
    if (verbose())
      std::fprintf(stderr, "[m1] newton %d |R|=%.3e rel=%.3e psi=%.2e gmres_iters=%d restarts=%d lin_rel=%.2e%s\n", it, rn,
                   rel, psi, sr.iters, sr.restarts, sr.rel, sr.converged ? "" : " (not converged)");
    if (sr.nonfinite) { nonfinite = true; break; }
    double r_new = 0.0;
    bool rejected = false;
    if (!line_search) {
      update(c->Uk, 1.0);
      if ((st = evaluate(r_new)) != M1_OK) { finish(); return st; }
    } else {
      // backtracking: the first lam in 1, 1/2, ..., 1/128 with ||R|| <= (1 - 1e-4 lam) ||R(U^k)||;
      // if none passes the step is rejected (PTC) or the best trial is taken
      HIPCHK(c, hipMemcpyAsync(c->Uprev, c->Uk, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
      const double ref = rn;
      double lam = 1.0, best_r = 0.0, best_lam = 1.0, last_lam = 0.0;
      bool have_best = false, passed = false;
      for (int trial = 0; trial < 8; ++trial) {
        update(c->Uprev, lam);
        double rt = 0.0;
        if ((st = evaluate(rt)) != M1_OK) { finish(); return st; }
        last_lam = lam;
        if (verbose() > 1) std::fprintf(stderr, "[m1]     trial lam=%.4g |R|=%.6e (ref %.6e)\n", lam, rt, ref);
        if (!have_best || (std::isfinite(rt) && !(rt >= best_r))) { best_r = rt; best_lam = lam; have_best = true; }
        if (std::isfinite(rt) && rt <= (1.0 - 1e-4 * lam) * ref) { best_r = rt; best_lam = lam; passed = true; break; }
        lam *= 0.5;
      }
      if (!passed && psi0 > 0) {
        // reject the step: back to U^k (re-evaluated), raise the shift and re-solve
        rejected = true;
        HIPCHK(c, hipMemcpyAsync(c->Uk, c->Uprev, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
        double rk = 0.0;
        if ((st = evaluate(rk)) != M1_OK) { finish(); return st; }
        r_new = rn;
        if (verbose()) std::fprintf(stderr, "[m1]   step rejected (best trial |R| %.3e vs %.3e)\n", best_r, rn);
      } else {
        if (best_lam != last_lam) {
          update(c->Uprev, best_lam);
          if ((st = evaluate(best_r)) != M1_OK) { finish(); return st; }
        }
        r_new = best_r;
        if (verbose() && best_lam < 1.0) std::fprintf(stderr, "[m1]   line search: step %.4g, |R| %.3e -> %.3e\n", best_lam, rn, r_new);
      }
    }
    if (rejected) {
      psi = std::max(10.0 * psi, 1e-3 * psi0);
    } else if (psi > 0) {
      psi = r_new < rn ? psi * r_new / rn : 2.0 * psi;   // switched evolution relaxation
      if (psi < 1e-6 * psi0) psi = 0.0;
    }
    rn = r_new;
    ++it;
  }
  finish();
  unsigned long long nf = 0, ne = 0;
  k_zero_u64<<<1, 64, 0, c->stream>>>(c->dcount);
  launch_count_f(c->nd, c->g, c->Uk, c->cfg.c, c->dcount, c->stream);
  HIPCHK(c, hipMemcpyAsync(&nf, c->dcount, sizeof(nf), hipMemcpyDeviceToHost, c->stream));
  k_zero_u64<<<1, 64, 0, c->stream>>>(c->dcount);
  {
    const int64_t grd = std::max<int64_t>(1, std::min<int64_t>((c->g.N + 255) / 256, 2048));
    k_count_nonpos<<<grd, 256, 0, c->stream>>>(c->Uk, c->g.N, c->dcount);
  }
  HIPCHK(c, hipMemcpyAsync(&ne, c->dcount, sizeof(ne), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  const bool admissible = ne == 0;
  // newton_flags bit 1: a converged root with E <= 0 is still written back
  if (converged && (admissible || (c->cfg.newton_flags & 2))) {
    if ((st = copy_state_out(c, c->Uk, U)) != M1_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (stats) {
    stats->newton_iters = it;
    stats->krylov_iters = kry;
    stats->restarts = rst;
    stats->fell_back = fell_back;
    stats->rel_residual = lin_rel;
    stats->nonlinear_residual = rel;
    stats->cells_f_gt_1 = (int64_t)nf;
    stats->cells_e_nonpos = (int64_t)ne;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (nonfinite) { c->err = "non-finite value in the Newton/GMRES iteration"; return M1_ERR_NONFINITE; }
  if (!converged) { c->err = "Newton iteration did not converge"; return M1_NOT_CONVERGED; }
  if (!admissible) {
    c->err = "the converged state has E <= 0 in " + std::to_string(ne) + " cells (not admissible)";
    return M1_NOT_ADMISSIBLE;
  }
  return M1_OK;
}

m1_status m1_explicit_step(m1_ctx* c, m1_state* U, double dt, int32_t nsteps, m1_stats* stats) {
  return time_steps(c, U, dt, nsteps, stats, false);
}

m1_status m1_semi_implicit_step(m1_ctx* c, m1_state* U, double dt, int32_t nsteps, m1_stats* stats) {
  return time_steps(c, U, dt, nsteps, stats, true);
}

m1_status m1_time_steps_noalloc(const m1_config* cfg, const m1_fields* fields, m1_state* U, double dt,
                                int32_t nsteps, int32_t semi, void* hip_stream, m1_stats* stats) {
  std::string err;
  const m1_status st = time_steps_noalloc(cfg, fields, U, dt, nsteps, semi, hip_stream, stats, err);
  if (st != M1_OK) g_setup_err = err;
  return st;
}

m1_status m1_velocity_sources(m1_ctx* c, m1_state* U, const double* ux, const double* uy, const double* uz,
                              double dt, m1_stats* stats) {
  return velocity_sources(c, U, ux, uy, uz, dt, stats);
}

m1_status m1_set_network(m1_ctx* c, m1nn* net) {
  if (!c) return M1_ERR_INVALID_ARG;
  if (net == nullptr) { c->net = nullptr; return M1_OK; }
  if (c->cfg.pc != M1_PC_LEARNED || c->nd != 2 || c->nu != 3) {
    c->err = "the context must be 2D radiation-only with pc = M1_PC_LEARNED";
    return M1_ERR_INVALID_ARG;
  }
  if (nn_cin(net) != 9 || nn_cout(net) != 3) { c->err = "the network must map 9 input channels to 3"; return M1_ERR_INVALID_ARG; }
  const int q = 1 << (nn_levels(net) - 1);
  if (c->g.n[0] % q || c->g.n[1] % q) { c->err = "nx and ny must be multiples of 2^(levels-1)"; return M1_ERR_INVALID_ARG; }
  if (c->g.n[0] > nn_wmax(net) || c->g.n[1] > nn_hmax(net)) {
    c->err = "the grid is larger than the network's Hmax x Wmax";
    return M1_ERR_INVALID_ARG;
  }
  c->net = net;
  return M1_OK;
}

m1_status m1_nn_features(m1_ctx* c, const double* r, float* features) {
  if (!c || !r || !features) return M1_ERR_INVALID_ARG;
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  if (ensure_bj(c) != M1_OK) return M1_ERR_HIP;
  if (c->nd != 2 || c->nu != 3) { c->err = "features are defined for 2D radiation-only problems"; return M1_ERR_INVALID_ARG; }
  launch_dot<double>(0, nullptr, 0, r, nullptr, c->n, c->part, c->nb, nullptr, c->stream);
  launch_reduce(c->part, 1, c->nb, c->dscal + 3, c->stream);
  launch_nn_features<double>(c->g.N, r, c->dscal + 3, c->cf64.bjinv, c->Uk, c->cf64.sigma, c->cfg.c, c->sc.cdt, 0,
                             nullptr, features, c->stream);
  HIPCHK(c, hipGetLastError());
  return M1_OK;
}

m1_status m1_nn_target(m1_ctx* c, const double* r, const double* e, float* target) {
  if (!c || !r || !e || !target) return M1_ERR_INVALID_ARG;
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  if (ensure_bj(c) != M1_OK) return M1_ERR_HIP;
  if (c->nd != 2 || c->nu != 3) { c->err = "targets are defined for 2D radiation-only problems"; return M1_ERR_INVALID_ARG; }
  launch_dot<double>(0, nullptr, 0, r, nullptr, c->n, c->part, c->nb, nullptr, c->stream);
  launch_reduce(c->part, 1, c->nb, c->dscal + 3, c->stream);
  launch_nn_target(c->g.N, r, e, c->dscal + 3, c->cf64.bjinv, target, c->stream);
  HIPCHK(c, hipGetLastError());
  return M1_OK;
}

m1_status m1_solve_linear(m1_ctx* c, const double* b, double* x, m1_stats* stats) {
  if (!c || !b || !x) return M1_ERR_INVALID_ARG;
  if (!c->linearized) { c->err = "no linearisation yet"; return M1_ERR_STATE; }
  if (ensure_bj(c) != M1_OK) return M1_ERR_HIP;
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(c, hipMemcpyAsync(c->b, b, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
  norm2_into(c, c->b, 0);
  HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double bn = std::sqrt(std::max(c->hscal[0], 0.0));
  SolveResult sr;
  int fell_back = 0;
  m1_status st = solve(c, bn, sr, fell_back);
  if (st != M1_OK) return st;
  HIPCHK(c, hipMemcpyAsync(x, c->x, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->krylov_iters = sr.iters;
    stats->restarts = sr.restarts;
    stats->fell_back = fell_back;
    stats->rel_residual = sr.rel;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (sr.nonfinite) { c->err = "non-finite value in GMRES"; return M1_ERR_NONFINITE; }
  if (!sr.converged) { c->err = "GMRES did not converge"; return M1_NOT_CONVERGED; }
  return M1_OK;
}

void m1_destroy(m1_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

const char* m1_last_error(const m1_ctx* c) { return c ? c->err.c_str() : g_setup_err.c_str(); }

m1_status m1_profile_enable(m1_ctx* c, int32_t on) {
  if (!c) return M1_ERR_INVALID_ARG;
  prof_collect(c);
  c->prof.on = on != 0;
  for (int k = 0; k < KC_COUNT; ++k) {
    c->prof.seen[k] = 0;
    c->prof.launches[k] = 0;
    c->prof.ms[k] = 0.0;
    c->prof.bytes[k] = 0.0;
  }
  return M1_OK;
}

m1_status m1_profile_query(m1_ctx* c, int32_t kc, int64_t* launches, double* total_ms, double* total_bytes) {
  if (!c || kc < 0 || kc >= KC_COUNT || !launches || !total_ms) return M1_ERR_INVALID_ARG;
  prof_collect(c);
  *launches = c->prof.launches[kc];
  *total_ms = c->prof.ms[kc];
  if (total_bytes) *total_bytes = c->prof.bytes[kc];
  return M1_OK;
}

m1_status m1_profile_issued(m1_ctx* c, int32_t kc, int64_t* issued) {
  if (!c || kc < 0 || kc >= KC_COUNT || !issued) return M1_ERR_INVALID_ARG;
  *issued = c->prof.seen[kc];
  return M1_OK;
}

}  // extern "C"
