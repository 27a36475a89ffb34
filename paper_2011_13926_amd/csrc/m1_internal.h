// Host-side internals shared by the kernel translation units and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "m1_device.h"

namespace m1 {

// Pointers into one coefficient slab (FP64 master or FP32 shadow, same layout).
template <typename R> struct Coefs {
  R* jac;        // njac x N        : c^2 dP_pair/d(E,F_l) per cell
  R* face;       // 3*ND x N        : (a, dd, alpha) of the +face of each cell, direction-major
  R* lowface;    // per direction d : 3 x plane_n[d] at lowoff[d] (-face of the first cell, non-periodic)
  R* gjac;       // per face f      : njac x plane_n[f/2] at gjoff[f] (ghost Jacobians, non-periodic)
  R* sigma;      // N
  R* kap;        // N  : 4 a_r T_k^3 (coupled)
  R* rcv;        // N  : rho c_v (coupled)
  R* bjinv;      // nu*nu x N : inverse of the diagonal block, row-major per cell
  int64_t lowoff[3];
  int64_t gjoff[6];
};

// Boundary data and time-level state needed by the residual and the setup.
struct Bdry {
  const double* plane[6];  // Dirichlet ghost (E, F) planes (context copies)
  const double* mask[6];   // optional masks
};

struct GmresState {
  int done;       // cycle finished (estimate below tolerance, breakdown, or final step)
  int k;          // columns used for the solution
  int breakdown;
  int nonfinite;
  double beta;    // residual norm at the cycle start
  double tol;     // absolute tolerance on the least-squares estimate
  double est;     // current least-squares residual estimate |g_k|
  double inv_nu;
  double cc;
  double hprev[kMaxRestart + 1];
  double Hraw[(kMaxRestart + 1) * kMaxRestart];  // unrotated Hessenberg, column-major (ld = kMaxRestart+1)
  double Rm[(kMaxRestart + 1) * kMaxRestart];    // rotated (upper triangular) Hessenberg
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double coef_s[kMaxRestart];
  double coef_t[kMaxRestart];
  double y[kMaxRestart];
};

// ---- aggregation multigrid (m1_multigrid.hip) ----
struct MgGeom {
  int n[3];      // extents (x, y, z; 1 beyond ndim)
  int64_t N;     // cells
  int per[3];    // periodic axes
};

// One level: explicit block stencil S (block 0 diagonal, block 1 + 2d + side the
// neighbour along d, entry (r, c) of block b at S[((b * NU + r) * NU + c) * N + cell]),
// inverse diagonal blocks, and the cycle's vectors (NU * N values of the
// preconditioner's type; 8 bytes each are reserved).  Level 0 is the grid of the
// step: its S64 is the finest stencil, only used to form level 1.
struct MgLevel {
  MgGeom g{};
  double* S64 = nullptr;
  float* S32 = nullptr;
  double* Dinv64 = nullptr;
  float* Dinv32 = nullptr;
  void* b = nullptr;
  void* z = nullptr;
  void* w = nullptr;
  void* t = nullptr;
};

constexpr int kMgMaxLevels = 24;
constexpr int kMgMaxCoarse = 1024;   // unknowns of the coarsest level (dense inverse)

struct MgHierarchy {
  int nlev = 0;
  int nu1 = 1, nu2 = 1;     // sweeps on the finest level
  int nu1c = 1, nu2c = 1;   // sweeps on the coarser levels
  double omega = 0.7;
  MgLevel lev[kMgMaxLevels];
  double* Ainv64 = nullptr;   // coarsest level inverse, row-major
  float* Ainv32 = nullptr;
  double* work = nullptr;     // Gauss-Jordan workspace n x 2n
  int* bad = nullptr;         // a zero pivot was met (device flag)
};

// The finest level as the cycle sees it: the context's block-Jacobi inverses and
// y = A x with the matrix-free operator.
template <typename R> struct MgFine {
  int nd = 2, nu = 3;
  double apply_bytes = 0.0;   // algorithmic bytes of one finest-level apply
  double coef_bytes = 0.0;    // of which the operator's coefficients (no vectors)
  const R* bjinv = nullptr;
  void (*apply)(const void* self, const R* x, R* y, hipStream_t s, const int* skip) = nullptr;
  // fused sweep / restricted residual on the staged operator (launch_mg_sweep2d; r of
  // FP64 or FP32 type as r_fp64 says); null where not available (3D, direct apply)
  bool (*sweep)(const void* self, int op, int xin, int ns, const void* r, int r_fp64, const R* zin, const R* zc,
                R omega, R* out, const R* dinv1, int sm, R* b1, R* z1, hipStream_t s, const int* skip) = nullptr;
  const void* self = nullptr;
  void operator()(const R* x, R* y, hipStream_t s, const int* skip) const { apply(self, x, y, s, skip); }
};

// stencils of levels 1.. (Galerkin), their inverse diagonal blocks, the coarsest inverse (FP64)
void mg_build(MgHierarchy& h, int nd, int nu, hipStream_t s);
// optional timing hook: called with each launch's kernel class and algorithmic bytes
using MgWrap = std::function<void(int kclass, double bytes, const std::function<void()>& launch)>;
// z = one V-cycle applied to r (r of the input type TIN, z of the preconditioner's type R)
template <typename R, typename TIN>
void mg_vcycle(const MgHierarchy& h, const MgFine<R>& fine, const TIN* r, R* z, hipStream_t s, const int* skip,
               const MgWrap* wrap = nullptr);
template <typename R> void mg_axpy(const R* z, double* x, int64_t n, hipStream_t s);
void launch_fine_stencil(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                         double* S, hipStream_t s);

enum KernelClass {
  KC_SETUP = 0, KC_SETUP_BJ, KC_RESIDUAL, KC_APPLY, KC_BJ, KC_DOT, KC_SCALAR, KC_UPDATE, KC_XUPDATE,
  KC_TRUE_RESID, KC_NEWTON_UPDATE, KC_NORM, KC_CONVERT, KC_NN, KC_APPLY_PC, KC_TIME_STEP, KC_VELOCITY, KC_MG_SETUP,
  KC_MG_FINE, KC_MG_SMOOTH, KC_MG_DOWN, KC_MG_COARSE, KC_COUNT
};

// ---- launchers (defined in m1_kernels.hip / m1_krylov.hip) ----
void launch_fn(int nd, const Geom& g, const Scheme& sc, const double* Un, double* fn, hipStream_t s);
void launch_setup(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                  const double* Uk, const double* Un, const double* fn, hipStream_t s);
void launch_setup_bj(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                     hipStream_t s);
// mode: 0 y = A x, 1 y = b - A x
template <typename R, typename VI, typename VO>
void launch_apply(int nd, bool cpl, int mode, const Geom& g, const Scheme& sc, const Coefs<R>& cf, const Bdry& bd,
                  const VI* x, const double* b, VO* y, hipStream_t s, const int* skip = nullptr);
bool fused_apply_available(int nd);
// multigrid finest level in 2D (LDS-staged operator): op 0 out = x + omega M^{-1} (r - A x),
// op 1 b1 = P^T (r - A x) and z1 = omega D1^{-1} b1 (0 unless sm); the input x is zin
// (xin 0), zin + P zc (xin 1; zin may be null) or omega M^{-1} r (xin 2); with ns = 2 a
// sweep x <- x + omega M^{-1} (r - A x) comes first, in the same launch.  False when not
// available.
template <typename R, typename TIN>
bool launch_mg_sweep2d(int nd, bool cpl, int op, int xin, int ns, const Geom& g, const Scheme& sc, const Coefs<R>& cf,
                       const Bdry& bd, const TIN* r, const R* zin, const R* zc, R omega, R* out, const R* dinv1, int sm,
                       R* b1, R* z1, hipStream_t s, const int* skip);
template <typename R, typename VI, typename VO>
bool launch_apply_pre(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<R>& cf, const Bdry& bd,
                      const VI* u, VO* y, hipStream_t s, const int* skip);
void launch_residual(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                     const double* Uk, const double* Un, double* out_negR, hipStream_t s);
// one explicit (semi = false) or semi-implicit time step Un -> Uo (distinct buffers);
// reads only sigma and rho_cv of the coefficient slab
void launch_time_step(int nd, bool cpl, bool semi, const Geom& g, const Scheme& sc, const Coefs<double>& cf,
                      const Bdry& bd, const double* Un, double* Uo, hipStream_t s);
// velocity-dependent sources added explicitly: U -> V (distinct buffers); u[0..nd-1] device fields
void launch_velocity_sources(int nd, bool cpl, const Geom& g, const Scheme& sc, const double* sigma, const double* U,
                             const double* const* u, double dt, double* V, hipStream_t s);
template <typename R, typename VI, typename VO>
void launch_bj(int nd, bool cpl, const Geom& g, const Coefs<R>& cf, const VI* r, VO* z, hipStream_t s,
               const int* skip = nullptr);
void launch_convert(const double* src, float* dst, int64_t n, hipStream_t s);

// Krylov pieces
int dot_blocks(int64_t n);
template <typename TV>
void launch_dot(int j, const TV* V, int64_t vstride, const TV* u, const TV* p, int64_t n, double* partials, int nb,
                const GmresState* gs, hipStream_t s);
void launch_scalar(int j, int final_step, const double* partials, int nb, GmresState* gs, hipStream_t s,
                   int classical = 0);
template <typename TV>
void launch_update(int j, TV* V, int64_t vstride, const TV* u, const TV* p, TV* unext, int64_t n,
                   const GmresState* gs, hipStream_t s);
template <typename R, typename TV>
void launch_xupdate(int nd, bool cpl, const Geom& g, const Coefs<R>& cf, const TV* V, int64_t vstride,
                    const GmresState* gs, double* x, int use_pc, hipStream_t s);
void launch_reduce(const double* partials, int nv, int nb, double* out, hipStream_t s);
void launch_cycle_init(GmresState* gs, const double* beta2, double tol_abs, double tol_rel, hipStream_t s);
// Uk = U0 + lam * dx (U0 may be Uk), counting cells with |F| > c E
void launch_newton_update(int nd, const Geom& g, double* Uk, const double* U0, const double* dx, double lam,
                          double clip, int nu, double c, unsigned long long* fcount, hipStream_t s);
void launch_count_f(int nd, const Geom& g, const double* U, double c, unsigned long long* fcount, hipStream_t s);
void launch_scale(double* v, double a, int64_t n, hipStream_t s);
template <typename TS, typename TD>
void launch_copy_cast(const TS* src, TD* dst, int64_t n, hipStream_t s);

}  // namespace m1
