/*
 * m1.h -- C ABI of the MI355X implicit M1 radiative-transfer step.
 *
 * The library advances the gray, LTE, scattering-free M1 moment system
 * (E, F) -- optionally coupled to the gas internal energy rho c_v T -- by one
 * backward-Euler step of the asymptotic-preserving, well-balanced finite-volume
 * scheme of Bloch et al. (A&A 2021):
 *   - HLL fluxes F* and P* with the M1 closure (Sect. 2.2) and the wave speeds of
 *     Eq. "eigenvalues" (Sect. 3.1.1);
 *   - the asymptotic correction alpha on the energy flux (Eq.
 *     "asymptoticCorrection", Sect. 3.1.3);
 *   - the flux source term {sigma F}, well balanced (Eq. "wb_smart") or centred
 *     (Eq. "wb_naive"), Sect. 3.1.2;
 *   - radiation/matter exchange c sigma (a_r T^4 - E) on the E and T rows
 *     (Eqs. "momentModel", "internalEnergyEqua"), or pure absorption -c sigma E;
 *   - the implicit system of Sect. 3.1.1 solved by Newton iterations (Sect. 3.3.1)
 *     with restarted, right-preconditioned GMRES (right preconditioning as in
 *     Sect. 3.3.2) and a block-Jacobi preconditioner.
 * Hydrodynamics is frozen during the step (Sect. 3.2, step 2 of the splitting).
 *
 * Memory: every array argument is a DEVICE pointer unless marked "host".  Fields
 * are structure-of-arrays, component-major, x fastest:
 *     value(comp, i, j, k) = a[((comp * nz + k) * ny + j) * nx + i]      (nz = 1 in 2D)
 * A "vector" (x, y, r, z below) holds n_u * N doubles in the component order
 * (E, F_x, F_y[, F_z][, T]), N = nx*ny*nz, n_u = 1 + ndim (+1 with the T row).
 * Caller arrays carry no ghost cells; boundaries are described by m1_config.bc.
 *
 * Ownership: the caller owns every buffer it passes; buffers are borrowed for the
 * duration of the call.  The context copies sigma, rho_cv and the boundary planes
 * at m1_setup and owns all workspace (coefficients, Krylov basis, scratch).
 * Everything is enqueued on the HIP stream given to m1_setup; m1_apply_operator,
 * m1_precondition and m1_residual return once the work is enqueued;
 * m1_setup, m1_linearize and m1_implicit_step block until their result is known.  A context is bound to one
 * stream and one device and is not thread safe.
 *
 * Errors: every call returns an m1_status; nothing aborts or throws across the
 * ABI.  Host-side arguments are validated before any launch.  On M1_NOT_CONVERGED
 * and M1_NOT_ADMISSIBLE m1_implicit_step leaves the caller's state unchanged (unless
 * newton_flags bit 1 asks for the non-admissible root) and still fills the stats.
 * m1_last_error() gives a human-readable message for the last failure.
 */
#ifndef M1_H
#define M1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct m1_ctx m1_ctx;

typedef enum {
  M1_OK = 0,
  M1_NOT_CONVERGED = 1,     /* Newton or GMRES hit its iteration cap */
  M1_NOT_ADMISSIBLE = 2,    /* the step converged to a root with E <= 0 in some cell (the scheme is not
                               positivity preserving, Sect. 3.1.3); the state is left unchanged */
  M1_ERR_INVALID_ARG = -1,  /* bad pointer, size, enum or scalar */
  M1_ERR_OUT_OF_MEMORY = -2,
  M1_ERR_HIP = -3,          /* a HIP runtime call failed */
  M1_ERR_NONFINITE = -4,    /* NaN/Inf in an input field or in the iteration */
  M1_ERR_STATE = -5         /* call made before the context holds a linearisation */
} m1_status;

/* Source on the energy row (and the gas-temperature row). */
typedef enum {
  M1_SRC_NONE = 0,        /* radiation only: S_E = 0 */
  M1_SRC_ABSORPTION = 1,  /* S_E = -c sigma E (the absorption form of the ionisation model, Sect. 5.6) */
  M1_SRC_COUPLED_T = 2    /* S_E = c sigma (a_r T^4 - E) with the T row (Eq. "internalEnergyEqua") */
} m1_source;

typedef enum {
  M1_FSRC_WELL_BALANCED = 0, /* Eq. "wb_smart": face-averaged sigma and F */
  M1_FSRC_CENTERED = 1       /* Eq. "wb_naive": sigma_i F_i */
} m1_flux_source;

typedef enum {
  M1_CLOSURE_M1 = 0,  /* chi = (3 + 4f^2) / (5 + 2 sqrt(4 - 3f^2)) (Sect. 2.2) */
  M1_CLOSURE_P1 = 1   /* D = I/3, speeds +-c/sqrt(3) (the f = 0 limit) */
} m1_closure;

/* How the Newton linearisation treats the Eddington tensor; the HLL speeds
 * and alpha are always lagged at the iterate.  The converged root is the same. */
typedef enum {
  M1_LIN_NEWTON = 0,  /* dP/d(E,F) of P = D(E,F) E is differentiated (default) */
  M1_LIN_PICARD = 1   /* the tensor D is frozen at the iterate */
} m1_linearization;

/* Boundary conditions through one layer of ghost cells. */
typedef enum {
  M1_BC_PERIODIC = 0,  /* wrap (must be set on both faces of a direction) */
  M1_BC_OUTFLOW = 1,   /* zero-gradient copy of the boundary cell */
  M1_BC_DIRICHLET = 2, /* ghost (E, F) given by m1_fields.bc_ghost (optionally masked) */
  M1_BC_REFLECT = 3    /* copy with the normal flux component negated */
} m1_bc;

typedef enum { M1_FP64 = 0, M1_MIXED = 1 } m1_precision;
/* Preconditioners: block-Jacobi (the exact n_u x n_u diagonal blocks), none, the
 * learned one (flexible GMRES, block-Jacobi fallback), or aggregation multigrid:
 * one V(mg_nu1, mg_nu2) cycle per application on a hierarchy of 2 x 2 (x 2)
 * aggregates with Galerkin coarse operators A_{l+1} = P^T A_l P (P piecewise
 * constant), damped block-Jacobi smoothing and an exact coarsest solve -- the
 * geometric counterpart of the algebraic multigrid the paper found best
 * (Sect. 4.1-4.2). */
typedef enum { M1_PC_BLOCK_JACOBI = 0, M1_PC_NONE = 1, M1_PC_LEARNED = 2, M1_PC_MULTIGRID = 3 } m1_pc;

typedef struct {
  int32_t ndim;            /* 2 or 3 */
  int32_t newton_flags;    /* bit 0: backtracking line search on ||R||: the first lam in 1, 1/2,
                              ..., 1/128 with ||R(U + lam delta)|| <= (1 - 1e-4 lam) ||R(U)||
                              (Armijo); if none passes, with
                              ptc_psi0 > 0 the step is rejected (U kept, psi = max(10 psi,
                              1e-3 ptc_psi0)), else the trial with the smallest ||R|| is taken
                              (never in fixed-iteration mode);
                              bit 1: a converged root with E <= 0 in some cell is written to U
                              (the call still returns M1_NOT_ADMISSIBLE; for diagnostics and
                              for measuring what the solver does on such roots) */
  int64_t n[3];            /* nx, ny, nz (nz ignored in 2D); each >= 1 */
  double dx;               /* cell size (> 0) */
  double c;                /* speed of light (> 0) */
  double a_r;              /* radiation constant (> 0) */
  int32_t source;          /* m1_source */
  int32_t flux_source;     /* m1_flux_source */
  int32_t closure;         /* m1_closure */
  int32_t ap_correction;   /* 1: alpha of Eq. "asymptoticCorrection"; 0: alpha = 1 (plain HLL) */
  double lambda_floor;     /* >= 0: lambda+ >= floor*c, lambda- <= -floor*c (shadow test, Sect. 5.4) */
  int32_t bc[6];           /* m1_bc for faces -x,+x,-y,+y,-z,+z */
  int32_t linearization;   /* m1_linearization */
  int32_t precision;       /* m1_precision */
  int32_t pc;              /* m1_pc */
  int32_t restart;         /* GMRES restart length m, 1..48 (30 by default) */
  int32_t max_iters;       /* total GMRES iterations per linear solve */
  int32_t newton_max;      /* Newton iterations per step */
  int32_t fixed_iters;     /* > 0: every linear solve runs exactly this many GMRES iterations and
                              every step exactly newton_max Newton iterations (no early exit) */
  int32_t basis_fp32;      /* mixed precision only: 1 stores the Krylov basis in FP32 */
  double rtol;             /* linear: ||b - A x|| <= rtol ||b|| (true residual) */
  double newton_rtol;      /* nonlinear: ||R(U^k)|| <= newton_rtol ||R(U^0)|| */
  double inner_rtol;       /* mixed precision: a GMRES cycle stops once its own estimate drops by this */
  double ptc_psi0;         /* > 0: pseudo-transient continuation (Kelley & Keyes 1998).  Newton
                              iteration k solves (A + psi_k M) delta = -R, M = 1 on the E and F
                              rows and rho c_v on the T row; block-Jacobi uses the shifted blocks.
                              psi_0 = ptc_psi0, psi_{k+1} = psi_k ||R_{k+1}||/||R_k|| when the
                              residual fell, else 2 psi_k; 0 once below 1e-6 ptc_psi0.  The
                              residual, hence the converged root, is unchanged.  0: off */
  double ptc_rtol;         /* > 0: linear tolerance max(rtol, min(ptc_rtol, psi/ptc_psi0)) while
                              psi > 0 (0: rtol throughout) */
  double positivity_clip;  /* in [0, 1): each Newton update lowers a cell's E (and T) by at most
                              this fraction (dE >= -clip E^k, dT >= -clip T^k); 0: off */
  double newton_forcing;   /* > 0: inexact Newton (Eisenstat & Walker 1996 in spirit): iteration k
                              solves to max(rtol, min(0.1, newton_forcing ||R_k||/||R_0||)); the
                              looser of this and the PTC tolerance applies; 0: rtol */
  const char* nn_weights_path; /* host string or NULL (learned preconditioner) */
  /* aggregation multigrid (pc = M1_PC_MULTIGRID; ignored otherwise) */
  double mg_omega;         /* damping of the block-Jacobi smoother, in (0, 2) */
  int32_t mg_nu1;          /* pre-smoothing sweeps, 0..16 */
  int32_t mg_nu2;          /* post-smoothing sweeps, 0..16 */
  int32_t mg_nmin;         /* coarsen while an extent exceeds this (>= 2; 0: 8 in 2D, 4 in 3D); the
                              coarsest level (solved exactly) may hold at most 512 unknowns */
  int32_t wb_boundary;     /* 1: Eq. "boundaryCondition" (Sect. 3.1.2): on every face between a cell and a
                              ghost the well-balanced source takes sigma F = -c (P_dd(inside) -
                              P_dd(ghost)) / dx instead of the face average (well-balanced source
                              only; the implicit step, residual, operator and preconditioners honour
                              it, the explicit and semi-implicit steps refuse it); 0: off */
  int32_t mg_nu1_coarse;   /* multigrid sweeps on the levels below the finest, 0..4; -1: mg_nu1 */
  int32_t mg_nu2_coarse;   /* likewise for mg_nu2 */
} m1_config;

typedef struct {
  double* E;        /* N */
  double* F[3];     /* F[d] for d < ndim, each N */
  double* T;        /* N, required iff source == M1_SRC_COUPLED_T, else ignored */
} m1_state;

typedef struct {
  const double* sigma;       /* N, opacity (>= 0, finite), fixed over the step */
  const double* rho_cv;      /* N, gas heat capacity per volume (> 0); COUPLED_T only */
  /* Dirichlet faces: ghost (E, F_0..F_{ndim-1}) on the face plane, component-major,
   * plane index in grid order with the normal direction removed (x fastest).
   * Optional mask (same plane, values 0 or 1): 1 takes the given ghost, 0 takes
   * the outflow copy of the boundary cell.  NULL mask = all ones. */
  const double* bc_ghost[6];
  const double* bc_mask[6];
} m1_fields;

typedef struct {
  int32_t newton_iters;      /* linear solves made */
  int32_t krylov_iters;      /* GMRES iterations summed over the step */
  int32_t restarts;          /* GMRES restarts summed over the step */
  int32_t fell_back;         /* 1 if the learned preconditioner fell back to block-Jacobi */
  double rel_residual;       /* last linear solve's true relative residual */
  double nonlinear_residual; /* ||R(U_final)|| / ||R(U^n)|| */
  int64_t cells_f_gt_1;      /* cells with |F| > (1 + 1e-12) c E after the step (Sect. 3.1.3 caveat) */
  int64_t cells_e_nonpos;    /* implicit step: cells with E <= 0 in the final iterate (> 0 gives
                                M1_NOT_ADMISSIBLE); 0 for the other calls */
  double seconds;            /* wall time of the call */
} m1_stats;

/* Size of m1_config / m1_stats as compiled (ABI check for bindings). */
size_t m1_config_size(void);
size_t m1_stats_size(void);
const char* m1_status_string(int32_t status);

/*
 * m1_setup -- validate the configuration, allocate the workspace, copy the fields
 * and (when U_lin and U_n are both non-NULL) linearise the scheme at U_lin with
 * the time-level state U_n and time step dt (dt > 0).  U_lin = U_n is the first
 * Newton iterate of a step.  hip_stream is a hipStream_t (NULL = default stream).
 * On success *out holds a new context; on failure *out is NULL.
 */
m1_status m1_setup(const m1_config* cfg, const m1_fields* fields, const m1_state* U_lin,
                   const m1_state* U_n, double dt, void* hip_stream, m1_ctx** out);

/* Re-linearise an existing context at (U_lin, U_n, dt) (Newton iterate update). */
m1_status m1_linearize(m1_ctx* ctx, const m1_state* U_lin, const m1_state* U_n, double dt);

/* y = A x with A the Jacobian of the scheme's residual at the current linearisation
 * (HLL speeds, alpha lagged; tensor per m1_config.linearization; T^4 linearised).
 * x, y: vectors (n_u*N), must not overlap.  M1_ERR_STATE before a linearisation. */
m1_status m1_apply_operator(m1_ctx* ctx, const double* x, double* y);

/* z = M^{-1} r with M the block diagonal of A (one n_u x n_u block per cell, boundary
 * ghost contributions included).  r, z: vectors; may be the same buffer. */
m1_status m1_precondition(m1_ctx* ctx, const double* r, double* z);

/* R = R(U_lin), the residual of the backward-Euler scheme (Sect. 3.1.1) at the
 * linearisation state; R is a vector (n_u*N). */
m1_status m1_residual(m1_ctx* ctx, double* R);

/* One implicit step: U holds U^n on entry and U^{n+1} on M1_OK.  dt > 0.
 * U.E > 0 on entry.  A converged iterate with E <= 0 in any cell is not committed:
 * the call returns M1_NOT_ADMISSIBLE with stats.cells_e_nonpos set (U unchanged),
 * so an M1_OK result is always a valid input of the next step.
 * stats may be NULL.  Blocks until the step's status is known. */
m1_status m1_implicit_step(m1_ctx* ctx, m1_state* U, double dt, m1_stats* stats);

/* nsteps explicit (forward-Euler) steps of the same spatial scheme:
 * U^{n+1} = U^n - R(U^n), the residual of Sect. 3.1.1 evaluated at U^n (closure,
 * HLL speeds and alpha at time n); the T row is divided by rho c_v.  U holds
 * U^n on entry and U^{n+nsteps} on return (device buffers, not retained).
 * dt > 0, nsteps >= 1; U.E > 0 and finite on entry (M1_ERR_INVALID_ARG /
 * M1_ERR_NONFINITE otherwise, U unchanged).  Positivity of E needs the
 * hyperbolic CFL bound c dt <= dx / ndim and, with sources, c dt sigma < 1;
 * neither is checked, and E is not checked between the steps.  A non-finite
 * final state returns M1_ERR_NONFINITE and leaves U unchanged.  stats (may be
 * NULL): iteration counts 0, cells_f_gt_1 of the final state, wall time.
 * Blocks until done.  The context's linearisation (m1_linearize) is kept. */
m1_status m1_explicit_step(m1_ctx* ctx, m1_state* U, double dt, int32_t nsteps, m1_stats* stats);

/* nsteps semi-implicit steps (Sect. 3.1: sources implicit, hyperbolic part
 * explicit): with H = R(U^n) - S(U^n) the flux divergence at time n and S the
 * source part of the residual, U^{n+1} solves U - U^n + H + S(U) = 0 cell by
 * cell: F_m = (F_m^n - H_Fm)/(1 + k), k = c dt sigma; E = (E^n - H_E)/(1 + k)
 * with absorption, E^n - H_E without a source; with the T row, T is the root
 * of rho c_v (T - T^n) + k/(1+k) (a_r T^4 - E*) (E* = E^n - H_E; Newton from
 * T^n, at most 60 iterations, stopping once |dT| <= 1e-15 T) and
 * E = (E* + k a_r T^4)/(1 + k).  Requires the centred flux source (Eq.
 * "wb_naive"): the well-balanced source couples neighbouring cells, and the
 * call returns M1_ERR_INVALID_ARG.  Arguments, errors and stats as for
 * m1_explicit_step; the CFL bound still applies, for any sigma. */
m1_status m1_semi_implicit_step(m1_ctx* ctx, m1_state* U, double dt, int32_t nsteps, m1_stats* stats);

/* Step 3 of the splitting (Sect. 3.2): the velocity-dependent sources of Sect. 2.3,
 * added explicitly and cell-centred after the radiation step,
 *   E += dt S_E(u),  S_E = sigma/c [u.F + E u.u + u.(u.P)]
 *   F += dt c S_F(u), S_F = sigma u.P + sigma a_r T^4 u + sigma/c^2 u (u.F)
 * with P = D(E, F) E (the closure of Sect. 2.2) and sigma the context's opacity.
 * Without a T row (M1_SRC_NONE, M1_SRC_ABSORPTION) there is no emission term; T
 * itself is not changed (the matching gas terms belong to the hydrodynamics).
 * U: the state (device, in/out, not retained); ux, uy, uz: the material velocity,
 * N doubles each, same cell order (uz ignored in 2D, may be NULL there).  dt > 0,
 * U.E > 0 and all inputs finite, else M1_ERR_INVALID_ARG / M1_ERR_NONFINITE and U
 * unchanged; a non-finite result returns M1_ERR_NONFINITE, U unchanged.  stats
 * (may be NULL): cells_f_gt_1 of the result, wall time.  Blocks until done; the
 * context's linearisation is kept. */
m1_status m1_velocity_sources(m1_ctx* ctx, m1_state* U, const double* ux, const double* uy, const double* uz,
                              double dt, m1_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the explicit (semi = 0)
 * or semi-implicit (semi = 1) steps of m1_explicit_step / m1_semi_implicit_step
 * without a context.  The call allocates nothing: its work memory (two state
 * buffers and a counter) is one static device array of the library, 64 MiB +
 * 256 B per GPU, held from the library's first use on that GPU until the
 * process ends.  Limit: n_u * N <= 4 194 304 (e.g. 1024 x 1024 in 2D radiation
 * only, 100^3 in 3D with 4 unknowns); larger grids return M1_ERR_INVALID_ARG.
 * cfg and fields are read as by m1_setup (fields are used in place, not copied,
 * and validated on every call); U, dt, nsteps, stats and the results are those
 * of m1_explicit_step / m1_semi_implicit_step, bit for bit.  hip_stream: a
 * stream of the current device (NULL = default).  Calls that overlap on one GPU
 * share the array and race: serialise them.  Errors: m1_last_error(NULL). */
m1_status m1_time_steps_noalloc(const m1_config* cfg, const m1_fields* fields, m1_state* U, double dt,
                                int32_t nsteps, int32_t semi, void* hip_stream, m1_stats* stats);

void m1_destroy(m1_ctx* ctx);
const char* m1_last_error(const m1_ctx* ctx);

/* Per-kernel-class timing with HIP events on the context's stream (for
 * measurement; off by default; enabling resets the counters).  For each class:
 * timed launches, their summed event time (ms) and summed algorithmic bytes
 * (each array element a launch must read or write, counted once).  Classes
 * launched once per Krylov iteration (apply, block-Jacobi, fused apply, multi-dot,
 * Hessenberg step, update, network) are timed on every 13th launch only, the
 * others on every launch.  total_bytes may be NULL.
 * Class ids 0..m1_kernel_class_count()-1, names from m1_kernel_class_name. */
m1_status m1_profile_enable(m1_ctx* ctx, int32_t on);
m1_status m1_profile_query(m1_ctx* ctx, int32_t kclass, int64_t* launches, double* total_ms, double* total_bytes);
/* Launches of a class issued while profiling was on, timed or not (the sampled classes'
 * total time is about total_ms * issued / launches). */
m1_status m1_profile_issued(m1_ctx* ctx, int32_t kclass, int64_t* issued);
const char* m1_kernel_class_name(int32_t kclass);
int32_t m1_kernel_class_count(void);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (not in the paper).  A small U-Net on 2D fields, NHWC:
 * per level l two 3x3 convolutions (ReLU) with channels[l], 2x2 average pooling
 * between levels, nearest upsampling + skip concatenation on the way up, and a
 * 1x1 head with cout channels.  BF16 MFMA kernels, FP32 accumulation, FP32
 * master weights with Adam.  x, y, target: device FP32 arrays H x W x channels.
 * Used inside flexible GMRES as z = M^{-1} (r + (|r|/s) NN(features(r))),
 * s = sqrt(3N): the network corrects the residual and block-Jacobi maps it to
 * each cell's scale; block-Jacobi is the fallback (m1_stats.fell_back).
 * ------------------------------------------------------------------------- */
typedef struct m1nn m1nn;

m1_status m1nn_create(int32_t cin, int32_t cout, int32_t levels, const int32_t* channels, int32_t Hmax,
                      int32_t Wmax, void* hip_stream, m1nn** out);
int64_t m1nn_param_count(const m1nn* net);
/* host arrays in definition order: each 3x3 weight as [dy][dx][ci][co], its bias,
 * then the head weight [ci][co] and bias */
m1_status m1nn_set_params(m1nn* net, const float* host, int64_t count);
m1_status m1nn_get_params(m1nn* net, float* host, int64_t count);
m1_status m1nn_get_grads(m1nn* net, float* host, int64_t count);
/* Draw initial parameters in the library: He-normal 3x3 weights N(0, 2/(9 C_in)) (He et
 * al. 2015), zero biases, head weights N(0, 1/C_0) * head_scale.  Deterministic in seed
 * (SplitMix64 counter stream, Box-Muller).  Resets nothing else (Adam moments kept). */
m1_status m1nn_init_params(m1nn* net, uint64_t seed, float head_scale);
m1_status m1nn_forward(m1nn* net, const float* x, int32_t H, int32_t W, float* y);
/* forward + relative loss |y - t|^2/|t|^2 + backward (gradients kept for get_grads / adam_step) */
m1_status m1nn_backward(m1nn* net, const float* x, const float* target, int32_t H, int32_t W, double* loss);
m1_status m1nn_adam_step(m1nn* net, float lr);
m1_status m1nn_train_step(m1nn* net, const float* x, const float* target, int32_t H, int32_t W, float lr,
                          double* loss);
m1_status m1nn_save(m1nn* net, const char* path);   /* host path */
m1_status m1nn_load(m1nn* net, const char* path);
void m1nn_destroy(m1nn* net);
const char* m1nn_last_error(const m1nn* net);

/* Attach a network (borrowed; must outlive its use) as the context's learned
 * preconditioner; the context must be 2D radiation-only (n_u = 3) with
 * pc = M1_PC_LEARNED, nx and ny multiples of 2^(levels-1). */
m1_status m1_set_network(m1_ctx* ctx, m1nn* net);
/* Network input features (H x W x 9 FP32) of a residual vector r at the current
 * linearisation: s r/|r| (3), s M^{-1} r/|r| (3), log10(1 + c sigma dt)/4, f_x, f_y. */
m1_status m1_nn_features(m1_ctx* ctx, const double* r, float* features);
/* Training target s (M e - r)/|r| (H x W x 3 FP32) for a residual r with error e, M the
 * diagonal block of A (for e = A^{-1} r this is s (M - A) e/|r|, what the network must add
 * to r so that M^{-1} maps it onto e). */
m1_status m1_nn_target(m1_ctx* ctx, const double* r, const double* e, float* target);
/* Solve A x = b at the current linearisation with the configured GMRES and
 * preconditioner (x0 = 0).  stats may be NULL.  Blocks. */
m1_status m1_solve_linear(m1_ctx* ctx, const double* b, double* x, m1_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* M1_H */
