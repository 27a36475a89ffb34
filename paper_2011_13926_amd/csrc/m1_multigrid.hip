// Aggregation multigrid preconditioner for gfx950.
//
// Not in the paper's own solver set-up verbatim: the method's implicit systems
// were solved with Trilinos preconditioners, algebraic multigrid being the best
// (about ten Krylov iterations against about 250 for damped Jacobi, Sect.
// 4.1-4.2).  Here the hierarchy is geometric: level l+1 has one cell per 2 x 2
// (x 2) aggregate of level-l cells; prolongation is piecewise constant,
// restriction its transpose (the sum over an aggregate), and the coarse
// operators are the Galerkin products A_{l+1} = P^T A_l P, held as explicit
// block stencils (one n_u x n_u diagonal block and one block per face
// neighbour and cell).  Damped block-Jacobi smoothing, a V(nu1, nu2) cycle from
// zero, and an exact solve (a precomputed dense inverse) on the coarsest level.
//
// The finest level stays matrix-free (the operator kernels of m1_kernels.hip
// and the context's block-Jacobi inverses); its explicit stencil is written once
// per linearisation only to form level 1.  Coarse-level kernels are fused per
// level: on the way down one kernel forms the residual of every child cell,
// restricts it and takes the first smoothing sweep of the coarser level; on the
// way up one kernel prolongs and takes the first smoothing sweep.  Stencil
// entries and vectors are component-major (SoA) per level, so consecutive
// threads (cells) read consecutive addresses.
#include <algorithm>
#include <cstdlib>
#include <functional>
#include <vector>

#include "m1_internal.h"

namespace m1 {

constexpr int kMgThreads = 256;

// (i, j, k) of a level-local cell index; a level has at most 2^31 cells, so the
// index arithmetic is 32-bit unsigned (64-bit division is a long instruction
// sequence on the GPU and dominated the small coarse-level kernels)
__device__ __forceinline__ void mg_idx(const MgGeom& g, int64_t cell, int* id) {
  const unsigned c = (unsigned)cell;
  const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
  const unsigned r = c / nx;
  id[0] = (int)(c - r * nx);
  const unsigned k = r / ny;
  id[1] = (int)(r - k * ny);
  id[2] = (int)k;
}

__device__ __forceinline__ int64_t mg_lin(const MgGeom& g, const int* id) {
  return (int64_t)(((unsigned)id[2] * (unsigned)g.n[1] + (unsigned)id[1]) * (unsigned)g.n[0] + (unsigned)id[0]);
}

// neighbour of cell id along d (side 0 lower, 1 upper): -1 if it is outside a
// non-periodic boundary
__device__ __forceinline__ int64_t mg_nb(const MgGeom& g, const int* id, int d, int side) {
  int j[3] = {id[0], id[1], id[2]};
  j[d] += side ? 1 : -1;
  if (j[d] < 0 || j[d] >= g.n[d]) {
    if (!g.per[d]) return -1;
    j[d] = j[d] < 0 ? g.n[d] - 1 : 0;
  }
  return mg_lin(g, j);
}

// the same, also returning the neighbour's (i, j, k)
__device__ __forceinline__ int64_t mg_nb_id(const MgGeom& g, const int* id, int d, int side, int* j) {
  j[0] = id[0];
  j[1] = id[1];
  j[2] = id[2];
  j[d] += side ? 1 : -1;
  if (j[d] < 0 || j[d] >= g.n[d]) {
    if (!g.per[d]) return -1;
    j[d] = j[d] < 0 ? g.n[d] - 1 : 0;
  }
  return mg_lin(g, j);
}

// aggregate (coarse cell) of the fine cell at (i, j, k): no division
__device__ __forceinline__ int64_t mg_parent_id(const MgGeom& gc, const int* id) {
  const int p[3] = {id[0] >> 1, id[1] >> 1, id[2] >> 1};
  return mg_lin(gc, p);
}

// aggregate of a fine cell index
__device__ __forceinline__ int64_t mg_parent(const MgGeom& gf, const MgGeom& gc, int64_t cell) {
  int id[3];
  mg_idx(gf, cell, id);
  return mg_parent_id(gc, id);
}

// ----------------------------------------------------------------------------
// Galerkin coarse operator from the finer level's stencil (FP64).  One thread
// per (coarse cell, output block): the diagonal block collects every child's
// diagonal block and the child-to-child couplings inside the aggregate (and
// couplings that wrap onto the aggregate itself); face block (d, side)
// collects the children's couplings that leave the aggregate on that face.
// ----------------------------------------------------------------------------
template <int ND, int NU>
__global__ __launch_bounds__(kMgThreads) void k_mg_galerkin(MgGeom gf, MgGeom gc, const double* __restrict__ Sf,
                                                            double* __restrict__ Sc) {
  constexpr int NB = 1 + 2 * ND;
  constexpr int BS = NU * NU;
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int blk = blockIdx.y;
  if (I >= gc.N) return;
  int ci[3];
  mg_idx(gc, I, ci);
  double acc[BS];
#pragma unroll
  for (int q = 0; q < BS; ++q) acc[q] = 0.0;
  const int64_t Nf = gf.N;
  for (int cz = 0; cz < (ND == 3 ? 2 : 1); ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int f[3] = {2 * ci[0] + cx, 2 * ci[1] + cy, ND == 3 ? 2 * ci[2] + cz : 0};
        if (f[0] >= gf.n[0] || f[1] >= gf.n[1] || f[2] >= gf.n[2]) continue;
        const int64_t c = mg_lin(gf, f);
        if (blk == 0) {
#pragma unroll
          for (int q = 0; q < BS; ++q) acc[q] += Sf[(int64_t)q * Nf + c];
        }
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int b = 1 + 2 * d + side;
            const int64_t j = mg_nb(gf, f, d, side);
            if (j < 0) continue;
            const bool inside = mg_parent(gf, gc, j) == I;
            if ((blk == 0 && inside) || (blk == b && !inside)) {
#pragma unroll
              for (int q = 0; q < BS; ++q) acc[q] += Sf[((int64_t)b * BS + q) * Nf + c];
            }
          }
      }
#pragma unroll
  for (int q = 0; q < BS; ++q) Sc[((int64_t)blk * BS + q) * gc.N + I] = acc[q];
  (void)NB;
}

// inverse of every cell's diagonal block (FP64)
template <int NU>
__global__ __launch_bounds__(kMgThreads) void k_mg_invert(int64_t N, const double* __restrict__ S,
                                                          double* __restrict__ Dinv, int* __restrict__ bad) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double A[NU][NU], Ai[NU][NU];
#pragma unroll
  for (int r = 0; r < NU; ++r)
#pragma unroll
    for (int k = 0; k < NU; ++k) A[r][k] = S[(int64_t)(r * NU + k) * N + c];
  const bool ok = invert_block<NU>(A, Ai);
  if (!ok) atomicOr(bad, 1);
#pragma unroll
  for (int r = 0; r < NU; ++r)
#pragma unroll
    for (int k = 0; k < NU; ++k) Dinv[(int64_t)(r * NU + k) * N + c] = Ai[r][k];
}

// ----------------------------------------------------------------------------
// Coarsest level: dense matrix of the stencil (component-major unknowns,
// row = comp * N + cell), inverted by Gauss-Jordan elimination with partial
// pivoting in one workgroup.  W: n x 2n workspace, Ainv: n x n row-major.
// ----------------------------------------------------------------------------
constexpr int kGjThreads = 1024;

template <int ND, int NU>
__global__ __launch_bounds__(kGjThreads) void k_mg_dense_inverse(MgGeom g, const double* __restrict__ S,
                                                                 double* __restrict__ W, double* __restrict__ Ainv,
                                                                 int* __restrict__ bad) {
  constexpr int BS = NU * NU;
  const int64_t N = g.N;
  const int n = (int)(NU * N);
  const int n2 = 2 * n;
  const int tid = threadIdx.x;
  for (int r = tid >> 6; r < n; r += kGjThreads / 64)
    for (int c = tid & 63; c < n2; c += 64) W[(int64_t)r * n2 + c] = (c >= n && c - n == r) ? 1.0 : 0.0;
  __syncthreads();
  // scatter the stencil (one thread per cell)
  for (int64_t cell = tid; cell < N; cell += kGjThreads) {
    int id[3];
    mg_idx(g, cell, id);
    for (int rr = 0; rr < NU; ++rr)
      for (int k = 0; k < NU; ++k) {
        const int64_t row = rr * N + cell;
        W[row * n2 + k * N + cell] += S[(int64_t)(rr * NU + k) * N + cell];
        for (int d = 0; d < ND; ++d)
          for (int side = 0; side < 2; ++side) {
            const int64_t j = mg_nb(g, id, d, side);
            if (j < 0) continue;
            const int b = 1 + 2 * d + side;
            W[row * n2 + k * N + j] += S[((int64_t)b * BS + rr * NU + k) * N + cell];
          }
      }
  }
  __syncthreads();
  __shared__ int s_piv;
  __shared__ double s_val[kGjThreads];
  __shared__ int s_idx[kGjThreads];
  const int lane = tid & 63, wave = tid >> 6, nwave = kGjThreads / 64;
  for (int col = 0; col < n; ++col) {
    // pivot: largest |W[r][col]|, r >= col (ties: smallest row)
    double best = -1.0;
    int bi = col;
    for (int r = col + tid; r < n; r += kGjThreads) {
      const double v = fabs(W[(int64_t)r * n2 + col]);
      if (v > best) { best = v; bi = r; }
    }
    s_val[tid] = best;
    s_idx[tid] = bi;
    __syncthreads();
    for (int off = kGjThreads / 2; off > 0; off >>= 1) {
      if (tid < off) {
        const double v2 = s_val[tid + off];
        const int i2 = s_idx[tid + off];
        if (v2 > s_val[tid] || (v2 == s_val[tid] && i2 < s_idx[tid])) {
          s_val[tid] = v2;
          s_idx[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      s_piv = s_idx[0];
      if (!(s_val[0] > 0.0)) atomicOr(bad, 1);
    }
    __syncthreads();
    const int piv = s_piv;
    double* prow = W + (int64_t)col * n2;
    if (piv != col) {
      double* qrow = W + (int64_t)piv * n2;
      for (int c = tid; c < n2; c += kGjThreads) {
        const double t = prow[c];
        prow[c] = qrow[c];
        qrow[c] = t;
      }
    }
    __syncthreads();
    const double inv = 1.0 / prow[col];
    __syncthreads();
    for (int c = tid; c < n2; c += kGjThreads) prow[c] *= inv;
    __syncthreads();
    // eliminate column col from every other row: one wavefront per row, lanes
    // over the columns (the pivot column itself is cleared afterwards)
    for (int r = wave; r < n; r += nwave) {
      if (r == col) continue;
      double* row = W + (int64_t)r * n2;
      const double f = row[col];
      if (f == 0.0) continue;
      for (int c = lane; c < n2; c += 64)
        if (c != col) row[c] -= f * prow[c];
    }
    __syncthreads();
    for (int r = tid; r < n; r += kGjThreads)
      if (r != col) W[(int64_t)r * n2 + col] = 0.0;
    __syncthreads();
  }
  for (int r = wave; r < n; r += nwave)
    for (int c = lane; c < n; c += 64) Ainv[(int64_t)r * n + c] = W[(int64_t)r * n2 + n + c];
}

// value of lane l (uniform) of a double, read into scalar registers
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same inversion for n <= 192 unknowns held in registers: wave w owns the
// rows w, w + 16, ... (12 at most), lane l the columns l, l + 64, l + 128.  Per
// column k: every wave proposes its largest |a_ik| over rows not yet used as
// pivots (lane k % 64 holds column k), the block takes the largest (ties: the
// smallest row), the pivot row's wave passes the row through LDS, and every row
// is updated in place (multipliers from lane k % 64 by cross-lane reads).  Rows are
// never moved: the pivot row of each step is recorded, and the inverse is written
// out with the row and column permutations that the interchanges imply (row k of
// the interchanged matrix is the k-th pivot row; the columns of the in-place result
// are exchanged in reverse order of the row interchanges).  The whole matrix stays
// on chip instead of streaming an n x 2n workspace through L2 once per column.
constexpr int kGjRegRows = 12, kGjRegCols = 3;
constexpr int kGjRegMax = 192;   // 16 waves x 12 rows = 64 lanes x 3 columns

template <int ND, int NU>
__global__ __launch_bounds__(kGjThreads) void k_mg_dense_inverse_reg(MgGeom g, const double* __restrict__ S,
                                                                     double* __restrict__ Ainv, int* __restrict__ bad) {
  static_assert(kGjThreads == 1024, "16 waves");
  constexpr int BS = NU * NU;
  const int N = (int)g.N;
  const int n = NU * N;
  // the wave index as a scalar: it and every address derived from it stay out of the
  // vector registers (which the matrix fills)
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ double s_cv[2][16];
  __shared__ int s_ci[2][16];
  __shared__ double s_prow[2][kGjRegMax];
  __shared__ int s_q[kGjRegMax], s_perm[kGjRegMax], s_invp[kGjRegMax], s_pk[kGjRegMax], s_src[kGjRegMax],
      s_srcinv[kGjRegMax];
  double a[kGjRegRows][kGjRegCols];
  unsigned used = 0;   // bit rI: row wave + 16 rI is a pivot row already (or beyond n)
  // the dense matrix: entry (rr * N + cell, cc * N + cj) sums the stencil blocks b
  // (diagonal, then the face neighbours) whose cell is cj
#pragma unroll
  for (int rI = 0; rI < kGjRegRows; ++rI) {
    const int i = wave + 16 * rI;
    if (i >= n) used |= 1u << rI;
    int rr = 0, cell = 0;
    int nbc[1 + 2 * ND];
    if (i < n) {
      rr = i / N;
      cell = i - rr * N;
      int id[3];
      mg_idx(g, cell, id);
      nbc[0] = cell;
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) nbc[1 + 2 * d + side] = (int)mg_nb(g, id, d, side);
    }
#pragma unroll
    for (int cb = 0; cb < kGjRegCols; ++cb) {
      const int j = lane + 64 * cb;
      double v = 0.0;
      if (i < n && j < n) {
        const int cc = j / N, cj = j - cc * N;
#pragma unroll
        for (int b = 0; b < 1 + 2 * ND; ++b)
          if (nbc[b] == cj) v += S[((int64_t)b * BS + rr * NU + cc) * N + cell];
      }
      a[rI][cb] = v;
    }
  }
  for (int k = 0; k < n; ++k) {
    const int kl = k & 63, kb = k >> 6, buf = k & 1;
    // this wave's candidate for column k
    double best = -1.0;
    int bi = n;
#pragma unroll
    for (int rI = 0; rI < kGjRegRows; ++rI) {
      double v = 0.0;
#pragma unroll
      for (int cb = 0; cb < kGjRegCols; ++cb)
        if (cb == kb) v = a[rI][cb];
      v = fabs(v);
      if (!((used >> rI) & 1u) && v > best) { best = v; bi = wave + 16 * rI; }
    }
    best = readlane_f64(best, kl);
    bi = __builtin_amdgcn_readlane(bi, kl);
    if (lane == 0) { s_cv[buf][wave] = best; s_ci[buf][wave] = bi; }
    __syncthreads();
    double pv = -1.0;
    int q = n;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const double v = s_cv[buf][w];
      const int r = s_ci[buf][w];
      if (v > pv || (v == pv && r < q)) { pv = v; q = r; }
    }
    if (q >= n) q = k;   // no candidate left (cannot happen with n rows and n steps)
    if (tid == 0) {
      s_q[k] = q;
      if (!(pv > 0.0)) atomicOr(bad, 1);
    }
    if (wave == (q & 15)) {
      const int rq = q >> 4;
#pragma unroll
      for (int rI = 0; rI < kGjRegRows; ++rI)
        if (rI == rq) {
#pragma unroll
          for (int cb = 0; cb < kGjRegCols; ++cb)
            if (lane + 64 * cb < kGjRegMax) s_prow[buf][lane + 64 * cb] = a[rI][cb];
        }
    }
    __syncthreads();
    const double inv = 1.0 / s_prow[buf][k];
    double pr[kGjRegCols];
#pragma unroll
    for (int cb = 0; cb < kGjRegCols; ++cb) pr[cb] = s_prow[buf][lane + 64 * cb] * inv;
#pragma unroll
    for (int rI = 0; rI < kGjRegRows; ++rI) {
      double m = 0.0;
#pragma unroll
      for (int cb = 0; cb < kGjRegCols; ++cb)
        if (cb == kb) m = a[rI][cb];
      m = readlane_f64(m, kl);
      const bool pivrow = wave + 16 * rI == q;
      if (pivrow) used |= 1u << rI;
#pragma unroll
      for (int cb = 0; cb < kGjRegCols; ++cb) {
        const bool colk = lane + 64 * cb == k;
        if (pivrow) a[rI][cb] = colk ? inv : pr[cb];
        else a[rI][cb] = colk ? -m * inv : a[rI][cb] - m * pr[cb];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // replay the interchanges: logical row k is the physical row s_q[k]
    for (int k = 0; k < n; ++k) { s_perm[k] = k; s_invp[k] = k; s_src[k] = k; }
    for (int k = 0; k < n; ++k) {
      const int p = s_invp[s_q[k]];
      s_pk[k] = p;
      const int a0 = s_perm[k], b0 = s_perm[p];
      s_perm[k] = b0; s_perm[p] = a0;
      s_invp[b0] = k; s_invp[a0] = p;
    }
    for (int k = n - 1; k >= 0; --k) {
      const int p = s_pk[k];
      const int t = s_src[k];
      s_src[k] = s_src[p];
      s_src[p] = t;
    }
    for (int j = 0; j < n; ++j) s_srcinv[s_src[j]] = j;
  }
  __syncthreads();
#pragma unroll
  for (int rI = 0; rI < kGjRegRows; ++rI) {
    const int i = wave + 16 * rI;
    if (i >= n) continue;
    const int64_t row = (int64_t)s_invp[i] * n;
#pragma unroll
    for (int cb = 0; cb < kGjRegCols; ++cb) {
      const int j = lane + 64 * cb;
      if (j < n) Ainv[row + s_srcinv[j]] = a[rI][cb];
    }
  }
}

// z = Ainv b on the coarsest level (one wavefront per row)
template <typename R>
__global__ __launch_bounds__(256) void k_mg_coarse_solve(int n, const R* __restrict__ Ainv, const R* __restrict__ b,
                                                         R* __restrict__ z, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  double acc = 0.0;
  for (int c = lane; c < n; c += 64) acc += (double)Ainv[(int64_t)row * n + c] * (double)b[c];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) z[row] = (R)acc;
}

// ----------------------------------------------------------------------------
// Finest level (matrix-free operator, the context's block-Jacobi inverses)
// ----------------------------------------------------------------------------
// z0 = omega M^{-1} r (or, with zp, z = zp + omega M^{-1} (r - t)); r of the input type
template <int NU, typename R, typename TIN>
__global__ __launch_bounds__(kMgThreads) void k_mg_fine_smooth(int64_t N, const R* __restrict__ inv, R omega,
                                                               const TIN* __restrict__ r, const R* __restrict__ t,
                                                               const R* __restrict__ zp, R* __restrict__ z,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  R rv[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) rv[k] = (R)r[k * N + c] - (t ? t[k * N + c] : (R)0);
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R acc = (R)0;
#pragma unroll
    for (int k = 0; k < NU; ++k) acc += inv[(rr * NU + k) * N + c] * rv[k];
    z[rr * N + c] = (zp ? zp[rr * N + c] : (R)0) + omega * acc;
  }
}

// level 1 from the finest level: b1 = P^T (r - t) (t = A z0, or none when z0 = 0)
// and the first sweep z1 = omega D1^{-1} b1 (z1 = 0 without pre-smoothing)
template <int ND, int NU, typename R, typename TIN>
__global__ __launch_bounds__(kMgThreads) void k_mg_restrict_fine(MgGeom gf, MgGeom gc, const TIN* __restrict__ r,
                                                                 const R* __restrict__ t, const R* __restrict__ Dinv,
                                                                 R omega, int smooth, R* __restrict__ b1,
                                                                 R* __restrict__ z1, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= gc.N) return;
  int ci[3];
  mg_idx(gc, I, ci);
  R acc[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) acc[k] = (R)0;
  for (int cz = 0; cz < (ND == 3 ? 2 : 1); ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int f[3] = {2 * ci[0] + cx, 2 * ci[1] + cy, ND == 3 ? 2 * ci[2] + cz : 0};
        if (f[0] >= gf.n[0] || f[1] >= gf.n[1] || f[2] >= gf.n[2]) continue;
        const int64_t c = mg_lin(gf, f);
#pragma unroll
        for (int k = 0; k < NU; ++k) acc[k] += (R)r[k * gf.N + c] - (t ? t[k * gf.N + c] : (R)0);
      }
  const int64_t Nc = gc.N;
#pragma unroll
  for (int k = 0; k < NU; ++k) b1[k * Nc + I] = acc[k];
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R z = (R)0;
    if (smooth) {
#pragma unroll
      for (int k = 0; k < NU; ++k) z += Dinv[(rr * NU + k) * Nc + I] * acc[k];
      z *= omega;
    }
    z1[rr * Nc + I] = z;
  }
}

// zp = z0 + P z1 on the finest level
template <int ND, int NU, typename R>
__global__ __launch_bounds__(kMgThreads) void k_mg_prolong_fine(MgGeom gf, MgGeom gc, const R* __restrict__ z0,
                                                                const R* __restrict__ z1, R* __restrict__ zp,
                                                                const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= gf.N) return;
  const int64_t I = mg_parent(gf, gc, c);
#pragma unroll
  for (int k = 0; k < NU; ++k) zp[k * gf.N + c] = z0[k * gf.N + c] + z1[k * gc.N + I];
}

// ----------------------------------------------------------------------------
// Coarse levels (explicit stencils)
// ----------------------------------------------------------------------------
// y = S x at cell c (x given by a functor of (cell, its (i, j, k), comp))
template <int ND, int NU, typename R, typename X>
__device__ __forceinline__ void mg_row(const MgGeom& g, const R* __restrict__ S, int64_t c, const int* id, X&& x,
                                       R (&y)[NU]) {
  constexpr int BS = NU * NU;
  const int64_t N = g.N;
  R xs[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) xs[k] = x(c, id, k);
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R acc = (R)0;
#pragma unroll
    for (int k = 0; k < NU; ++k) acc += S[(int64_t)(rr * NU + k) * N + c] * xs[k];
    y[rr] = acc;
  }
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int jid[3];
      const int64_t j = mg_nb_id(g, id, d, side, jid);
      if (j < 0) continue;
      const int b = 1 + 2 * d + side;
      R xn[NU];
#pragma unroll
      for (int k = 0; k < NU; ++k) xn[k] = x(j, jid, k);
#pragma unroll
      for (int rr = 0; rr < NU; ++rr) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NU; ++k) acc += S[((int64_t)b * BS + rr * NU + k) * N + c] * xn[k];
        y[rr] += acc;
      }
    }
}

// down from level l to l+1: b_{l+1} = P^T (b_l - A_l z_l), z_{l+1} = omega D^{-1} b_{l+1}
// (or 0 without pre-smoothing).
// One thread per child: the 2^ND children of a coarse
// cell sit on consecutive lanes of one wavefront, each forms its own residual,
// two or three butterfly exchanges sum them, and the group's first lane writes the
// coarse values.  (One thread per coarse cell walked the children one after the
// other: a four- or eight-fold longer chain of dependent loads.)
template <int ND, int NU, typename R>
__device__ __forceinline__ void mg_down_group(const MgGeom& gf, const MgGeom& gc, const R* __restrict__ S,
                                              const R* __restrict__ bf, const R* __restrict__ zf,
                                              const R* __restrict__ Dinvc, R omega, int smooth, R* __restrict__ bc,
                                              R* __restrict__ zc, int64_t t) {
  constexpr int G = ND == 3 ? 8 : 4;
  const int64_t I = t / G;
  const int child = (int)(t % G);
  const bool live = I < gc.N;   // every lane of a group has the same I
  R acc[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) acc[k] = (R)0;
  int ci[3] = {0, 0, 0};
  if (live) {
    mg_idx(gc, I, ci);
    int f[3] = {2 * ci[0] + (child & 1), 2 * ci[1] + ((child >> 1) & 1), ND == 3 ? 2 * ci[2] + (child >> 2) : 0};
    if (f[0] < gf.n[0] && f[1] < gf.n[1] && f[2] < gf.n[2]) {
      const int64_t Nf = gf.N;
      const int64_t c = mg_lin(gf, f);
      auto xf = [&](int64_t cell, const int*, int k) { return zf[k * Nf + cell]; };
      R y[NU];
      mg_row<ND, NU, R>(gf, S, c, f, xf, y);
#pragma unroll
      for (int k = 0; k < NU; ++k) acc[k] = bf[k * Nf + c] - y[k];
    }
  }
  // butterfly sum over the group (lanes t ^ 1, t ^ 2 [, t ^ 4]); fixed order
#pragma unroll
  for (int off = 1; off < G; off <<= 1)
#pragma unroll
    for (int k = 0; k < NU; ++k) acc[k] += __shfl_xor(acc[k], off, 64);
  if (!live || child != 0) return;
  const int64_t Nc = gc.N;
#pragma unroll
  for (int k = 0; k < NU; ++k) bc[k * Nc + I] = acc[k];
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R z = (R)0;
    if (smooth) {
#pragma unroll
      for (int k = 0; k < NU; ++k) z += Dinvc[(rr * NU + k) * Nc + I] * acc[k];
      z *= omega;
    }
    zc[rr * Nc + I] = z;
  }
}

// down from level l to l+1: b_{l+1} = P^T (b_l - A_l z_l), z_{l+1} = omega D^{-1} b_{l+1}
// (or 0 without pre-smoothing).
// One thread per child: the 2^ND children of a coarse
// cell sit on consecutive lanes of one wavefront, each forms its own residual,
// two or three butterfly exchanges sum them, and the group's first lane writes the
// coarse values.  (One thread per coarse cell walked the children one after the
// other: a four- or eight-fold longer chain of dependent loads.)
template <int ND, int NU, typename R>
__global__ __launch_bounds__(kMgThreads) void k_mg_down_lanes(MgGeom gf, MgGeom gc, const R* __restrict__ S,
                                                              const R* __restrict__ bf, const R* __restrict__ zf,
                                                              const R* __restrict__ Dinvc, R omega, int smooth,
                                                              R* __restrict__ bc, R* __restrict__ zc,
                                                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  mg_down_group<ND, NU, R>(gf, gc, S, bf, zf, Dinvc, omega, smooth, bc, zc,
                           (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// one damped block-Jacobi sweep on a coarse level, with an optional
// prolongation of the coarser correction first (zc != nullptr):
//   zp = z + P zc,  out = zp + omega D^{-1} (b - A zp)
template <int ND, int NU, typename R>
__device__ __forceinline__ void mg_smooth_cell(const MgGeom& g, const MgGeom& gc, const R* __restrict__ S,
                                               const R* __restrict__ Dinv, R omega, const R* __restrict__ b,
                                               const R* __restrict__ z, const R* __restrict__ zc,
                                               R* __restrict__ out, int64_t c) {
  int id[3];
  mg_idx(g, c, id);
  const int64_t N = g.N;
  auto zp = [&](int64_t cell, const int* cid, int k) {
    R v = z[k * N + cell];
    if (zc) v += zc[k * gc.N + mg_parent_id(gc, cid)];
    return v;
  };
  R y[NU];
  mg_row<ND, NU, R>(g, S, c, id, zp, y);
  R rv[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) rv[k] = b[k * N + c] - y[k];
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R acc = (R)0;
#pragma unroll
    for (int k = 0; k < NU; ++k) acc += Dinv[(rr * NU + k) * N + c] * rv[k];
    out[rr * N + c] = zp(c, id, rr) + omega * acc;
  }
}

template <int ND, int NU, typename R>
__global__ __launch_bounds__(kMgThreads) void k_mg_smooth(MgGeom g, MgGeom gc, const R* __restrict__ S,
                                                          const R* __restrict__ Dinv, R omega, const R* __restrict__ b,
                                                          const R* __restrict__ z, const R* __restrict__ zc,
                                                          R* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  mg_smooth_cell<ND, NU, R>(g, gc, S, Dinv, omega, b, z, zc, out, c);
}

// out = z + P zc (prolongation without smoothing; z may be NULL for zero)
template <int NU, typename R>
__global__ __launch_bounds__(kMgThreads) void k_mg_prolong(MgGeom g, MgGeom gc, const R* __restrict__ z,
                                                           const R* __restrict__ zc, R* __restrict__ out,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int64_t I = mg_parent(g, gc, c);
#pragma unroll
  for (int k = 0; k < NU; ++k) out[k * g.N + c] = (z ? z[k * g.N + c] : (R)0) + zc[k * gc.N + I];
}

// out = (R) in
template <typename R, typename TIN>
__global__ __launch_bounds__(kMgThreads) void k_mg_cast(int64_t n, const TIN* __restrict__ in, R* __restrict__ out,
                                                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = (R)in[e];
}

// x += z (FP64 solution update by a preconditioned correction)
template <typename R>
__global__ __launch_bounds__(kMgThreads) void k_mg_axpy(int64_t n, const R* __restrict__ z, double* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] += (double)z[e];
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------
static inline unsigned grid1(int64_t n) { return (unsigned)((n + kMgThreads - 1) / kMgThreads); }

#define M1_MG_NU_SWITCH(NU_EXPR, CALL) \
  switch (NU_EXPR) {                   \
    case 3: { constexpr int NU = 3; CALL; } break; \
    case 4: { constexpr int NU = 4; CALL; } break; \
    case 5: { constexpr int NU = 5; CALL; } break; \
  }

void mg_build(MgHierarchy& h, int nd, int nu, hipStream_t s) {
  // level l+1 stencils from level l (FP64), diagonal inverses, coarsest inverse
  for (int l = 0; l + 1 < h.nlev; ++l) {
    const MgGeom& gf = h.lev[l].g;
    const MgGeom& gc = h.lev[l + 1].g;
    dim3 grd(grid1(gc.N), 1 + 2 * nd);
    if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_galerkin<2, NU><<<grd, kMgThreads, 0, s>>>(gf, gc, h.lev[l].S64, h.lev[l + 1].S64))) }
    else { M1_MG_NU_SWITCH(nu, (k_mg_galerkin<3, NU><<<grd, kMgThreads, 0, s>>>(gf, gc, h.lev[l].S64, h.lev[l + 1].S64))) }
  }
  for (int l = 1; l + 1 < h.nlev; ++l) {
    M1_MG_NU_SWITCH(nu, (k_mg_invert<NU><<<grid1(h.lev[l].g.N), kMgThreads, 0, s>>>(h.lev[l].g.N, h.lev[l].S64, h.lev[l].Dinv64, h.bad)))
  }
  const MgLevel& L = h.lev[h.nlev - 1];
  if ((int64_t)nu * L.g.N <= kGjRegMax) {
    if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_dense_inverse_reg<2, NU><<<1, kGjThreads, 0, s>>>(L.g, L.S64, h.Ainv64, h.bad))) }
    else { M1_MG_NU_SWITCH(nu, (k_mg_dense_inverse_reg<3, NU><<<1, kGjThreads, 0, s>>>(L.g, L.S64, h.Ainv64, h.bad))) }
  } else {
    if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_dense_inverse<2, NU><<<1, kGjThreads, 0, s>>>(L.g, L.S64, h.work, h.Ainv64, h.bad))) }
    else { M1_MG_NU_SWITCH(nu, (k_mg_dense_inverse<3, NU><<<1, kGjThreads, 0, s>>>(L.g, L.S64, h.work, h.Ainv64, h.bad))) }
  }
}

// operator applications per fused finest-level launch (M1_MG_SWEEPS_PER_LAUNCH=1: one)
static int g_per_launch = -1;
static int sweeps_per_launch() {
  if (g_per_launch < 0) {
    const char* e = getenv("M1_MG_SWEEPS_PER_LAUNCH");
    g_per_launch = (e && e[0] == '1') ? 1 : 2;
  }
  return g_per_launch;
}

template <typename R> static const R* stencil(const MgLevel& L);
template <> const double* stencil<double>(const MgLevel& L) { return L.S64; }
template <> const float* stencil<float>(const MgLevel& L) { return L.S32; }
template <typename R> static const R* dinv(const MgLevel& L);
template <> const double* dinv<double>(const MgLevel& L) { return L.Dinv64; }
template <> const float* dinv<float>(const MgLevel& L) { return L.Dinv32; }
template <typename R> static const R* ainv(const MgHierarchy& h);
template <> const double* ainv<double>(const MgHierarchy& h) { return h.Ainv64; }
template <> const float* ainv<float>(const MgHierarchy& h) { return h.Ainv32; }

template <typename R, typename TIN>
void mg_vcycle(const MgHierarchy& h, const MgFine<R>& fine, const TIN* r, R* z, hipStream_t s, const int* skip,
               const MgWrap* wrap) {
  const int nd = fine.nd;
  const int nu = fine.nu;
  const R om = (R)h.omega;
  const MgGeom& g0 = h.lev[0].g;
  const int64_t N0 = g0.N;
  R* z0 = (R*)h.lev[0].z;
  R* zp = (R*)h.lev[0].w;
  R* t = (R*)h.lev[0].t;
  const double rs = sizeof(R), ti = sizeof(TIN), nb = 1 + 2 * nd, cu = nu, bs = (double)nu * nu;
  const double agg = nd == 3 ? 8.0 : 4.0;
  // every launch goes through the optional timing hook with its class and algorithmic bytes
  auto run = [&](int kc, double bytes, const std::function<void()>& launch) {
    if (wrap && *wrap) (*wrap)(kc, bytes, launch);
    else launch();
  };
  const double fine_apply_bytes = fine.apply_bytes;
  auto fine_smooth_bytes = [&](bool with_t, bool with_zp) {
    return N0 * (cu * ti + bs * rs + cu * rs + (with_t ? cu * rs : 0.0) + (with_zp ? cu * rs : 0.0));
  };
  auto smooth_bytes = [&](const MgLevel& L, bool prolong) {
    return (double)L.g.N * (nb * bs + bs + 3.0 * cu) * rs + (prolong ? (double)L.g.N / agg * cu * rs : 0.0);
  };
  if (h.nlev == 1) {
    // the grid is already at the coarsest size: the cycle is the exact solve
    const int64_t n = (int64_t)nu * N0;
    run(KC_MG_FINE, (double)n * (ti + rs), [&] { k_mg_cast<R, TIN><<<grid1(n), kMgThreads, 0, s>>>(n, r, (R*)h.lev[0].b, skip); });
    run(KC_MG_COARSE, ((double)n * n + 2.0 * n) * rs, [&] { k_mg_coarse_solve<R><<<(unsigned)((n + 3) / 4), 256, 0, s>>>((int)n, ainv<R>(h), (const R*)h.lev[0].b, z, skip); });
    return;
  }
  // ---- finest level, down ----
  // fused form (2D): sweeps and the restricted residual on the LDS-staged operator,
  // the first two sweeps in one launch (its input omega M^{-1} r formed while staging)
  const bool fused = fine.sweep != nullptr;
  const int per_launch = sweeps_per_launch();
  const int r64 = sizeof(TIN) == 8 ? 1 : 0;
  const double Nc1 = (double)h.lev[1].g.N;
  // algorithmic bytes of a fused launch: coefficients, the input (xin), r, M^{-1}, the output
  auto sweep_bytes = [&](int op, int xin, bool with_zin, int sm1) {
    double b = fine.coef_bytes;
    if (xin == 0) b += N0 * cu * rs;
    if (xin == 1) b += (with_zin ? N0 * cu * rs : 0.0) + Nc1 * cu * rs;
    b += N0 * cu * ti;                                  // r (read once, also for xin 2)
    if (xin == 2 || op == 0) b += N0 * bs * rs;         // M^{-1}
    b += op == 0 ? N0 * cu * rs : Nc1 * (2.0 * cu + (sm1 ? bs : 0.0)) * rs;
    return b;
  };
  const MgLevel& Lv1 = h.lev[1];
  const int sm1 = (h.nu1c > 0 && h.nlev > 2) ? 1 : 0;
  if (fused && h.nu1 > 0) {
    // the first sweep is the staged input omega M^{-1} r of the first launch; the nu1 - 1
    // further sweeps and the restricted residual are nu1 operator applications, two per
    // launch; the last launch restricts and writes its input, the pre-smoothed z0
    int apps = h.nu1;
    int xin = 2;
    while (apps > 0) {
      const int ns = apps >= per_launch ? per_launch : 1;
      apps -= ns;
      if (apps > 0) {
        run(KC_MG_FINE, sweep_bytes(0, xin, true, 0), [&] { fine.sweep(fine.self, 0, xin, ns, r, r64, z0, nullptr, om, zp, nullptr, 0, nullptr, nullptr, s, skip); });
        std::swap(z0, zp);
      } else {
        // z0 already holds the input when it came from memory (xin 0 and one application)
        R* keep = (xin == 0 && ns == 1) ? nullptr : zp;
        run(KC_MG_FINE, sweep_bytes(1, xin, true, sm1) + (keep ? N0 * cu * rs : 0.0), [&] { fine.sweep(fine.self, 1, xin, ns, r, r64, z0, nullptr, om, keep, dinv<R>(Lv1), sm1, (R*)Lv1.b, (R*)Lv1.z, s, skip); });
        if (keep) std::swap(z0, zp);
      }
      xin = 0;
    }
  } else {
    if (h.nu1 > 0) {
      run(KC_MG_FINE, fine_smooth_bytes(false, false), [&] { M1_MG_NU_SWITCH(nu, (k_mg_fine_smooth<NU, R, TIN><<<grid1(N0), kMgThreads, 0, s>>>(N0, fine.bjinv, om, r, nullptr, nullptr, z0, skip))) });
      for (int k = 1; k < h.nu1; ++k) {
        run(KC_APPLY, fine_apply_bytes, [&] { fine(z0, t, s, skip); });
        run(KC_MG_FINE, fine_smooth_bytes(true, true), [&] { M1_MG_NU_SWITCH(nu, (k_mg_fine_smooth<NU, R, TIN><<<grid1(N0), kMgThreads, 0, s>>>(N0, fine.bjinv, om, r, t, z0, zp, skip))) });
        std::swap(z0, zp);
      }
      run(KC_APPLY, fine_apply_bytes, [&] { fine(z0, t, s, skip); });
    }
    const R* tt = h.nu1 > 0 ? t : nullptr;
    const double bytes = (double)N0 * cu * (ti + (tt ? rs : 0.0)) + Nc1 * (2.0 * cu + (sm1 ? bs : 0.0)) * rs;
    run(KC_MG_FINE, bytes, [&] {
      if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_restrict_fine<2, NU, R, TIN><<<grid1(Lv1.g.N), kMgThreads, 0, s>>>(g0, Lv1.g, r, tt, dinv<R>(Lv1), om, sm1, (R*)Lv1.b, (R*)Lv1.z, skip))) }
      else { M1_MG_NU_SWITCH(nu, (k_mg_restrict_fine<3, NU, R, TIN><<<grid1(Lv1.g.N), kMgThreads, 0, s>>>(g0, Lv1.g, r, tt, dinv<R>(Lv1), om, sm1, (R*)Lv1.b, (R*)Lv1.z, skip))) }
    });
  }
  // ---- coarse levels, down ----
  // level l holds b_l and z_l (first sweep done, or zero); extra sweeps ping-pong z <-> w
  std::vector<R*> zl(h.nlev), wl(h.nlev);
  for (int l = 1; l < h.nlev; ++l) {
    zl[l] = (R*)h.lev[l].z;
    wl[l] = (R*)h.lev[l].w;
  }
  for (int l = 1; l + 1 < h.nlev; ++l) {
    const MgLevel& L = h.lev[l];
    const MgLevel& C = h.lev[l + 1];
    for (int k = 1; k < h.nu1c; ++k) {
      run(KC_MG_SMOOTH, smooth_bytes(L, false), [&] {
        if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_smooth<2, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], nullptr, wl[l], skip))) }
        else { M1_MG_NU_SWITCH(nu, (k_mg_smooth<3, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], nullptr, wl[l], skip))) }
      });
      std::swap(zl[l], wl[l]);
    }
    const int sm = (h.nu1c > 0 && l + 2 < h.nlev) ? 1 : 0;
    const double bytes = (double)L.g.N * (nb * bs + 2.0 * cu) * rs + (double)C.g.N * (2.0 * cu + (sm ? bs : 0.0)) * rs;
    run(KC_MG_DOWN, bytes, [&] {
      if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_down_lanes<2, NU, R><<<grid1(4 * C.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), (const R*)L.b, zl[l], dinv<R>(C), om, sm, (R*)C.b, zl[l + 1], skip))) }
      else { M1_MG_NU_SWITCH(nu, (k_mg_down_lanes<3, NU, R><<<grid1(8 * C.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), (const R*)L.b, zl[l], dinv<R>(C), om, sm, (R*)C.b, zl[l + 1], skip))) }
    });
  }
  {
    // ---- coarsest: exact ----
    const int last = h.nlev - 1;
    const MgLevel& L = h.lev[last];
    const int n = (int)(nu * L.g.N);
    run(KC_MG_COARSE, ((double)n * n + 2.0 * n) * rs, [&] { k_mg_coarse_solve<R><<<(n + 3) / 4, 256, 0, s>>>(n, ainv<R>(h), (const R*)L.b, zl[last], skip); });
  }
  // ---- coarse levels, up ----
  for (int l = h.nlev - 2; l >= 1; --l) {
    const MgLevel& L = h.lev[l];
    const MgLevel& C = h.lev[l + 1];
    if (h.nu2c > 0) {
      run(KC_MG_SMOOTH, smooth_bytes(L, true), [&] {
        if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_smooth<2, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], zl[l + 1], wl[l], skip))) }
        else { M1_MG_NU_SWITCH(nu, (k_mg_smooth<3, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], zl[l + 1], wl[l], skip))) }
      });
      std::swap(zl[l], wl[l]);
      for (int k = 1; k < h.nu2c; ++k) {
        run(KC_MG_SMOOTH, smooth_bytes(L, false), [&] {
          if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_smooth<2, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], nullptr, wl[l], skip))) }
          else { M1_MG_NU_SWITCH(nu, (k_mg_smooth<3, NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, stencil<R>(L), dinv<R>(L), om, (const R*)L.b, zl[l], nullptr, wl[l], skip))) }
        });
        std::swap(zl[l], wl[l]);
      }
    } else {
      run(KC_MG_SMOOTH, ((double)L.g.N * 2.0 + (double)C.g.N) * cu * rs, [&] { M1_MG_NU_SWITCH(nu, (k_mg_prolong<NU, R><<<grid1(L.g.N), kMgThreads, 0, s>>>(L.g, C.g, zl[l], zl[l + 1], wl[l], skip))) });
      std::swap(zl[l], wl[l]);
    }
  }
  // ---- finest level, up ----
  {
    const MgLevel& L1 = h.lev[1];
    const R* zin = h.nu1 > 0 ? z0 : nullptr;
    if (fused && h.nu2 > 0) {
      // the first launch's input is z0 + P z1, formed while staging; two sweeps per launch
      int left = h.nu2;
      const R* src = zin;
      R* bufs[2] = {zp, z0};
      int nb2 = 0;
      bool first = true;
      while (left > 0) {
        const int ns = left >= per_launch ? per_launch : 1;
        left -= ns;
        R* dst = left == 0 ? z : bufs[nb2++ % 2];
        if (first) run(KC_MG_FINE, sweep_bytes(0, 1, zin != nullptr, 0), [&] { fine.sweep(fine.self, 0, 1, ns, r, r64, src, zl[1], om, dst, nullptr, 0, nullptr, nullptr, s, skip); });
        else run(KC_MG_FINE, sweep_bytes(0, 0, true, 0), [&] { fine.sweep(fine.self, 0, 0, ns, r, r64, src, nullptr, om, dst, nullptr, 0, nullptr, nullptr, s, skip); });
        src = dst;
        first = false;
      }
      return;
    }
    R* out = h.nu2 > 0 ? zp : z;
    const double bytes = ((double)N0 * ((zin ? 1.0 : 0.0) + 1.0) + (double)L1.g.N) * cu * rs;
    if (zin) {
      run(KC_MG_FINE, bytes, [&] {
        if (nd == 2) { M1_MG_NU_SWITCH(nu, (k_mg_prolong_fine<2, NU, R><<<grid1(N0), kMgThreads, 0, s>>>(g0, L1.g, zin, zl[1], out, skip))) }
        else { M1_MG_NU_SWITCH(nu, (k_mg_prolong_fine<3, NU, R><<<grid1(N0), kMgThreads, 0, s>>>(g0, L1.g, zin, zl[1], out, skip))) }
      });
    } else {
      // z0 = 0: the prolonged coarse correction alone
      run(KC_MG_FINE, bytes, [&] { M1_MG_NU_SWITCH(nu, (k_mg_prolong<NU, R><<<grid1(N0), kMgThreads, 0, s>>>(g0, L1.g, nullptr, zl[1], out, skip))) });
    }
    for (int k = 0; k < h.nu2; ++k) {
      R* src = (k % 2 == 0) ? zp : z0;
      R* dst = (k == h.nu2 - 1) ? z : ((k % 2 == 0) ? z0 : zp);
      run(KC_APPLY, fine_apply_bytes, [&] { fine(src, t, s, skip); });
      run(KC_MG_FINE, fine_smooth_bytes(true, true), [&] { M1_MG_NU_SWITCH(nu, (k_mg_fine_smooth<NU, R, TIN><<<grid1(N0), kMgThreads, 0, s>>>(N0, fine.bjinv, om, r, t, src, dst, skip))) });
    }
  }
}

template <typename R>
void mg_axpy(const R* z, double* x, int64_t n, hipStream_t s) {
  k_mg_axpy<R><<<grid1(n), kMgThreads, 0, s>>>(n, z, x);
}

template void mg_vcycle<double, double>(const MgHierarchy&, const MgFine<double>&, const double*, double*, hipStream_t,
                                        const int*, const MgWrap*);
template void mg_vcycle<float, double>(const MgHierarchy&, const MgFine<float>&, const double*, float*, hipStream_t,
                                       const int*, const MgWrap*);
template void mg_vcycle<float, float>(const MgHierarchy&, const MgFine<float>&, const float*, float*, hipStream_t,
                                      const int*, const MgWrap*);
template void mg_axpy<double>(const double*, double*, int64_t, hipStream_t);
template void mg_axpy<float>(const float*, double*, int64_t, hipStream_t);

}  // namespace m1
