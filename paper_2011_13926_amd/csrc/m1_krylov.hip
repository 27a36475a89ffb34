// Krylov kernels for gfx950: restarted GMRES with a one-reduction Arnoldi that
// delays the second Gram-Schmidt pass by one iteration.
//
// Iteration j (Q_j = [q_0..q_{j-1}] orthonormal, u_j the once-projected candidate
// for q_j, p = B u_j with B = A M^{-1}):
//   one fused pass     s = Q_j^T u_j, t = Q_j^T p, alpha = u_j.u_j, gamma = u_j.p
//   one workgroup      nu = sqrt(alpha - |s|^2); column j-1 of H = h'_{j-1} + s, H[j,j-1] = nu;
//                      Givens update; cc = (gamma - s.t)/nu^2;
//                      h'_j = ([t; (gamma - s.t)/nu] - H s) / nu
//   one fused pass     q_j = (u_j - Q_j s)/nu,  u_{j+1} = (p - Q_j (t - cc s) - cc u_j)/nu
// which follows from q_j = (u_j - Q_j s)/nu, B q_j = (p - Q_{j+1} H s)/nu and the
// orthonormality of Q_{j+1}.  The vector passes read the basis twice per iteration
// instead of four times for classical Gram-Schmidt with reorthogonalisation.
// All sums accumulate in FP64 whatever the basis storage type; reductions are
// two-stage (per-block partials, then one workgroup) in a fixed order, so results
// repeat bit for bit run to run.
#include <algorithm>

#include "m1_internal.h"

namespace m1 {

constexpr int kDotThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Enough blocks to fill the chip, few enough that each thread streams several
// quads and the partials (2j+2 values per block) stay small for the one-workgroup
// Hessenberg step.  Measured at n = 786432 (FP32 and FP64 basis): 256 blocks of
// quad loads with the LDS block reduction run at 4.8 / 5.9 TB/s; scalar loads
// with 768..1024 blocks at 1.6 / 3.2 TB/s.
int dot_blocks(int64_t n) {
  const int64_t per = (int64_t)kDotThreads * 4 * 3;
  return (int)std::max<int64_t>(1, std::min<int64_t>(512, (n + per - 1) / per));
}

template <typename TV> struct Quad;
template <> struct Quad<float> { using T = float4; };
template <> struct Quad<double> { using T = double4; };

// partial layout: value v of block b at part[v * nb + b];
// values: s_i (i < J), then t_i (i < J) if HASP, then alpha, then gamma if HASP
template <int J, bool HASP, typename TV>
__global__ __launch_bounds__(kDotThreads) void k_dot(const TV* __restrict__ V, int64_t vs, const TV* __restrict__ u,
                                                     const TV* __restrict__ p, int64_t n, double* __restrict__ part,
                                                     int nb, const GmresState* __restrict__ gs) {
  if (gs && gs->done) return;
  constexpr int NV = HASP ? 2 * J + 2 : J + 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; e < n; e += (int64_t)nb * kDotThreads) {
    const double uv = (double)u[e];
    const double pv = HASP ? (double)p[e] : 0.0;
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const double q = (double)V[i * vs + e];
      acc[i] += q * uv;
      if (HASP) acc[J + i] += q * pv;
    }
    if (HASP) {
      acc[2 * J] += uv * uv;
      acc[2 * J + 1] += uv * pv;
    } else {
      acc[J] += uv * uv;
    }
  }
  __shared__ double red[kDotThreads / 64][NV > 0 ? NV : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double t = wave_sum(acc[v]);
    if (lane == 0) red[w][v] = t;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < NV; v += kDotThreads) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < kDotThreads / 64; ++ww) t += red[ww][v];
    part[(int64_t)v * nb + blockIdx.x] = t;
  }
}

// Same sums with four consecutive elements per load (16-byte float4 or two
// 16-byte halves of a double4): u, p and every basis vector must start on a
// quad boundary (the basis stride is padded to 64 elements).  The n % 4 tail
// elements are added by the first threads of block 0.  Each quad's four
// products are summed first, then added to the accumulator (fixed order).
template <int J, bool HASP, typename TV>
__global__ __launch_bounds__(kDotThreads) void k_dot4(const TV* __restrict__ V, int64_t vs,
                                                      const TV* __restrict__ u, const TV* __restrict__ p, int64_t n,
                                                      double* __restrict__ part, int nb,
                                                      const GmresState* __restrict__ gs) {
  if (gs && gs->done) return;
  using T4 = typename Quad<TV>::T;
  constexpr int NV = HASP ? 2 * J + 2 : J + 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const int64_t n4 = n >> 2;
  const T4* u4 = reinterpret_cast<const T4*>(u);
  const T4* p4 = reinterpret_cast<const T4*>(p);
  for (int64_t e = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; e < n4; e += (int64_t)nb * kDotThreads) {
    const T4 uq = u4[e];
    const double u0 = uq.x, u1 = uq.y, u2 = uq.z, u3 = uq.w;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    if (HASP) {
      const T4 pq = p4[e];
      p0 = pq.x; p1 = pq.y; p2 = pq.z; p3 = pq.w;
    }
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const T4 q = reinterpret_cast<const T4*>(V + i * vs)[e];
      const double q0 = q.x, q1 = q.y, q2 = q.z, q3 = q.w;
      acc[i] += (q0 * u0 + q1 * u1) + (q2 * u2 + q3 * u3);
      if (HASP) acc[J + i] += (q0 * p0 + q1 * p1) + (q2 * p2 + q3 * p3);
    }
    const double uu = (u0 * u0 + u1 * u1) + (u2 * u2 + u3 * u3);
    if (HASP) {
      acc[2 * J] += uu;
      acc[2 * J + 1] += (u0 * p0 + u1 * p1) + (u2 * p2 + u3 * p3);
    } else {
      acc[J] += uu;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < (int)(n - 4 * n4)) {
    const int64_t e = 4 * n4 + threadIdx.x;
    const double uv = (double)u[e];
    const double pv = HASP ? (double)p[e] : 0.0;
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const double q = (double)V[i * vs + e];
      acc[i] += q * uv;
      if (HASP) acc[J + i] += q * pv;
    }
    if (HASP) {
      acc[2 * J] += uv * uv;
      acc[2 * J + 1] += uv * pv;
    } else {
      acc[J] += uv * uv;
    }
  }
  // block reduction: fold each wavefront's lanes to 16 (two exchanges per
  // value), park the 4 x 16 folded sums of every value in LDS, then four threads
  // per value add 16 each and fold; a full six-step exchange per value cost as
  // much as the loads themselves (measured 17.7 -> 11.2 us at n = 786432, FP32)
  __shared__ double lds[NV > 0 ? NV : 1][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double a = acc[v];
    a += __shfl_xor(a, 32, 64);
    a += __shfl_xor(a, 16, 64);
    acc[v] = a;
  }
  if (lane < 16) {
#pragma unroll
    for (int v = 0; v < NV; ++v) lds[v][w * 16 + lane] = acc[v];
  }
  __syncthreads();
  for (int base = 0; base < NV * 4; base += kDotThreads) {
    const int idx = base + threadIdx.x;
    const int v = idx >> 2, q = idx & 3;
    double a = 0.0;
    if (v < NV) {
#pragma unroll
      for (int k = 0; k < 16; ++k) a += lds[v][q * 16 + k];
    }
    a += __shfl_xor(a, 1, 64);
    a += __shfl_xor(a, 2, 64);
    if (v < NV && q == 0) part[(int64_t)v * nb + blockIdx.x] = a;
  }
}

template <typename TV>
static bool quad_aligned(const TV* a) {
  return (reinterpret_cast<uintptr_t>(a) % (4 * sizeof(TV))) == 0;
}

template <int J, bool HASP, typename TV>
static void dot_one(const TV* V, int64_t vs, const TV* u, const TV* p, int64_t n, double* part, int nb,
                    const GmresState* gs, hipStream_t s) {
  const bool quads = quad_aligned(u) && (!HASP || quad_aligned(p)) && (J == 0 || (quad_aligned(V) && vs % 4 == 0));
  if (quads) k_dot4<J, HASP, TV><<<nb, kDotThreads, 0, s>>>(V, vs, u, p, n, part, nb, gs);
  else k_dot<J, HASP, TV><<<nb, kDotThreads, 0, s>>>(V, vs, u, p, n, part, nb, gs);
}

template <typename TV, int... Js>
static void dot_dispatch(std::integer_sequence<int, Js...>, int j, bool hasp, const TV* V, int64_t vs, const TV* u,
                         const TV* p, int64_t n, double* part, int nb, const GmresState* gs, hipStream_t s) {
  using Fn = void (*)(const TV*, int64_t, const TV*, const TV*, int64_t, double*, int, const GmresState*, hipStream_t);
  static const Fn with_p[] = {&dot_one<Js, true, TV>...};
  static const Fn without_p[] = {&dot_one<Js, false, TV>...};
  (hasp ? with_p : without_p)[j](V, vs, u, p, n, part, nb, gs, s);
}

template <typename TV>
void launch_dot(int j, const TV* V, int64_t vs, const TV* u, const TV* p, int64_t n, double* partials, int nb,
                const GmresState* gs, hipStream_t s) {
  dot_dispatch<TV>(std::make_integer_sequence<int, kMaxRestart + 1>{}, j, p != nullptr, V, vs, u, p, n, partials,
                   nb, gs, s);
}

// ----------------------------------------------------------------------------
// a6: one workgroup: reduce the partials, finalise Hessenberg column j-1,
// Givens rotation, residual estimate, coefficients of the next update pass.
// ----------------------------------------------------------------------------
constexpr int kScalarThreads = 1024;
constexpr int kLd = kMaxRestart + 1;

// classical = 1: the standard Arnoldi ordering (flexible GMRES with a nonlinear
// preconditioner): the column is s = V^T w alone (no delayed part), and the update
// coefficients normalise w against V: coef_s = s, coef_t = 0, cc = 0, inv_nu = 1/nu.
__global__ __launch_bounds__(kScalarThreads) void k_scalar(int j, int final_step, int classical,
                                                           const double* __restrict__ part, int nb, GmresState* gs) {
  if (gs->done) return;
  const int hasp = !final_step && !classical;
  const int nv = hasp ? 2 * j + 2 : j + 1;
  const int tid = threadIdx.x;
  __shared__ double psum[kScalarThreads];
  __shared__ double red[2 * kMaxRestart + 2];
  __shared__ double sH[kLd * kMaxRestart];   // unrotated Hessenberg, columns 0..j-1
  __shared__ double sR[kLd * kMaxRestart];   // rotated Hessenberg
  __shared__ double sHp[kLd], sCs[kMaxRestart], sSn[kMaxRestart], sG[kLd], sHs[kLd], sY[kMaxRestart];
  __shared__ double sh_nu;
  __shared__ int sh_done, sh_k;
  // (1) reduce the per-block partials: Q threads per value, fixed order
  const int Q = max(1, kScalarThreads / nv);
  {
    // 8 independent partial sums per thread so the loads overlap (fixed order)
    const int v = tid / Q, q = tid % Q;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (v < nv) {
      const double* pv = part + (int64_t)v * nb;
      int b = q;
      for (; b + 7 * Q < nb; b += 8 * Q) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += pv[b + u * Q];
      }
      for (int u = 0; b < nb; b += Q, ++u) acc[u] += pv[b];
    }
    psum[tid] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  // (2) stage the small GMRES state in LDS (the serial part below makes no
  // global loads: each would stall the one thread for a memory round trip)
  const double tol = gs->tol;
  for (int t = tid; t < j * kLd; t += kScalarThreads) {
    sH[t] = gs->Hraw[t];
    sR[t] = gs->Rm[t];
  }
  for (int t = tid; t <= j; t += kScalarThreads) {
    sHp[t] = gs->hprev[t];
    sG[t] = gs->g[t];
  }
  for (int t = tid; t < j; t += kScalarThreads) {
    sCs[t] = gs->cs[t];
    sSn[t] = gs->sn[t];
  }
  __syncthreads();
  if (tid < nv) {
    double sacc = 0.0;
    for (int q = 0; q < Q; ++q) sacc += psum[tid * Q + q];
    red[tid] = sacc;
  }
  __syncthreads();
  const double* s = red;
  const double* t = red + j;
  const double alpha = hasp ? red[2 * j] : red[j];
  const double gamma = hasp ? red[2 * j + 1] : 0.0;
  // (3a) one wavefront: |s|^2, |h'+s|^2 and the new Hessenberg column h = h' + s
  // (unrotated and, before rotation, rotated copies) in parallel
  __shared__ double sh_ss, sh_hh;
  if (tid < 64) {
    double a = 0.0, b = 0.0;
    for (int i = tid; i < j; i += 64) {
      const double h = sHp[i] + s[i];
      a += s[i] * s[i];
      b += h * h;
      sH[(j - 1) * kLd + i] = h;
      sR[(j - 1) * kLd + i] = h;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (tid == 0) {
      sh_ss = a;
      sh_hh = b;
    }
  }
  __syncthreads();
  // (3b) serial part on LDS
  if (tid == 0) {
    const double ss = sh_ss;
    const double nu2 = alpha - ss;
    int done = 0, k = 0;
    double nu = 0.0;
    if (j == 0) {
      nu = sqrt(fmax(alpha, 0.0));
      gs->beta = nu;
      sG[0] = nu;
      gs->est = nu;
      if (!(nu > 0.0)) {  // zero right-hand side (or NaN)
        done = 1;
        if (nu != nu) gs->nonfinite = 1;
      }
    } else {
      const double col2 = (nu2 > 0.0 ? nu2 : 0.0) + sh_hh;
      nu = (nu2 > 1e-28 * col2) ? sqrt(nu2) : 0.0;
      if (nu == 0.0) gs->breakdown = 1;
      bool nonfinite = false;
      const int c = j - 1;
      double* hc = sH + c * kLd;
      double* rc = sR + c * kLd;
      hc[j] = nu;
      rc[j] = nu;
      // apply the previous rotations; the running element stays in a register
      double carry = rc[0];
      for (int i = 0; i < c; ++i) {
        const double cs_i = sCs[i], sn_i = sSn[i], nxt = rc[i + 1];
        rc[i] = cs_i * carry + sn_i * nxt;
        carry = -sn_i * carry + cs_i * nxt;
      }
      rc[c] = carry;
      const double den = sqrt(rc[c] * rc[c] + rc[j] * rc[j]);
      const double cs = den > 0.0 ? rc[c] / den : 1.0;
      const double sn = den > 0.0 ? rc[j] / den : 0.0;
      sCs[c] = cs;
      sSn[c] = sn;
      rc[c] = den;
      rc[j] = 0.0;
      sG[j] = -sn * sG[c];
      sG[c] = cs * sG[c];
      const double est = fabs(sG[j]);
      gs->est = est;
      if (!(est == est) || !(den == den)) {
        gs->nonfinite = 1;
        nonfinite = true;
      }
      if (est <= tol || nu == 0.0 || final_step || nonfinite) {
        done = 1;
        k = j;
        // back substitution R y = g
        for (int i = j - 1; i >= 0; --i) {
          double acc = sG[i];
          for (int l = i + 1; l < j; ++l) acc -= sR[l * kLd + i] * sY[l];
          sY[i] = acc / sR[i * kLd + i];
        }
      }
    }
    sh_nu = nu;
    sh_done = done;
    sh_k = k;
  }
  __syncthreads();
  // (4) write back: new column, rotation, g, y
  if (j > 0) {
    const int c = j - 1;
    for (int t2 = tid; t2 <= j; t2 += kScalarThreads) {
      gs->Hraw[c * kLd + t2] = sH[c * kLd + t2];
      gs->Rm[c * kLd + t2] = sR[c * kLd + t2];
    }
    if (tid == 0) {
      gs->cs[c] = sCs[c];
      gs->sn[c] = sSn[c];
    }
  }
  for (int t2 = tid; t2 <= j; t2 += kScalarThreads) gs->g[t2] = sG[t2];
  if (sh_done) {
    for (int t2 = tid; t2 < sh_k; t2 += kScalarThreads) gs->y[t2] = sY[t2];
    __syncthreads();
    if (tid == 0) {
      gs->k = sh_k;
      gs->done = 1;
    }
    return;
  }
  const double nu = sh_nu;
  if (classical) {
    for (int i = tid; i <= j; i += kScalarThreads) {
      if (i < j) {
        gs->coef_s[i] = s[i];
        gs->coef_t[i] = 0.0;
      }
      gs->hprev[i] = 0.0;
    }
    if (tid == 0) {
      gs->cc = 0.0;
      gs->inv_nu = 1.0 / nu;
    }
    return;
  }
  // (5) (H s)[r], r = 0..j, with the unrotated Hessenberg (columns 0..j-1)
  for (int r = tid; r <= j; r += kScalarThreads) {
    double acc = 0.0;
    for (int i = 0; i < j; ++i) acc += sH[i * kLd + r] * s[i];
    sHs[r] = acc;
  }
  __syncthreads();
  double st = 0.0;
  for (int i = 0; i < j; ++i) st += s[i] * t[i];
  const double qp = (gamma - st) / nu;  // q_j . p
  const double cc = qp / nu;
  for (int i = tid; i < j; i += kScalarThreads) {
    gs->coef_s[i] = s[i];
    gs->coef_t[i] = t[i] - cc * s[i];
    gs->hprev[i] = (t[i] - sHs[i]) / nu;
  }
  if (tid == 0) {
    gs->hprev[j] = (qp - sHs[j]) / nu;
    gs->cc = cc;
    gs->inv_nu = 1.0 / nu;
  }
}

void launch_scalar(int j, int final_step, const double* partials, int nb, GmresState* gs, hipStream_t s,
                   int classical) {
  k_scalar<<<1, kScalarThreads, 0, s>>>(j, final_step, classical, partials, nb, gs);
}

// ----------------------------------------------------------------------------
// update pass: q_j and u_{j+1}
// ----------------------------------------------------------------------------
template <int J, typename TV>
__global__ __launch_bounds__(kDotThreads) void k_update(TV* __restrict__ V, int64_t vs, const TV* __restrict__ u,
                                                        const TV* __restrict__ p, TV* __restrict__ unext, int64_t n,
                                                        const GmresState* __restrict__ gs) {
  if (gs->done) return;
  double cs_[J > 0 ? J : 1], ct_[J > 0 ? J : 1];
#pragma unroll
  for (int i = 0; i < J; ++i) {
    cs_[i] = gs->coef_s[i];
    ct_[i] = gs->coef_t[i];
  }
  const double cc = gs->cc, inv = gs->inv_nu;
  TV* __restrict__ qj = V + (int64_t)J * vs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double uv = (double)u[e];
    double a1 = uv;
    double a2 = (double)p[e] - cc * uv;
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const double q = (double)V[i * vs + e];
      a1 -= cs_[i] * q;
      a2 -= ct_[i] * q;
    }
    qj[e] = (TV)(a1 * inv);
    unext[e] = (TV)(a2 * inv);
  }
}

// Same update on quads (one 16-byte FP32 or two 16-byte FP64 accesses per
// vector per thread); operands quad-aligned, the n % 4 tail done by block 0.
template <int J, typename TV>
__global__ __launch_bounds__(kDotThreads) void k_update4(TV* __restrict__ V, int64_t vs, const TV* __restrict__ u,
                                                         const TV* __restrict__ p, TV* __restrict__ unext, int64_t n,
                                                         const GmresState* __restrict__ gs) {
  if (gs->done) return;
  using T4 = typename Quad<TV>::T;
  double cs_[J > 0 ? J : 1], ct_[J > 0 ? J : 1];
#pragma unroll
  for (int i = 0; i < J; ++i) {
    cs_[i] = gs->coef_s[i];
    ct_[i] = gs->coef_t[i];
  }
  const double cc = gs->cc, inv = gs->inv_nu;
  TV* __restrict__ qj = V + (int64_t)J * vs;
  const int64_t n4 = n >> 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += (int64_t)gridDim.x * blockDim.x) {
    const T4 uq = reinterpret_cast<const T4*>(u)[e];
    const T4 pq = reinterpret_cast<const T4*>(p)[e];
    double a1[4] = {(double)uq.x, (double)uq.y, (double)uq.z, (double)uq.w};
    double a2[4] = {(double)pq.x - cc * a1[0], (double)pq.y - cc * a1[1], (double)pq.z - cc * a1[2],
                    (double)pq.w - cc * a1[3]};
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const T4 q = reinterpret_cast<const T4*>(V + i * vs)[e];
      const double qv[4] = {(double)q.x, (double)q.y, (double)q.z, (double)q.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a1[k] -= cs_[i] * qv[k];
        a2[k] -= ct_[i] * qv[k];
      }
    }
    T4 o1, o2;
    o1.x = (TV)(a1[0] * inv); o1.y = (TV)(a1[1] * inv); o1.z = (TV)(a1[2] * inv); o1.w = (TV)(a1[3] * inv);
    o2.x = (TV)(a2[0] * inv); o2.y = (TV)(a2[1] * inv); o2.z = (TV)(a2[2] * inv); o2.w = (TV)(a2[3] * inv);
    reinterpret_cast<T4*>(qj)[e] = o1;
    reinterpret_cast<T4*>(unext)[e] = o2;
  }
  if (blockIdx.x == 0 && threadIdx.x < (int)(n - 4 * n4)) {
    const int64_t e = 4 * n4 + threadIdx.x;
    const double uv = (double)u[e];
    double a1 = uv;
    double a2 = (double)p[e] - cc * uv;
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const double q = (double)V[i * vs + e];
      a1 -= cs_[i] * q;
      a2 -= ct_[i] * q;
    }
    qj[e] = (TV)(a1 * inv);
    unext[e] = (TV)(a2 * inv);
  }
}

template <int J, typename TV>
static void upd_one(TV* V, int64_t vs, const TV* u, const TV* p, TV* un, int64_t n, const GmresState* gs,
                    hipStream_t s) {
  const bool quads = quad_aligned(u) && quad_aligned(p) && quad_aligned(un) && quad_aligned(V) && vs % 4 == 0;
  if (quads) {
    const int64_t n4 = n >> 2;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n4 + kDotThreads - 1) / kDotThreads));
    k_update4<J, TV><<<nb, kDotThreads, 0, s>>>(V, vs, u, p, un, n, gs);
  } else {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + kDotThreads - 1) / kDotThreads));
    k_update<J, TV><<<nb, kDotThreads, 0, s>>>(V, vs, u, p, un, n, gs);
  }
}

template <typename TV, int... Js>
static void upd_dispatch(std::integer_sequence<int, Js...>, int j, TV* V, int64_t vs, const TV* u, const TV* p,
                         TV* un, int64_t n, const GmresState* gs, hipStream_t s) {
  using Fn = void (*)(TV*, int64_t, const TV*, const TV*, TV*, int64_t, const GmresState*, hipStream_t);
  static const Fn tab[] = {&upd_one<Js, TV>...};
  tab[j](V, vs, u, p, un, n, gs, s);
}

template <typename TV>
void launch_update(int j, TV* V, int64_t vs, const TV* u, const TV* p, TV* unext, int64_t n, const GmresState* gs,
                   hipStream_t s) {
  upd_dispatch<TV>(std::make_integer_sequence<int, kMaxRestart>{}, j, V, vs, u, p, unext, n, gs, s);
}

// ----------------------------------------------------------------------------
// a7: x += M^{-1} (Q_k y)
// ----------------------------------------------------------------------------
template <int NU, typename R, typename TV>
__global__ __launch_bounds__(256) void k_xupdate(int64_t N, const R* __restrict__ inv, const TV* __restrict__ V,
                                                 int64_t vs, const GmresState* __restrict__ gs, double* __restrict__ x,
                                                 int use_pc) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  const int k = gs->k;
  double v[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) v[c] = 0.0;
  for (int i = 0; i < k; ++i) {
    const double yi = gs->y[i];
#pragma unroll
    for (int c = 0; c < NU; ++c) v[c] += yi * (double)V[i * vs + c * N + cell];
  }
#pragma unroll
  for (int r = 0; r < NU; ++r) {
    double z = v[r];
    if (use_pc) {
      z = 0.0;
#pragma unroll
      for (int c = 0; c < NU; ++c) z += (double)inv[(r * NU + c) * N + cell] * v[c];
    }
    x[r * N + cell] += z;
  }
}

template <typename R, typename TV>
void launch_xupdate(int nd, bool cpl, const Geom& g, const Coefs<R>& cf, const TV* V, int64_t vs,
                    const GmresState* gs, double* x, int use_pc, hipStream_t s) {
  const int nu = 1 + nd + (cpl ? 1 : 0);
  const int64_t grd = (g.N + 255) / 256;
  switch (nu) {
    case 3: k_xupdate<3, R, TV><<<grd, 256, 0, s>>>(g.N, cf.bjinv, V, vs, gs, x, use_pc); break;
    case 4: k_xupdate<4, R, TV><<<grd, 256, 0, s>>>(g.N, cf.bjinv, V, vs, gs, x, use_pc); break;
    case 5: k_xupdate<5, R, TV><<<grd, 256, 0, s>>>(g.N, cf.bjinv, V, vs, gs, x, use_pc); break;
  }
}

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------
__global__ void k_reduce(const double* __restrict__ part, int nv, int nb, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int v = w; v < nv; v += blockDim.x / 64) {
    double t = 0.0;
    for (int b = lane; b < nb; b += 64) t += part[(int64_t)v * nb + b];
    t = wave_sum(t);
    if (lane == 0) out[v] = t;
  }
}

void launch_reduce(const double* partials, int nv, int nb, double* out, hipStream_t s) {
  k_reduce<<<1, 256, 0, s>>>(partials, nv, nb, out);
}

__global__ void k_cycle_init(GmresState* gs, const double* beta2, double tol_abs, double tol_rel) {
  if (threadIdx.x == 0) {
    gs->done = 0;
    gs->k = 0;
    gs->breakdown = 0;
    gs->nonfinite = 0;
    const double beta = sqrt(fmax(beta2[0], 0.0));
    gs->tol = fmax(tol_abs, tol_rel * beta);
  }
}

void launch_cycle_init(GmresState* gs, const double* beta2, double tol_abs, double tol_rel, hipStream_t s) {
  k_cycle_init<<<1, 64, 0, s>>>(gs, beta2, tol_abs, tol_rel);
}

template <int ND>
__device__ __forceinline__ bool f_gt_1(const double* U, int64_t N, int64_t cell, double c) {
  double F2 = 0.0;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    const double f = U[(1 + m) * N + cell];
    F2 += f * f;
  }
  return sqrt(F2) > kFgt1 * c * U[cell];
}

template <int ND>
__global__ __launch_bounds__(256) void k_newton_update(int64_t N, int nu, double* __restrict__ U,
                                                       const double* __restrict__ U0, const double* __restrict__ dx,
                                                       double lam, double clip, double c,
                                                       unsigned long long* fcount) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool gt = false;
  if (cell < N) {
    // positivity clip: the energy (and temperature) step is at least -clip of the
    // current value (clip = 0: off)
    const int tq = (nu == ND + 2) ? nu - 1 : -1;   // T row index with the coupled source
    for (int q = 0; q < nu; ++q) {
      const double u0 = U0[q * N + cell];
      double d = dx[q * N + cell];
      if (clip > 0.0 && (q == 0 || q == tq)) d = fmax(d, -clip * u0);
      U[q * N + cell] = u0 + lam * d;
    }
    gt = f_gt_1<ND>(U, N, cell, c);
  }
  const unsigned long long ballot = __ballot(gt);
  if ((threadIdx.x & 63) == 0 && ballot) atomicAdd(fcount, (unsigned long long)__popcll(ballot));
}

void launch_newton_update(int nd, const Geom& g, double* Uk, const double* U0, const double* dx, double lam,
                          double clip, int nu, double c, unsigned long long* fcount, hipStream_t s) {
  const int64_t grd = (g.N + 255) / 256;
  if (nd == 2) k_newton_update<2><<<grd, 256, 0, s>>>(g.N, nu, Uk, U0, dx, lam, clip, c, fcount);
  else k_newton_update<3><<<grd, 256, 0, s>>>(g.N, nu, Uk, U0, dx, lam, clip, c, fcount);
}

template <int ND>
__global__ __launch_bounds__(256) void k_count_f(int64_t N, const double* __restrict__ U, double c,
                                                 unsigned long long* fcount) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool gt = cell < N && f_gt_1<ND>(U, N, cell, c);
  const unsigned long long ballot = __ballot(gt);
  if ((threadIdx.x & 63) == 0 && ballot) atomicAdd(fcount, (unsigned long long)__popcll(ballot));
}

void launch_count_f(int nd, const Geom& g, const double* U, double c, unsigned long long* fcount, hipStream_t s) {
  const int64_t grd = (g.N + 255) / 256;
  if (nd == 2) k_count_f<2><<<grd, 256, 0, s>>>(g.N, U, c, fcount);
  else k_count_f<3><<<grd, 256, 0, s>>>(g.N, U, c, fcount);
}

template <typename TS, typename TD>
__global__ void k_copy_cast(const TS* __restrict__ src, TD* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (TD)src[i];
}

template <typename TS, typename TD>
void launch_copy_cast(const TS* src, TD* dst, int64_t n, hipStream_t s) {
  const int64_t grd = std::min<int64_t>((n + 255) / 256, 4096);
  k_copy_cast<TS, TD><<<grd, 256, 0, s>>>(src, dst, n);
}

__global__ void k_scale(double* __restrict__ v, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] *= a;
}

void launch_scale(double* v, double a, int64_t n, hipStream_t s) {
  const int64_t grd = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  k_scale<<<grd, 256, 0, s>>>(v, a, n);
}

// explicit instantiations
template void launch_dot<double>(int, const double*, int64_t, const double*, const double*, int64_t, double*, int,
                                 const GmresState*, hipStream_t);
template void launch_dot<float>(int, const float*, int64_t, const float*, const float*, int64_t, double*, int,
                                const GmresState*, hipStream_t);
template void launch_update<double>(int, double*, int64_t, const double*, const double*, double*, int64_t,
                                    const GmresState*, hipStream_t);
template void launch_update<float>(int, float*, int64_t, const float*, const float*, float*, int64_t,
                                   const GmresState*, hipStream_t);
template void launch_xupdate<double, double>(int, bool, const Geom&, const Coefs<double>&, const double*, int64_t,
                                             const GmresState*, double*, int, hipStream_t);
template void launch_xupdate<float, double>(int, bool, const Geom&, const Coefs<float>&, const double*, int64_t,
                                            const GmresState*, double*, int, hipStream_t);
template void launch_xupdate<float, float>(int, bool, const Geom&, const Coefs<float>&, const float*, int64_t,
                                           const GmresState*, double*, int, hipStream_t);
template void launch_copy_cast<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_copy_cast<double, double>(const double*, double*, int64_t, hipStream_t);

}  // namespace m1
