// Scheme kernels for gfx950: linearisation setup (closure, HLL weights, alpha,
// tensor Jacobian), block-Jacobi assembly and apply, and the stencil kernel that
// evaluates the residual R(U) or applies the linearised operator A.
//
// Thread mapping of the stencil kernels: a 64 x 4 block covers 64 consecutive x
// cells (one wavefront per grid row, coalesced SoA loads) on 4 rows.  In 2D
// blockIdx.y walks rows.  In 3D the blocks are launched 1D in "pencil" order:
// workgroups go to the 8 XCDs round-robin by launch index and each XCD has its
// own L2, so launch index L takes work item (L % 8) * per + L / 8 (per = items / 8,
// rounded up) and every XCD owns a contiguous run of items; an item is one
// 64 x 4 x 1 tile, ordered z-fastest within chunks of kChunkZ planes, then x-tile,
// then y-tile, then z-chunk.  A cell's data is then read by its z-neighbours'
// blocks (the adjacent items) and its y-neighbours' blocks (a few dozen items
// away) while it is still in the XCD's L2; in row order a z-neighbour plane lies
// a whole plane (8 MB of Jacobians at 192^2) away.
#include <algorithm>
#include <cstdlib>
#include <string>

#include "m1_internal.h"

namespace m1 {

constexpr int TX = 64;
constexpr int TY = 4;
constexpr int kChunkZ = 16;

struct CellPos {
  int idx[3];
  int64_t cell;
};

__host__ __device__ inline int pencil_items(const Geom& g) {
  return ((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) * kChunkZ * ((g.n[2] + kChunkZ - 1) / kChunkZ);
}

__device__ __forceinline__ bool cell_pos(const Geom& g, CellPos& p) {
  if (g.order3d) {
    const int items = pencil_items(g);
    const int per = (items + 7) / 8;
    const int L = blockIdx.x;
    const int item = (L % 8) * per + L / 8;
    if (item >= items) return false;
    const int gx = (g.n[0] + TX - 1) / TX, gy = (g.n[1] + TY - 1) / TY;
    const int zl = item % kChunkZ;
    int r = item / kChunkZ;
    const int xt = r % gx;
    r /= gx;
    const int yt = r % gy;
    const int zc = r / gy;
    const int i = xt * TX + threadIdx.x, j = yt * TY + threadIdx.y, k = zc * kChunkZ + zl;
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return false;
    p.idx[0] = i;
    p.idx[1] = j;
    p.idx[2] = k;
    p.cell = ((int64_t)k * g.n[1] + j) * g.n[0] + i;
    return true;
  }
  const int i = blockIdx.x * TX + threadIdx.x;
  const int row = blockIdx.y * TY + threadIdx.y;
  if (i >= g.n[0] || row >= g.rows) return false;
  p.idx[0] = i;
  p.idx[1] = row % g.n[1];
  p.idx[2] = row / g.n[1];
  p.cell = (int64_t)row * g.n[0] + i;
  return true;
}

// Launch shape of the cell kernels (64 x 4 blocks): rows in 2D, XCD pencils in 3D
// (M1_ORDER3D=rows keeps the row order in 3D).
static int g_order3d = -1;
struct CellLaunch {
  Geom g;
  dim3 grd, blk;
};
static CellLaunch cell_launch(const Geom& g0) {
  if (g_order3d < 0) {
    const char* e = getenv("M1_ORDER3D");
    g_order3d = (e && std::string(e) == "rows") ? 0 : 1;
  }
  CellLaunch L;
  L.g = g0;
  L.blk = dim3(TX, TY);
  L.g.order3d = (g0.n[2] > 1 && g_order3d == 1) ? 1 : 0;
  if (L.g.order3d) L.grd = dim3(8 * ((pencil_items(g0) + 7) / 8));
  else L.grd = dim3((g0.n[0] + TX - 1) / TX, (g0.rows + TY - 1) / TY);
  return L;
}

// Neighbour along direction d on side (0 = lower, 1 = upper).
// kind: 0 interior/periodic neighbour (index in nb), 1 ghost.
struct Nb {
  int kind;
  int64_t nb;
  int64_t pidx;
};

__device__ __forceinline__ Nb neighbour(const Geom& g, const CellPos& p, int d, int side) {
  Nb r;
  const int id = p.idx[d];
  const int n = g.n[d];
  const int bc = g.bc[2 * d + side];
  r.pidx = plane_index(d, p.idx[0], p.idx[1], p.idx[2], g);
  if (side == 1) {
    if (id < n - 1) { r.kind = 0; r.nb = p.cell + g.stride[d]; }
    else if (bc == BC_PERIODIC) { r.kind = 0; r.nb = p.cell - (int64_t)(n - 1) * g.stride[d]; }
    else { r.kind = 1; r.nb = p.cell; }
  } else {
    if (id > 0) { r.kind = 0; r.nb = p.cell - g.stride[d]; }
    else if (bc == BC_PERIODIC) { r.kind = 0; r.nb = p.cell + (int64_t)(n - 1) * g.stride[d]; }
    else { r.kind = 1; r.nb = p.cell; }
  }
  return r;
}

// ----------------------------------------------------------------------------
// |f^n| per cell (the reduced flux alpha averages, Sect. 3.1.3)
// ----------------------------------------------------------------------------
template <int ND>
__global__ __launch_bounds__(256) void k_fn(Geom g, Scheme sc, const double* __restrict__ Un, double* __restrict__ fn) {
  CellPos p;
  if (!cell_pos(g, p)) return;
  double F[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) F[m] = Un[(1 + m) * g.N + p.cell];
  fn[p.cell] = closure<ND>(Un[p.cell], F, sc.c, sc.p1).f;
}

void launch_fn(int nd, const Geom& g, const Scheme& sc, const double* Un, double* fn, hipStream_t s) {
  const CellLaunch L = cell_launch(g);
  if (nd == 2) k_fn<2><<<L.grd, L.blk, 0, s>>>(L.g, sc, Un, fn);
  else k_fn<3><<<L.grd, L.blk, 0, s>>>(L.g, sc, Un, fn);
}

// ----------------------------------------------------------------------------
// a1: linearisation setup at the iterate U^k
// ----------------------------------------------------------------------------
template <int ND>
__device__ __forceinline__ void load_rad(const double* U, int64_t N, int64_t cell, double* out) {
#pragma unroll
  for (int c = 0; c < 1 + ND; ++c) out[c] = U[c * N + cell];
}

template <int ND, bool CPL>
__global__ __launch_bounds__(256) void k_setup(Geom g, Scheme sc, Coefs<double> cf, Bdry bd,
                                               const double* __restrict__ Uk, const double* __restrict__ Un,
                                               const double* __restrict__ fn) {
  using D = Dims<ND>;
  CellPos p;
  if (!cell_pos(g, p)) return;
  const int64_t N = g.N;
  double Us[1 + ND];
  load_rad<ND>(Uk, N, p.cell, Us);
  const ClosureState<ND> cs = closure<ND>(Us[0], Us + 1, sc.c, sc.p1);
  {
    double J[D::njac];
    pressure_jacobian<ND>(cs, sc.c, sc.c2, sc.p1, sc.newton, J);
#pragma unroll
    for (int q = 0; q < D::njac; ++q) cf.jac[q * N + p.cell] = J[q];
  }
  const double sig = cf.sigma[p.cell];
  const double fself = fn[p.cell];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double lmax, lmin;
    wave_speeds<ND>(cs, d, sc.c, sc.p1, lmax, lmin);
    // + face: right neighbour or ghost
    const Nb r = neighbour(g, p, d, 1);
    double lmaxR, lminR, sigR, fR;
    if (r.kind == 0) {
      double UR[1 + ND];
      load_rad<ND>(Uk, N, r.nb, UR);
      const ClosureState<ND> cr = closure<ND>(UR[0], UR + 1, sc.c, sc.p1);
      wave_speeds<ND>(cr, d, sc.c, sc.p1, lmaxR, lminR);
      sigR = cf.sigma[r.nb];
      fR = fn[r.nb];
    } else {
      const int face = 2 * d + 1;
      const int64_t pn = g.plane_n[d];
      double UG[1 + ND], UnS[1 + ND], UnG[1 + ND];
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], r.pidx, pn, Us, UG);
      const ClosureState<ND> cg = closure<ND>(UG[0], UG + 1, sc.c, sc.p1);
      wave_speeds<ND>(cg, d, sc.c, sc.p1, lmaxR, lminR);
      load_rad<ND>(Un, N, p.cell, UnS);
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], r.pidx, pn, UnS, UnG);
      fR = closure<ND>(UnG[0], UnG + 1, sc.c, sc.p1).f;
      sigR = sig;
      double J[D::njac];
      pressure_jacobian<ND>(cg, sc.c, sc.c2, sc.p1, sc.newton, J);
#pragma unroll
      for (int q = 0; q < D::njac; ++q) cf.gjac[cf.gjoff[face] + q * pn + r.pidx] = J[q];
    }
    const FaceCoef fc = face_coef(lmax, lmin, lmaxR, lminR, 0.5 * (sig + sigR), 0.5 * (fself + fR), sc);
    cf.face[(3 * d + 0) * N + p.cell] = fc.a;
    cf.face[(3 * d + 1) * N + p.cell] = fc.dd;
    cf.face[(3 * d + 2) * N + p.cell] = fc.alpha;
    // - face of the first cell on a non-periodic direction: ghost on the left
    const Nb l = neighbour(g, p, d, 0);
    if (l.kind == 1) {
      const int face = 2 * d;
      const int64_t pn = g.plane_n[d];
      double UG[1 + ND], UnS[1 + ND], UnG[1 + ND];
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], l.pidx, pn, Us, UG);
      const ClosureState<ND> cg = closure<ND>(UG[0], UG + 1, sc.c, sc.p1);
      double lmaxL, lminL;
      wave_speeds<ND>(cg, d, sc.c, sc.p1, lmaxL, lminL);
      load_rad<ND>(Un, N, p.cell, UnS);
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], l.pidx, pn, UnS, UnG);
      const double fL = closure<ND>(UnG[0], UnG + 1, sc.c, sc.p1).f;
      const FaceCoef fl = face_coef(lmaxL, lminL, lmax, lmin, sig, 0.5 * (fL + fself), sc);
      cf.lowface[cf.lowoff[d] + 0 * pn + l.pidx] = fl.a;
      cf.lowface[cf.lowoff[d] + 1 * pn + l.pidx] = fl.dd;
      cf.lowface[cf.lowoff[d] + 2 * pn + l.pidx] = fl.alpha;
      double J[D::njac];
      pressure_jacobian<ND>(cg, sc.c, sc.c2, sc.p1, sc.newton, J);
#pragma unroll
      for (int q = 0; q < D::njac; ++q) cf.gjac[cf.gjoff[face] + q * pn + l.pidx] = J[q];
    }
  }
  if (CPL) {
    const double T = Uk[(1 + ND) * N + p.cell];
    cf.kap[p.cell] = 4.0 * sc.a_r * T * T * T;
  }
}

void launch_setup(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                  const double* Uk, const double* Un, const double* fn, hipStream_t s) {
  const CellLaunch L = cell_launch(g);
  if (nd == 2) {
    if (cpl) k_setup<2, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, Un, fn);
    else k_setup<2, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, Un, fn);
  } else {
    if (cpl) k_setup<3, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, Un, fn);
    else k_setup<3, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, Un, fn);
  }
}

// Coefficients of the -face of a cell (the +face of its left neighbour, or the
// boundary plane).
template <typename R>
__device__ __forceinline__ void minus_face(const Geom& g, const Coefs<R>& cf, const Nb& l, int d, R& a, R& dd,
                                           R& al) {
  if (l.kind == 0) {
    a = cf.face[(3 * d + 0) * g.N + l.nb];
    dd = cf.face[(3 * d + 1) * g.N + l.nb];
    al = cf.face[(3 * d + 2) * g.N + l.nb];
  } else {
    const int64_t pn = g.plane_n[d];
    a = cf.lowface[cf.lowoff[d] + 0 * pn + l.pidx];
    dd = cf.lowface[cf.lowoff[d] + 1 * pn + l.pidx];
    al = cf.lowface[cf.lowoff[d] + 2 * pn + l.pidx];
  }
}

// ----------------------------------------------------------------------------
// Block-Jacobi: assemble the exact diagonal block of A and invert it
// ----------------------------------------------------------------------------

// STENCIL: instead of the inverse, write the explicit block stencil of the cell's
// row of A (the multigrid's finest level): block 0 the diagonal block, block
// 1 + 2d + side the coupling to the neighbour along d (side 0 lower, 1 upper; zero
// where the neighbour is a ghost, whose coupling is in the diagonal block, or the
// cell itself), entry (r, c) of block b at S[((b * NU + r) * NU + c) * N + cell].
template <int ND, bool CPL, bool STENCIL>
__global__ __launch_bounds__(256) void k_setup_bj(Geom g, Scheme sc, Coefs<double> cf, Bdry bd, double* __restrict__ S) {
  using Dm = Dims<ND>;
  constexpr int NR = 1 + ND;
  constexpr int NU = NR + (CPL ? 1 : 0);
  CellPos p;
  if (!cell_pos(g, p)) return;
  const int64_t N = g.N;
  auto put_block = [&](int blk, const double (&Bk)[NU][NU]) {
#pragma unroll
    for (int rr = 0; rr < NU; ++rr)
#pragma unroll
      for (int c = 0; c < NU; ++c) S[((blk * NU + rr) * NU + c) * N + p.cell] = Bk[rr][c];
  };
  double B[NU][NU];
#pragma unroll
  for (int r = 0; r < NU; ++r)
#pragma unroll
    for (int c = 0; c < NU; ++c) B[r][c] = (r == c && r < NR) ? 1.0 : 0.0;
  const double sig = cf.sigma[p.cell];
  const double s = sc.s;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    // Jacobian rows (d, m) of this cell
    double Js[ND][NR];
#pragma unroll
    for (int m = 0; m < ND; ++m)
#pragma unroll
      for (int k = 0; k < NR; ++k) Js[m][k] = cf.jac[(pair_index<ND>(d, m) * NR + k) * N + p.cell];
    // ---- + face ----
    const double a = cf.face[(3 * d + 0) * N + p.cell];
    const double dd = cf.face[(3 * d + 1) * N + p.cell];
    const double al = cf.face[(3 * d + 2) * N + p.cell];
    const double b = 1.0 - a;
    const Nb r = neighbour(g, p, d, 1);
    double gR[NR];
    double JR[ND][NR];
    double sigR;
    if (r.kind == 1) {
      const int face = 2 * d + 1;
      const int64_t pn = g.plane_n[d];
#pragma unroll
      for (int k = 0; k < NR; ++k) gR[k] = ghost_weight(g.bc[face], d, k, bd.mask[face], r.pidx);
#pragma unroll
      for (int m = 0; m < ND; ++m)
#pragma unroll
        for (int k = 0; k < NR; ++k) JR[m][k] = cf.gjac[cf.gjoff[face] + (pair_index<ND>(d, m) * NR + k) * pn + r.pidx];
      sigR = sig;
    } else {
      const double self = (r.nb == p.cell) ? 1.0 : 0.0;  // periodic with one cell
#pragma unroll
      for (int k = 0; k < NR; ++k) gR[k] = self;
#pragma unroll
      for (int m = 0; m < ND; ++m)
#pragma unroll
        for (int k = 0; k < NR; ++k) JR[m][k] = Js[m][k];
      sigR = cf.sigma[r.nb];
    }
    if (STENCIL) {
      double Nbk[NU][NU];
#pragma unroll
      for (int rr = 0; rr < NU; ++rr)
#pragma unroll
        for (int c = 0; c < NU; ++c) Nbk[rr][c] = 0.0;
      if (r.kind == 0 && r.nb != p.cell) {
        Nbk[0][0] = s * al * dd;
        Nbk[0][1 + d] = s * al * b;
#pragma unroll
        for (int m = 0; m < ND; ++m) {
#pragma unroll
          for (int k = 0; k < NR; ++k) Nbk[1 + m][k] = s * b * cf.jac[(pair_index<ND>(d, m) * NR + k) * N + r.nb];
          Nbk[1 + m][1 + m] += s * dd;
        }
        if (sc.wb) Nbk[1 + d][1 + d] += 0.25 * sc.cdt * (0.5 * (sig + sigR));
      }
      put_block(2 + 2 * d, Nbk);
    }
    B[0][0] += s * al * dd * (gR[0] - 1.0);
    B[0][1 + d] += s * al * (a + b * gR[1 + d]);
#pragma unroll
    for (int m = 0; m < ND; ++m) {
#pragma unroll
      for (int k = 0; k < NR; ++k) B[1 + m][k] += s * (a * Js[m][k] + b * JR[m][k] * gR[k]);
      B[1 + m][1 + m] += s * dd * (gR[1 + m] - 1.0);
    }
    // ---- - face ----
    const Nb l = neighbour(g, p, d, 0);
    double am, ddm, alm;
    minus_face(g, cf, l, d, am, ddm, alm);
    const double bm = 1.0 - am;
    double gL[NR];
    double JL[ND][NR];
    double sigL;
    if (l.kind == 1) {
      const int face = 2 * d;
      const int64_t pn = g.plane_n[d];
#pragma unroll
      for (int k = 0; k < NR; ++k) gL[k] = ghost_weight(g.bc[face], d, k, bd.mask[face], l.pidx);
#pragma unroll
      for (int m = 0; m < ND; ++m)
#pragma unroll
        for (int k = 0; k < NR; ++k) JL[m][k] = cf.gjac[cf.gjoff[face] + (pair_index<ND>(d, m) * NR + k) * pn + l.pidx];
      sigL = sig;
    } else {
      const double self = (l.nb == p.cell) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < NR; ++k) gL[k] = self;
#pragma unroll
      for (int m = 0; m < ND; ++m)
#pragma unroll
        for (int k = 0; k < NR; ++k) JL[m][k] = Js[m][k];
      sigL = cf.sigma[l.nb];
    }
    if (STENCIL) {
      double Nbk[NU][NU];
#pragma unroll
      for (int rr = 0; rr < NU; ++rr)
#pragma unroll
        for (int c = 0; c < NU; ++c) Nbk[rr][c] = 0.0;
      if (l.kind == 0 && l.nb != p.cell) {
        Nbk[0][0] = s * alm * ddm;
        Nbk[0][1 + d] = -s * alm * am;
#pragma unroll
        for (int m = 0; m < ND; ++m) {
#pragma unroll
          for (int k = 0; k < NR; ++k) Nbk[1 + m][k] = -s * am * cf.jac[(pair_index<ND>(d, m) * NR + k) * N + l.nb];
          Nbk[1 + m][1 + m] += s * ddm;
        }
        if (sc.wb) Nbk[1 + d][1 + d] += 0.25 * sc.cdt * (0.5 * (sig + sigL));
      }
      put_block(1 + 2 * d, Nbk);
    }
    B[0][1 + d] -= s * alm * (am * gL[1 + d] + bm);
    B[0][0] -= s * alm * ddm * (1.0 - gL[0]);
#pragma unroll
    for (int m = 0; m < ND; ++m) {
#pragma unroll
      for (int k = 0; k < NR; ++k) B[1 + m][k] -= s * (am * JL[m][k] * gL[k] + bm * Js[m][k]);
      B[1 + m][1 + m] -= s * ddm * (1.0 - gL[1 + m]);
    }
    if (sc.wb) {
      // self-coupling of the well-balanced source (hi: + face, lo: - face); with the
      // boundary closure a face to a ghost contributes -s/2 (q_R - q_L) with q = J x
      // (the ghost's x = g x of this cell)
      if (sc.wbb && (r.kind == 1 || l.kind == 1)) {
        if (r.kind == 1) {
#pragma unroll
          for (int k = 0; k < NR; ++k) B[1 + d][k] -= 0.5 * s * (JR[d][k] * gR[k] - Js[d][k]);
        } else {
          B[1 + d][1 + d] += 0.25 * sc.cdt * (0.5 * (sig + sigR) * (1.0 + gR[1 + d]));
        }
        if (l.kind == 1) {
#pragma unroll
          for (int k = 0; k < NR; ++k) B[1 + d][k] -= 0.5 * s * (Js[d][k] - JL[d][k] * gL[k]);
        } else {
          B[1 + d][1 + d] += 0.25 * sc.cdt * (0.5 * (sig + sigL) * (gL[1 + d] + 1.0));
        }
      } else {
        B[1 + d][1 + d] +=
            0.25 * sc.cdt * (0.5 * (sig + sigR) * (1.0 + gR[1 + d]) + 0.5 * (sig + sigL) * (gL[1 + d] + 1.0));
      }
    }
  }
  if (!sc.wb) {
#pragma unroll
    for (int m = 0; m < ND; ++m) B[1 + m][1 + m] += sc.cdt * sig;
  }
  if (sc.src == SRC_ABS) B[0][0] += sc.cdt * sig;
  if (CPL) {
    const double kap = cf.kap[p.cell];
    const double rcv = cf.rcv[p.cell];
    const double k = sc.cdt * sig;
    B[0][0] += k;
    B[0][NU - 1] -= k * kap;
    B[NU - 1][0] -= k;
    B[NU - 1][NU - 1] += rcv + k * kap;
  }
  if (sc.psi != 0.0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) B[r][r] += sc.psi;
    if (CPL) B[NU - 1][NU - 1] += sc.psi * cf.rcv[p.cell];
  }
  if (STENCIL) {
    put_block(0, B);
    return;
  }
  double Bi[NU][NU];
  invert_block<NU>(B, Bi);
#pragma unroll
  for (int rr = 0; rr < NU; ++rr)
#pragma unroll
    for (int c = 0; c < NU; ++c) cf.bjinv[(rr * NU + c) * N + p.cell] = Bi[rr][c];
}

void launch_setup_bj(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                     hipStream_t s) {
  const CellLaunch L = cell_launch(g);
  if (nd == 2) {
    if (cpl) k_setup_bj<2, true, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, nullptr);
    else k_setup_bj<2, false, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, nullptr);
  } else {
    if (cpl) k_setup_bj<3, true, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, nullptr);
    else k_setup_bj<3, false, false><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, nullptr);
  }
}

void launch_fine_stencil(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                         double* S, hipStream_t s) {
  const CellLaunch L = cell_launch(g);
  if (nd == 2) {
    if (cpl) k_setup_bj<2, true, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, S);
    else k_setup_bj<2, false, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, S);
  } else {
    if (cpl) k_setup_bj<3, true, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, S);
    else k_setup_bj<3, false, true><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, S);
  }
}

// ----------------------------------------------------------------------------
// a2 / a3: stencil kernel.  MODE 0: y = A x; 1: y = b - A x; 2: y = -R(U), x = U^k
// ----------------------------------------------------------------------------
template <int ND, bool CPL, int MODE, typename R, typename VI, typename VO>
__global__ __launch_bounds__(256) void k_stencil(Geom g, Scheme sc, Coefs<R> cf, Bdry bd, const VI* __restrict__ x,
                                                 const double* __restrict__ b, const double* __restrict__ Un,
                                                 VO* __restrict__ y, const int* __restrict__ skip) {
  constexpr int NR = 1 + ND;
  constexpr int NU = NR + (CPL ? 1 : 0);
  if (skip && *skip) return;
  CellPos p;
  if (!cell_pos(g, p)) return;
  const int64_t N = g.N;
  const R s = (R)sc.s;
  const R cdt = (R)sc.cdt;
  R xs[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) xs[c] = (R)x[c * N + p.cell];
  R ys[NU];
#pragma unroll
  for (int c = 0; c < NR; ++c) ys[c] = (MODE == 2) ? xs[c] - (R)Un[c * N + p.cell] : xs[c];
  if (CPL) ys[NU - 1] = (R)0;
  const R sig = cf.sigma[p.cell];

  // c^2 P_{dm} (residual: from the state) or its linearisation J x (apply) of a cell
  auto pressure_cell = [&](int d, int64_t cell, const R* xc, R* q) {
    if (MODE == 2) {
      double Fd[ND];
#pragma unroll
      for (int m = 0; m < ND; ++m) Fd[m] = (double)xc[1 + m];
      const ClosureState<ND> cs = closure<ND>((double)xc[0], Fd, sc.c, sc.p1);
#pragma unroll
      for (int m = 0; m < ND; ++m) q[m] = (R)(c2D<ND>(cs, d, m, sc.c2) * (double)xc[0]);
    } else {
#pragma unroll
      for (int m = 0; m < ND; ++m) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc += cf.jac[(pair_index<ND>(d, m) * NR + k) * N + cell] * xc[k];
        q[m] = acc;
      }
    }
  };
  auto pressure_ghost = [&](int d, int face, int64_t pidx, const R* xg, R* q) {
    if (MODE == 2) {
      double Fd[ND];
#pragma unroll
      for (int m = 0; m < ND; ++m) Fd[m] = (double)xg[1 + m];
      const ClosureState<ND> cs = closure<ND>((double)xg[0], Fd, sc.c, sc.p1);
#pragma unroll
      for (int m = 0; m < ND; ++m) q[m] = (R)(c2D<ND>(cs, d, m, sc.c2) * (double)xg[0]);
    } else {
      const int64_t pn = g.plane_n[d];
#pragma unroll
      for (int m = 0; m < ND; ++m) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc += cf.gjac[cf.gjoff[face] + (pair_index<ND>(d, m) * NR + k) * pn + pidx] * xg[k];
        q[m] = acc;
      }
    }
  };
  // state or perturbation of the ghost beside this cell
  auto ghost_value = [&](int d, int face, int64_t pidx, R* xg) {
    if (MODE == 2) {
      double Us[NR], Ug[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) Us[c] = (double)xs[c];
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], pidx, g.plane_n[d], Us, Ug);
#pragma unroll
      for (int c = 0; c < NR; ++c) xg[c] = (R)Ug[c];
    } else {
#pragma unroll
      for (int c = 0; c < NR; ++c) xg[c] = (R)ghost_weight(g.bc[face], d, c, bd.mask[face], pidx) * xs[c];
    }
  };

#pragma unroll
  for (int d = 0; d < ND; ++d) {
    R qs[ND];
    pressure_cell(d, p.cell, xs, qs);
    // right neighbour
    const Nb r = neighbour(g, p, d, 1);
    R xr[NR], qr[ND], sigR;
    if (r.kind == 0) {
#pragma unroll
      for (int c = 0; c < NR; ++c) xr[c] = (R)x[c * N + r.nb];
      pressure_cell(d, r.nb, xr, qr);
      sigR = cf.sigma[r.nb];
    } else {
      ghost_value(d, 2 * d + 1, r.pidx, xr);
      pressure_ghost(d, 2 * d + 1, r.pidx, xr, qr);
      sigR = sig;
    }
    // left neighbour
    const Nb l = neighbour(g, p, d, 0);
    R xl[NR], ql[ND], sigL;
    if (l.kind == 0) {
#pragma unroll
      for (int c = 0; c < NR; ++c) xl[c] = (R)x[c * N + l.nb];
      pressure_cell(d, l.nb, xl, ql);
      sigL = cf.sigma[l.nb];
    } else {
      ghost_value(d, 2 * d, l.pidx, xl);
      pressure_ghost(d, 2 * d, l.pidx, xl, ql);
      sigL = sig;
    }
    const R ap = cf.face[(3 * d + 0) * N + p.cell];
    const R ddp = cf.face[(3 * d + 1) * N + p.cell];
    const R alp = cf.face[(3 * d + 2) * N + p.cell];
    const R bp = (R)1 - ap;
    R am, ddm, alm;
    minus_face(g, cf, l, d, am, ddm, alm);
    const R bm = (R)1 - am;
    // energy flux (HLL with the asymptotic correction alpha)
    const R FEp = alp * (ap * xs[1 + d] + bp * xr[1 + d] + ddp * (xr[0] - xs[0]));
    const R FEm = alm * (am * xl[1 + d] + bm * xs[1 + d] + ddm * (xs[0] - xl[0]));
    ys[0] += s * (FEp - FEm);
    // radiative-flux fluxes
#pragma unroll
    for (int m = 0; m < ND; ++m) {
      const R FPp = ap * qs[m] + bp * qr[m] + ddp * (xr[1 + m] - xs[1 + m]);
      const R FPm = am * ql[m] + bm * qs[m] + ddm * (xs[1 + m] - xl[1 + m]);
      ys[1 + m] += s * (FPp - FPm);
    }
    if (sc.wb) {
      // {sigma F_d}: trapezoidal face average over the two faces normal to d (hi, lo: twice
      // the face values); with the boundary closure a face to a ghost takes
      // sigma F = -c (P_dd(right) - P_dd(left)) / dx (q = c^2 P)
      R hi = (R)0.5 * (sig + sigR) * (xs[1 + d] + xr[1 + d]);
      R lo = (R)0.5 * (sig + sigL) * (xl[1 + d] + xs[1 + d]);
      if (sc.wbb) {
        if (r.kind == 1) hi = -(R)2 * (qr[d] - qs[d]) * (R)sc.inv_cdx;
        if (l.kind == 1) lo = -(R)2 * (qs[d] - ql[d]) * (R)sc.inv_cdx;
      }
      ys[1 + d] += (R)0.25 * cdt * (hi + lo);
    }
  }
  if (!sc.wb) {
#pragma unroll
    for (int m = 0; m < ND; ++m) ys[1 + m] += cdt * sig * xs[1 + m];
  }
  if (sc.src == SRC_ABS) ys[0] += cdt * sig * xs[0];
  if (CPL) {
    const R T = xs[NU - 1];
    R exch;
    if (MODE == 2) {
      const double Td = (double)T;
      exch = (R)(sc.cdt * (double)sig * (sc.a_r * Td * Td * Td * Td - (double)xs[0]));
      ys[NU - 1] = cf.rcv[p.cell] * (T - (R)Un[(NU - 1) * N + p.cell]) + exch;
    } else {
      exch = cdt * sig * (cf.kap[p.cell] * T - xs[0]);
      ys[NU - 1] = cf.rcv[p.cell] * T + exch;
    }
    ys[0] -= exch;
  }
  if (MODE != 2 && sc.psi != 0.0) {
    // pseudo-transient shift psi * (mass coefficient) on every row
    const R psi = (R)sc.psi;
#pragma unroll
    for (int c = 0; c < NR; ++c) ys[c] += psi * xs[c];
    if (CPL) ys[NU - 1] += psi * cf.rcv[p.cell] * xs[NU - 1];
  }
#pragma unroll
  for (int c = 0; c < NU; ++c) {
    R v = ys[c];
    if (MODE == 1) v = (R)b[c * N + p.cell] - v;
    if (MODE == 2) v = -v;
    y[c * N + p.cell] = (VO)v;
  }
}

// ----------------------------------------------------------------------------
// a3, 2D, LDS-staged: a block owns a 64 x 16 tile; its (66 x 18) halo tile of
// the input vector x and of the linearised pressure q = (J x) for the three
// independent pairs (xx, xy, yy) is computed once into LDS (ghosts included),
// then every cell assembles its fluxes from LDS.  Each input element and each
// Jacobian entry is read from memory once per tile instead of once per use.
//
// Tile order: workgroups go to the 8 XCDs round-robin by launch index, and each
// XCD has its own L2.  Launch index L takes tile (L % 8) * per + L / 8 of the
// row-major tile order (per = tiles / 8, rounded up), so every XCD works on a
// contiguous band of tiles and the halo lines that neighbouring tiles share
// meet in the same L2 instead of being fetched once per XCD.
// ----------------------------------------------------------------------------
// Tiles are LX = 64 cells wide (one wavefront per row) and TR rows high (16 or 8), one
// cell per thread.
constexpr int LX = 64, LHX = LX + 2;

template <int TR> __host__ __device__ inline int tiles2d(int nx, int ny) {
  return ((nx + LX - 1) / LX) * ((ny + TR - 1) / TR);
}
template <int TR> inline dim3 grid2d_xcd(const Geom& g) { return dim3(8 * ((tiles2d<TR>(g.n[0], g.n[1]) + 7) / 8)); }

// tile (tbx, tby) of this workgroup; false for the padding workgroups
template <int TR> __device__ __forceinline__ bool xcd_tile(int nx, int ny, int& tbx, int& tby) {
  const int gx = (nx + LX - 1) / LX;
  const int gt = tiles2d<TR>(nx, ny);
  const int per = (gt + 7) / 8;
  const int T = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (T >= gt) return false;
  tbx = T % gx;
  tby = T / gx;
  return true;
}

// Stage the HX x HY halo tile whose corner is grid cell (i0, j0): the input x of
// every cell, from xf(cell, i, j, xv) for grid cells (a position beyond a
// non-periodic face takes the value of the boundary cell beside it times the ghost
// weights, the ghost of that cell; positions outside in both directions are never
// read), q = J x for the pressure pairs (xx, xy, yy), and sigma.
template <int NT, int HY, int HX, typename R, typename XF>
__device__ __forceinline__ void stage2d(const Geom& g, const Coefs<R>& cf, const Bdry& bd, int i0, int j0, XF&& xf,
                                        R (&sx)[3][HY][HX], R (&sq)[3][HY][HX], R (&ss)[HY][HX]) {
  constexpr int NR = 3;
  constexpr int NP = (HX * HY + NT - 1) / NT;   // positions per thread
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  // first every position's loads (all positions of a thread in flight together; a
  // ghost reads its boundary cell like an interior position), then the ghosts' fix-up
  // and the stores
  R xv[NP][NR], qv[NP][3], sv[NP];
  int face[NP], dd[NP];
  bool valid[NP];
  int64_t pidx[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int t = threadIdx.x + u * NT;
    const int li = t % HX, lj = t / HX;
    int gi = i0 + li, gj = j0 + lj;
    bool outx = gi < 0 || gi >= nx, outy = gj < 0 || gj >= ny;
    // periodic coordinates wrap first (a position outside in both directions is a grid
    // cell, or the ghost of one, when either direction is periodic)
    if (outx && g.bc[0] == BC_PERIODIC) { gi = (gi % nx + nx) % nx; outx = false; }
    if (outy && g.bc[2] == BC_PERIODIC) { gj = (gj % ny + ny) % ny; outy = false; }
    valid[u] = t < HX * HY && !(outx && outy);
    face[u] = -1;
    dd[u] = 0;
    if (outx) {
      dd[u] = 0;
      face[u] = gi < 0 ? 0 : 1;
      gi = gi < 0 ? 0 : nx - 1;
    } else if (outy) {
      dd[u] = 1;
      face[u] = gj < 0 ? 2 : 3;
      gj = gj < 0 ? 0 : ny - 1;
    }
    pidx[u] = dd[u] == 0 ? (int64_t)gj : (int64_t)gi;
#pragma unroll
    for (int c = 0; c < NR; ++c) xv[u][c] = (R)0;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) qv[u][pq] = (R)0;
    sv[u] = (R)0;
    if (valid[u]) {
      const int64_t cell = (int64_t)gj * nx + gi;
      xf(cell, gi, gj, xv[u]);
      sv[u] = cf.sigma[cell];
#pragma unroll
      for (int pq = 0; pq < 3; ++pq) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc += cf.jac[(pq * NR + k) * N + cell] * xv[u][k];
        qv[u][pq] = acc;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t >= HX * HY) continue;
    const int li = t % HX, lj = t / HX;
    if (valid[u] && face[u] >= 0) {
      const int f = face[u], d = dd[u];
      const int64_t pn = g.plane_n[d];
#pragma unroll
      for (int c = 0; c < NR; ++c) xv[u][c] *= (R)ghost_weight(g.bc[f], d, c, bd.mask[f], pidx[u]);
#pragma unroll
      for (int pq = 0; pq < 3; ++pq) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc += cf.gjac[cf.gjoff[f] + (pq * NR + k) * pn + pidx[u]] * xv[u][k];
        qv[u][pq] = acc;
      }
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) sx[c][lj][li] = xv[u][c];
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) sq[pq][lj][li] = qv[u][pq];
    ss[lj][li] = sv[u];
  }
}

// (a, dd, alpha) of the four faces of grid cell (i, j): its own +x and +y faces, then
// its -x and -y faces (the lower neighbours' + faces, or the boundary planes); loaded
// before the halo tile is staged, so that these loads overlap the staging's
template <typename R>
__device__ __forceinline__ void faces2d(const Geom& g, const Coefs<R>& cf, int i, int j, int64_t cell, R (&fc)[12]) {
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int e = 0; e < 3; ++e) fc[3 * d + e] = cf.face[(3 * d + e) * N + cell];
    const int id = d == 0 ? i : j, n = d == 0 ? nx : ny;
    const int64_t stride = d == 0 ? 1 : nx;
    if (id > 0 || g.bc[2 * d] == BC_PERIODIC) {
      const int64_t nb = id > 0 ? cell - stride : cell + (int64_t)(n - 1) * stride;
#pragma unroll
      for (int e = 0; e < 3; ++e) fc[6 + 3 * d + e] = cf.face[(3 * d + e) * N + nb];
    } else {
      const int64_t pidx = d == 0 ? (int64_t)j : (int64_t)i;
      const int64_t pn = g.plane_n[d];
#pragma unroll
      for (int e = 0; e < 3; ++e) fc[6 + 3 * d + e] = cf.lowface[cf.lowoff[d] + e * pn + pidx];
    }
  }
}

// ys = (A x) at grid cell (i, j), staged at (li, lj) of the halo tile; xs[NU] is the
// cell's own input (the radiation part as staged, the temperature from the caller),
// fc its face coefficients (faces2d).
template <bool CPL, int HY, int HX, typename R>
__device__ __forceinline__ void apply2d_cell(const Geom& g, const Scheme& sc, const Coefs<R>& cf,
                                             const R (&sx)[3][HY][HX], const R (&sq)[3][HY][HX],
                                             const R (&ss)[HY][HX], int li, int lj, int i, int j, int64_t cell,
                                             const R (&fc)[12], const R* xs, R* ys) {
  constexpr int NR = 3;
  constexpr int NU = NR + (CPL ? 1 : 0);
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  const R s = (R)sc.s;
  const R cdt = (R)sc.cdt;
#pragma unroll
  for (int c = 0; c < NR; ++c) ys[c] = xs[c];
  if (CPL) ys[NU - 1] = (R)0;
  const R sig = ss[lj][li];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    // neighbours in LDS; pressure pair index of (d, m) in 2D: (0,0)=0 (0,1)=1 (1,1)=2
    const int ri = d == 0 ? li + 1 : li, rj = d == 0 ? lj : lj + 1;
    const int mi = d == 0 ? li - 1 : li, mj = d == 0 ? lj : lj - 1;
    R xr[NR], xl[NR], qs[2], qr[2], ql[2];
#pragma unroll
    for (int c = 0; c < NR; ++c) { xr[c] = sx[c][rj][ri]; xl[c] = sx[c][mj][mi]; }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int pq = d + m;
      qs[m] = sq[pq][lj][li];
      qr[m] = sq[pq][rj][ri];
      ql[m] = sq[pq][mj][mi];
    }
    const R sigR = ss[rj][ri], sigL = ss[mj][mi];
    const R ap = fc[3 * d + 0], ddp = fc[3 * d + 1], alp = fc[3 * d + 2];
    const R am = fc[6 + 3 * d + 0], ddm = fc[6 + 3 * d + 1], alm = fc[6 + 3 * d + 2];
    const R bp = (R)1 - ap;
    const R bm = (R)1 - am;
    const R FEp = alp * (ap * xs[1 + d] + bp * xr[1 + d] + ddp * (xr[0] - xs[0]));
    const R FEm = alm * (am * xl[1 + d] + bm * xs[1 + d] + ddm * (xs[0] - xl[0]));
    ys[0] += s * (FEp - FEm);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const R FPp = ap * qs[m] + bp * qr[m] + ddp * (xr[1 + m] - xs[1 + m]);
      const R FPm = am * ql[m] + bm * qs[m] + ddm * (xs[1 + m] - xl[1 + m]);
      ys[1 + m] += s * (FPp - FPm);
    }
    if (sc.wb) {
      R hi = (R)0.5 * (sig + sigR) * (xs[1 + d] + xr[1 + d]);
      R lo = (R)0.5 * (sig + sigL) * (xl[1 + d] + xs[1 + d]);
      if (sc.wbb) {
        // boundary closure on faces to a ghost (the halo tile holds the ghost's q)
        const int id = d == 0 ? i : j, n = d == 0 ? nx : ny;
        if (id == n - 1 && g.bc[2 * d + 1] != BC_PERIODIC) hi = -(R)2 * (qr[d] - qs[d]) * (R)sc.inv_cdx;
        if (id == 0 && g.bc[2 * d] != BC_PERIODIC) lo = -(R)2 * (qs[d] - ql[d]) * (R)sc.inv_cdx;
      }
      ys[1 + d] += (R)0.25 * cdt * (hi + lo);
    }
  }
  if (!sc.wb) {
#pragma unroll
    for (int m = 0; m < 2; ++m) ys[1 + m] += cdt * sig * xs[1 + m];
  }
  if (sc.src == SRC_ABS) ys[0] += cdt * sig * xs[0];
  if (CPL) {
    const R T = xs[NU - 1];
    const R exch = cdt * sig * (cf.kap[cell] * T - xs[0]);
    ys[NU - 1] = cf.rcv[cell] * T + exch;
    ys[0] -= exch;
  }
  if (sc.psi != 0.0) {
    const R psi = (R)sc.psi;
#pragma unroll
    for (int c = 0; c < NR; ++c) ys[c] += psi * xs[c];
    if (CPL) ys[NU - 1] += psi * cf.rcv[cell] * xs[NU - 1];
  }
}

// PRE = true: the input is u and the operator is applied to z = M^{-1} u, the
// block-Jacobi solve done per staged cell (fused right preconditioning).
template <int TR, bool CPL, int MODE, bool PRE, typename R, typename VI, typename VO>
__global__ __launch_bounds__(LX * TR) void k_apply2d_lds(Geom g, Scheme sc, Coefs<R> cf, Bdry bd, const VI* __restrict__ x,
                                                     const double* __restrict__ b, VO* __restrict__ y,
                                                     const int* __restrict__ skip) {
  constexpr int NR = 3;
  constexpr int NU = NR + (CPL ? 1 : 0);
  if (skip && *skip) return;
  __shared__ R sx[NR][(TR + 2)][LHX];
  __shared__ R sq[3][(TR + 2)][LHX];
  __shared__ R ss[(TR + 2)][LHX];
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  int tbx, tby;
  if (!xcd_tile<TR>(nx, ny, tbx, tby)) return;
  // one cell per thread; its face coefficients are loaded with the staging
  const int tx = threadIdx.x % LX, ty = threadIdx.x / LX;
  const int i = tbx * LX + tx, j = tby * TR + ty;
  const bool inside = i < nx && j < ny;
  const int64_t cell = (int64_t)j * nx + i;
  R fc[12];
  if (inside) faces2d(g, cf, i, j, cell, fc);
  stage2d<LX * TR>(g, cf, bd, tbx * LX - 1, tby * TR - 1, [&](int64_t cell, int, int, R* xv) {
    if (PRE) {
      R uv[NU];
#pragma unroll
      for (int c = 0; c < NU; ++c) uv[c] = (R)x[c * N + cell];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        R acc = (R)0;
#pragma unroll
        for (int c = 0; c < NU; ++c) acc += cf.bjinv[(r * NU + c) * N + cell] * uv[c];
        xv[r] = acc;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NR; ++c) xv[c] = (R)x[c * N + cell];
    }
  }, sx, sq, ss);
  __syncthreads();
  // ---- fluxes ----
  if (inside) {
    const int li = tx + 1, lj = ty + 1;
    R xs[NU], ys[NU];
#pragma unroll
    for (int c = 0; c < NR; ++c) xs[c] = sx[c][lj][li];
    if (CPL) {
      if (PRE) {
        R acc = (R)0;
#pragma unroll
        for (int c = 0; c < NU; ++c) acc += cf.bjinv[((NU - 1) * NU + c) * N + cell] * (R)x[c * N + cell];
        xs[NU - 1] = acc;
      } else {
        xs[NU - 1] = (R)x[(NU - 1) * N + cell];
      }
    }
    apply2d_cell<CPL, (TR + 2), LHX, R>(g, sc, cf, sx, sq, ss, li, lj, i, j, cell, fc, xs, ys);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      R v = ys[c];
      if (MODE == 1) v = (R)b[c * N + cell] - v;
      y[c * N + cell] = (VO)v;
    }
  }
}

// ----------------------------------------------------------------------------
// Multigrid, finest level in 2D: damped block-Jacobi sweeps and the restricted
// residual on the LDS-staged operator, one kernel each.  The operator's input x is
// formed while staging:
//   XIN 0: x = zin;   XIN 1: x = zin + P zc (zin null: x = P zc);   XIN 2: x = omega M^{-1} r
// and the epilogue writes
//   OP 0: out = x + omega M^{-1} (r - A x)                     (one sweep)
//   OP 1: b1 = P^T (r - A x), z1 = omega D1^{-1} b1 (0 if !sm)  (level 1's right-hand
//         side and its first sweep from zero); x itself goes to out unless out is null
// P: piecewise-constant prolongation from 2 x 2 aggregates (coarse extents
// (n + 1) / 2, cell (i, j) in aggregate (i / 2, j / 2)).  Tile origins are even, so
// each aggregate lies inside one tile.  M^{-1}: the block-Jacobi inverses.
// ----------------------------------------------------------------------------
template <int TR, bool CPL, int OP, int XIN, typename R, typename TIN>
__global__ __launch_bounds__(LX * TR) void k_mg_sweep2d(Geom g, Scheme sc, Coefs<R> cf, Bdry bd,
                                                                const TIN* __restrict__ r, const R* __restrict__ zin,
                                                                const R* __restrict__ zc, R omega, R* __restrict__ out,
                                                                const R* __restrict__ dinv1, int sm, R* __restrict__ b1,
                                                                R* __restrict__ z1, const int* __restrict__ skip) {
  constexpr int NR = 3;
  constexpr int NU = NR + (CPL ? 1 : 0);
  static_assert(LX % 2 == 0 && TR % 2 == 0, "aggregates inside a tile");
  if (skip && *skip) return;
  __shared__ R sx[NR][(TR + 2)][LHX];
  __shared__ R sq[3][(TR + 2)][LHX];
  __shared__ R ss[(TR + 2)][LHX];
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  const int ncx = (nx + 1) / 2;
  const int64_t Nc = (int64_t)ncx * ((ny + 1) / 2);
  int tbx, tby;
  if (!xcd_tile<TR>(nx, ny, tbx, tby)) return;
  // input component k of grid cell (gi, gj)
  auto xin_of = [&](int64_t cell, int gi, int gj, int k) -> R {
    if (XIN == 0) return zin[k * N + cell];
    if (XIN == 1) return (zin ? zin[k * N + cell] : (R)0) + zc[k * Nc + (int64_t)(gj / 2) * ncx + gi / 2];
    R acc = (R)0;
#pragma unroll
    for (int c = 0; c < NU; ++c) acc += cf.bjinv[(k * NU + c) * N + cell] * (R)r[c * N + cell];
    return omega * acc;
  };
  const int tx = threadIdx.x % LX, ty = threadIdx.x / LX;
  const int i = tbx * LX + tx, j = tby * TR + ty;
  const bool inside = i < nx && j < ny;
  const int64_t cell = (int64_t)j * nx + i;
  R fc[12];
  if (inside) faces2d(g, cf, i, j, cell, fc);
  stage2d<LX * TR>(g, cf, bd, tbx * LX - 1, tby * TR - 1, [&](int64_t cell, int gi, int gj, R* xv) {
#pragma unroll
    for (int c = 0; c < NR; ++c) xv[c] = xin_of(cell, gi, gj, c);
  }, sx, sq, ss);
  __syncthreads();
  R res[NU];
  if (inside) {
    const int li = tx + 1, lj = ty + 1;
    R xs[NU], ys[NU];
#pragma unroll
    for (int c = 0; c < NR; ++c) xs[c] = sx[c][lj][li];
    if (CPL) xs[NU - 1] = xin_of(cell, i, j, NU - 1);
    apply2d_cell<CPL, (TR + 2), LHX, R>(g, sc, cf, sx, sq, ss, li, lj, i, j, cell, fc, xs, ys);
#pragma unroll
    for (int k = 0; k < NU; ++k) res[k] = (R)r[k * N + cell] - ys[k];
    if (OP == 0) {
#pragma unroll
      for (int rr = 0; rr < NU; ++rr) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NU; ++k) acc += cf.bjinv[(rr * NU + k) * N + cell] * res[k];
        out[rr * N + cell] = xs[rr] + omega * acc;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NU; ++k) res[k] = (R)0;
  }
  if (OP == 1) {
    // the operator's input is the pre-smoothed vector: written out when asked for
    if (out && inside) {
#pragma unroll
      for (int k = 0; k < NU; ++k) out[k * N + cell] = k < NR ? sx[k][ty + 1][tx + 1] : xin_of(cell, i, j, NU - 1);
    }
    // gather the residuals of each 2 x 2 aggregate through LDS (the halo tile is no
    // longer read once every thread has passed the barrier)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      if (k < NR) sx[k][ty][tx] = res[k];
      else sq[0][ty][tx] = res[k];
    }
    __syncthreads();
    if (inside && (tx % 2) == 0 && (ty % 2) == 0) {
      const int64_t I = (int64_t)(j / 2) * ncx + i / 2;
      R acc[NU];
#pragma unroll
      for (int k = 0; k < NU; ++k) acc[k] = (R)0;
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          if (i + cx >= nx || j + cy >= ny) continue;
#pragma unroll
          for (int k = 0; k < NU; ++k) acc[k] += k < NR ? sx[k][ty + cy][tx + cx] : sq[0][ty + cy][tx + cx];
        }
#pragma unroll
      for (int k = 0; k < NU; ++k) b1[k * Nc + I] = acc[k];
#pragma unroll
      for (int rr = 0; rr < NU; ++rr) {
        R z = (R)0;
        if (sm) {
#pragma unroll
          for (int k = 0; k < NU; ++k) z += dinv1[(rr * NU + k) * Nc + I] * acc[k];
          z *= omega;
        }
        z1[rr * Nc + I] = z;
      }
    }
  }
}

// rows per 2D tile: 64 x 16 tiles of 1024 threads (64 x 8 tiles of 512 threads, two
// blocks per CU, measured slower for the two-sweep multigrid kernel at 512^2 -- 17.0
// against 15.3 us -- and equal for the fused apply at 1024^2)
constexpr int kTileRows = 16;

static int g_apply_variant = -1;  // -1: read M1_APPLY_KERNEL once ("lds" default in 2D, "direct")

static bool use_lds_2d() {
  if (g_apply_variant < 0) {
    const char* e = getenv("M1_APPLY_KERNEL");
    g_apply_variant = (e && std::string(e) == "direct") ? 0 : 1;
  }
  return g_apply_variant == 1;
}

template <typename R, typename VI, typename VO>
void launch_apply(int nd, bool cpl, int mode, const Geom& g, const Scheme& sc, const Coefs<R>& cf, const Bdry& bd,
                  const VI* x, const double* b, VO* y, hipStream_t s, const int* skip) {
  if (nd == 2 && use_lds_2d()) {
#define M1_LDS(CPL_, MODE_)                                                                                  \
  k_apply2d_lds<kTileRows, CPL_, MODE_, false, R, VI, VO><<<grid2d_xcd<kTileRows>(g), LX * kTileRows, 0, s>>>( \
      g, sc, cf, bd, x, b, y, skip);
    if (cpl) { if (mode == 0) M1_LDS(true, 0) else M1_LDS(true, 1) }
    else { if (mode == 0) M1_LDS(false, 0) else M1_LDS(false, 1) }
#undef M1_LDS
    return;
  }
  const CellLaunch L = cell_launch(g);
#define M1_ST(ND_, CPL_, MODE_) k_stencil<ND_, CPL_, MODE_, R, VI, VO><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, x, b, nullptr, y, skip)
  if (nd == 2) {
    if (cpl) { if (mode == 0) M1_ST(2, true, 0); else M1_ST(2, true, 1); }
    else { if (mode == 0) M1_ST(2, false, 0); else M1_ST(2, false, 1); }
  } else {
    if (cpl) { if (mode == 0) M1_ST(3, true, 0); else M1_ST(3, true, 1); }
    else { if (mode == 0) M1_ST(3, false, 0); else M1_ST(3, false, 1); }
  }
#undef M1_ST
}

void launch_residual(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<double>& cf, const Bdry& bd,
                     const double* Uk, const double* Un, double* out, hipStream_t s) {
  const CellLaunch L = cell_launch(g);
  if (nd == 2) {
    if (cpl) k_stencil<2, true, 2, double, double, double><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, nullptr, Un, out, nullptr);
    else k_stencil<2, false, 2, double, double, double><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, nullptr, Un, out, nullptr);
  } else {
    if (cpl) k_stencil<3, true, 2, double, double, double><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, nullptr, Un, out, nullptr);
    else k_stencil<3, false, 2, double, double, double><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf, bd, Uk, nullptr, Un, out, nullptr);
  }
}

// The same with two operator applications per launch: the input is staged with a
// halo of two cells (68 x 20), the first sweep x1 = x + omega M^{-1} (r - A x) is
// taken on the tile and its one-cell ring (66 x 18: the ring's sweep is
// recomputed by each of the tiles that share it) and kept in LDS with q1 = J x1,
// the ghosts beyond non-periodic faces are refreshed from the swept boundary cells,
// and the epilogue of OP is applied to x1 on the tile.  Halves the finest-level
// launches of a cycle.
template <int TR, bool CPL, int OP, int XIN, typename R, typename TIN>
__global__ __launch_bounds__(LX * TR) void k_mg_sweep2d_x2(Geom g, Scheme sc, Coefs<R> cf, Bdry bd,
                                                                   const TIN* __restrict__ r, const R* __restrict__ zin,
                                                                   const R* __restrict__ zc, R omega,
                                                                   R* __restrict__ out, const R* __restrict__ dinv1,
                                                                   int sm, R* __restrict__ b1, R* __restrict__ z1,
                                                                   const int* __restrict__ skip) {
  constexpr int NR = 3;
  constexpr int NU = NR + (CPL ? 1 : 0);
  if (skip && *skip) return;
  __shared__ R sx0[NR][(TR + 4)][(LX + 4)];
  __shared__ R sq0[3][(TR + 4)][(LX + 4)];
  __shared__ R ss0[(TR + 4)][(LX + 4)];
  __shared__ R sx1[NR][(TR + 2)][LHX];
  __shared__ R sq1[3][(TR + 2)][LHX];
  __shared__ R ss1[(TR + 2)][LHX];
  __shared__ R sT1[CPL ? (TR + 2) : 1][CPL ? LHX : 1];
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  const int ncx = (nx + 1) / 2;
  const int64_t Nc = (int64_t)ncx * ((ny + 1) / 2);
  const bool perx = g.bc[0] == BC_PERIODIC, pery = g.bc[2] == BC_PERIODIC;
  int tbx, tby;
  if (!xcd_tile<TR>(nx, ny, tbx, tby)) return;
  auto xin_of = [&](int64_t cell, int gi, int gj, int k) -> R {
    if (XIN == 0) return zin[k * N + cell];
    if (XIN == 1) return (zin ? zin[k * N + cell] : (R)0) + zc[k * Nc + (int64_t)(gj / 2) * ncx + gi / 2];
    R acc = (R)0;
#pragma unroll
    for (int c = 0; c < NU; ++c) acc += cf.bjinv[(k * NU + c) * N + cell] * (R)r[c * N + cell];
    return omega * acc;
  };
  stage2d<LX * TR>(g, cf, bd, tbx * LX - 2, tby * TR - 2, [&](int64_t cell, int gi, int gj, R* xv) {
#pragma unroll
    for (int c = 0; c < NR; ++c) xv[c] = xin_of(cell, gi, gj, c);
  }, sx0, sq0, ss0);
  __syncthreads();
  // ---- first sweep on the tile and its ring (grid cells only; ghosts below) ----
  // Thread t sweeps its own tile cell first (the cell of its second application) and,
  // for t < the ring's 2 (LX + 2) + 2 TR positions, one ring cell.  In FP32 the own
  // cell's face coefficients, right-hand side and block inverse stay in registers for
  // the second application instead of being read again.
  constexpr bool KEEP = sizeof(R) == 4;
  constexpr int NRING = 2 * LHX + 2 * TR;
  const int tx = threadIdx.x % LX, ty = threadIdx.x / LX;
  R kf[KEEP ? 12 : 1], kr[KEEP ? NU : 1], kb[KEEP ? NU * NU : 1];
  auto sweep1 = [&](int pi, int pj, bool keep) {
    int gi = tbx * LX - 1 + pi, gj = tby * TR - 1 + pj;
    const bool outx = gi < 0 || gi >= nx, outy = gj < 0 || gj >= ny;
    if ((outx && !perx) || (outy && !pery)) return;   // ghost or unused corner
    if (outx) gi = (gi + nx) % nx;
    if (outy) gj = (gj + ny) % ny;
    const int64_t cell = (int64_t)gj * nx + gi;
    R xs[NU], ys[NU];
#pragma unroll
    for (int c = 0; c < NR; ++c) xs[c] = sx0[c][pj + 1][pi + 1];
    if (CPL) xs[NU - 1] = xin_of(cell, gi, gj, NU - 1);
    R fr[12];
    faces2d(g, cf, gi, gj, cell, fr);
    apply2d_cell<CPL, (TR + 4), (LX + 4), R>(g, sc, cf, sx0, sq0, ss0, pi + 1, pj + 1, gi, gj, cell, fr, xs, ys);
    R rv[NU], bj[NU * NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) rv[k] = (R)r[k * N + cell];
#pragma unroll
    for (int k = 0; k < NU * NU; ++k) bj[k] = cf.bjinv[k * N + cell];
    R res[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) res[k] = rv[k] - ys[k];
    R x1[NU];
#pragma unroll
    for (int rr = 0; rr < NU; ++rr) {
      R acc = (R)0;
#pragma unroll
      for (int k = 0; k < NU; ++k) acc += bj[rr * NU + k] * res[k];
      x1[rr] = xs[rr] + omega * acc;
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) sx1[c][pj][pi] = x1[c];
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      R acc = (R)0;
#pragma unroll
      for (int k = 0; k < NR; ++k) acc += cf.jac[(pq * NR + k) * N + cell] * x1[k];
      sq1[pq][pj][pi] = acc;
    }
    ss1[pj][pi] = ss0[pj + 1][pi + 1];
    if (CPL) sT1[pj][pi] = x1[NU - 1];
    if (KEEP && keep) {
#pragma unroll
      for (int k = 0; k < 12; ++k) kf[k % (KEEP ? 12 : 1)] = fr[k];
#pragma unroll
      for (int k = 0; k < NU; ++k) kr[k % (KEEP ? NU : 1)] = rv[k];
#pragma unroll
      for (int k = 0; k < NU * NU; ++k) kb[k % (KEEP ? NU * NU : 1)] = bj[k];
    }
  };
  sweep1(tx + 1, ty + 1, true);
  if ((int)threadIdx.x < NRING) {
    const int k = threadIdx.x;
    int pi, pj;
    if (k < LHX) { pi = k; pj = 0; }
    else if (k < 2 * LHX) { pi = k - LHX; pj = TR + 1; }
    else if (k < 2 * LHX + TR) { pi = 0; pj = k - 2 * LHX + 1; }
    else { pi = LHX - 1; pj = k - 2 * LHX - TR + 1; }
    sweep1(pi, pj, false);
  }
  __syncthreads();
  // ---- ghosts of the swept boundary cells (the positions just beyond a non-periodic
  // face; positions further out and corners are never read) ----
  for (int t = threadIdx.x; t < LHX * (TR + 2); t += (LX * TR)) {
    const int pi = t % LHX, pj = t / LHX;
    int gi = tbx * LX - 1 + pi, gj = tby * TR - 1 + pj;
    bool outx = gi < 0 || gi >= nx, outy = gj < 0 || gj >= ny;
    if (outx && perx) { gi = (gi % nx + nx) % nx; outx = false; }
    if (outy && pery) { gj = (gj % ny + ny) % ny; outy = false; }
    if (!(outx || outy) || (outx && outy)) continue;   // a grid cell, or never read
    if ((outx && gi != -1 && gi != nx) || (outy && gj != -1 && gj != ny)) continue;
    int face, d, bi = pi, bj = pj;
    int64_t pidx;
    if (outx) {
      d = 0;
      face = gi < 0 ? 0 : 1;
      bi = gi < 0 ? pi + 1 : pi - 1;
      pidx = gj;
    } else {
      d = 1;
      face = gj < 0 ? 2 : 3;
      bj = gj < 0 ? pj + 1 : pj - 1;
      pidx = gi;
    }
    const int64_t pn = g.plane_n[d];
    R xv[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) xv[c] = sx1[c][bj][bi] * (R)ghost_weight(g.bc[face], d, c, bd.mask[face], pidx);
#pragma unroll
    for (int c = 0; c < NR; ++c) sx1[c][pj][pi] = xv[c];
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      R acc = (R)0;
#pragma unroll
      for (int k = 0; k < NR; ++k) acc += cf.gjac[cf.gjoff[face] + (pq * NR + k) * pn + pidx] * xv[k];
      sq1[pq][pj][pi] = acc;
    }
    ss1[pj][pi] = ss1[bj][bi];
  }
  __syncthreads();
  // ---- second application on the tile ----
  const int i = tbx * LX + tx, j = tby * TR + ty;
  const bool inside = i < nx && j < ny;
  const int64_t cell = (int64_t)j * nx + i;
  R res[NU];
  if (inside) {
    const int li = tx + 1, lj = ty + 1;
    R xs[NU], ys[NU];
#pragma unroll
    for (int c = 0; c < NR; ++c) xs[c] = sx1[c][lj][li];
    if (CPL) xs[NU - 1] = sT1[lj][li];
    R fc[12];
    if (KEEP) {
#pragma unroll
      for (int k = 0; k < 12; ++k) fc[k] = kf[k % (KEEP ? 12 : 1)];
    } else {
      faces2d(g, cf, i, j, cell, fc);   // read by the first sweep just before: cache hits
    }
    apply2d_cell<CPL, (TR + 2), LHX, R>(g, sc, cf, sx1, sq1, ss1, li, lj, i, j, cell, fc, xs, ys);
#pragma unroll
    for (int k = 0; k < NU; ++k) res[k] = (KEEP ? kr[k % (KEEP ? NU : 1)] : (R)r[k * N + cell]) - ys[k];
    if (OP == 0) {
#pragma unroll
      for (int rr = 0; rr < NU; ++rr) {
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < NU; ++k)
          acc += (KEEP ? kb[(rr * NU + k) % (KEEP ? NU * NU : 1)] : cf.bjinv[(rr * NU + k) * N + cell]) * res[k];
        out[rr * N + cell] = xs[rr] + omega * acc;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NU; ++k) res[k] = (R)0;
  }
  if (OP == 1) {
    // the operator's input (the first sweep's result) is the pre-smoothed vector
    if (out && inside) {
#pragma unroll
      for (int k = 0; k < NU; ++k) out[k * N + cell] = k < NR ? sx1[k][ty + 1][tx + 1] : sT1[CPL ? ty + 1 : 0][CPL ? tx + 1 : 0];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      if (k < NR) sx0[k][ty][tx] = res[k];
      else sq0[0][ty][tx] = res[k];
    }
    __syncthreads();
    if (inside && (tx % 2) == 0 && (ty % 2) == 0) {
      const int64_t I = (int64_t)(j / 2) * ncx + i / 2;
      R acc[NU];
#pragma unroll
      for (int k = 0; k < NU; ++k) acc[k] = (R)0;
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          if (i + cx >= nx || j + cy >= ny) continue;
#pragma unroll
          for (int k = 0; k < NU; ++k) acc[k] += k < NR ? sx0[k][ty + cy][tx + cx] : sq0[0][ty + cy][tx + cx];
        }
#pragma unroll
      for (int k = 0; k < NU; ++k) b1[k * Nc + I] = acc[k];
#pragma unroll
      for (int rr = 0; rr < NU; ++rr) {
        R z = (R)0;
        if (sm) {
#pragma unroll
          for (int k = 0; k < NU; ++k) z += dinv1[(rr * NU + k) * Nc + I] * acc[k];
          z *= omega;
        }
        z1[rr * Nc + I] = z;
      }
    }
  }
}

template <typename R, typename TIN>
bool launch_mg_sweep2d(int nd, bool cpl, int op, int xin, int ns, const Geom& g, const Scheme& sc, const Coefs<R>& cf,
                       const Bdry& bd, const TIN* r, const R* zin, const R* zc, R omega, R* out, const R* dinv1, int sm,
                       R* b1, R* z1, hipStream_t s, const int* skip) {
  if (!fused_apply_available(nd) || op < 0 || op > 1 || xin < 0 || xin > 2 || ns < 1 || ns > 2) return false;
#define M1_SW_T(TY_, CPL_, OP_, XIN_)                                                                                 \
  {                                                                                                                   \
    if (ns == 2)                                                                                                      \
      k_mg_sweep2d_x2<TY_, CPL_, OP_, XIN_, R, TIN><<<grid2d_xcd<TY_>(g), LX * TY_, 0, s>>>(                          \
          g, sc, cf, bd, r, zin, zc, omega, out, dinv1, sm, b1, z1, skip);                                            \
    else                                                                                                              \
      k_mg_sweep2d<TY_, CPL_, OP_, XIN_, R, TIN><<<grid2d_xcd<TY_>(g), LX * TY_, 0, s>>>(                             \
          g, sc, cf, bd, r, zin, zc, omega, out, dinv1, sm, b1, z1, skip);                                            \
  }
#define M1_SW(CPL_, OP_, XIN_) M1_SW_T(kTileRows, CPL_, OP_, XIN_)
#define M1_SW_X(CPL_, OP_) \
  { if (xin == 0) M1_SW(CPL_, OP_, 0) else if (xin == 1) M1_SW(CPL_, OP_, 1) else M1_SW(CPL_, OP_, 2) }
  if (cpl) { if (op == 0) M1_SW_X(true, 0) else M1_SW_X(true, 1) }
  else { if (op == 0) M1_SW_X(false, 0) else M1_SW_X(false, 1) }
#undef M1_SW_X
#undef M1_SW
#undef M1_SW_T
  return true;
}
template bool launch_mg_sweep2d<double, double>(int, bool, int, int, int, const Geom&, const Scheme&, const Coefs<double>&,
                                                const Bdry&, const double*, const double*, const double*, double,
                                                double*, const double*, int, double*, double*, hipStream_t, const int*);
template bool launch_mg_sweep2d<float, double>(int, bool, int, int, int, const Geom&, const Scheme&, const Coefs<float>&,
                                               const Bdry&, const double*, const float*, const float*, float, float*,
                                               const float*, int, float*, float*, hipStream_t, const int*);
template bool launch_mg_sweep2d<float, float>(int, bool, int, int, int, const Geom&, const Scheme&, const Coefs<float>&,
                                              const Bdry&, const float*, const float*, const float*, float, float*,
                                              const float*, int, float*, float*, hipStream_t, const int*);

// ----------------------------------------------------------------------------
// a4: z = M^{-1} r with the stored block inverses
// ----------------------------------------------------------------------------
template <int NU, typename R, typename VI, typename VO>
__global__ __launch_bounds__(256) void k_bj(int64_t N, const R* __restrict__ inv, const VI* __restrict__ r,
                                            VO* __restrict__ z, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  R rv[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) rv[c] = (R)r[c * N + cell];
#pragma unroll
  for (int rr = 0; rr < NU; ++rr) {
    R acc = (R)0;
#pragma unroll
    for (int c = 0; c < NU; ++c) acc += inv[(rr * NU + c) * N + cell] * rv[c];
    z[rr * N + cell] = (VO)acc;
  }
}

template <typename R, typename VI, typename VO>
void launch_bj(int nd, bool cpl, const Geom& g, const Coefs<R>& cf, const VI* r, VO* z, hipStream_t s,
               const int* skip) {
  const int nu = 1 + nd + (cpl ? 1 : 0);
  const int blk = 256;
  const int64_t grd = (g.N + blk - 1) / blk;
  switch (nu) {
    case 3: k_bj<3, R, VI, VO><<<grd, blk, 0, s>>>(g.N, cf.bjinv, r, z, skip); break;
    case 4: k_bj<4, R, VI, VO><<<grd, blk, 0, s>>>(g.N, cf.bjinv, r, z, skip); break;
    case 5: k_bj<5, R, VI, VO><<<grd, blk, 0, s>>>(g.N, cf.bjinv, r, z, skip); break;
  }
}

__global__ void k_convert(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

void launch_convert(const double* src, float* dst, int64_t n, hipStream_t s) {
  const int64_t grd = std::min<int64_t>((n + 255) / 256, 4096);
  k_convert<<<grd, 256, 0, s>>>(src, dst, n);
}

bool fused_apply_available(int nd) { return nd == 2 && use_lds_2d(); }

// y = A M^{-1} u in one kernel (2D, LDS path); returns false when not available
template <typename R, typename VI, typename VO>
bool launch_apply_pre(int nd, bool cpl, const Geom& g, const Scheme& sc, const Coefs<R>& cf, const Bdry& bd,
                      const VI* u, VO* y, hipStream_t s, const int* skip) {
  if (!use_lds_2d()) return false;
  if (nd != 2) return false;
  const dim3 grd2 = grid2d_xcd<kTileRows>(g);
  if (cpl) k_apply2d_lds<kTileRows, true, 0, true, R, VI, VO><<<grd2, LX * kTileRows, 0, s>>>(g, sc, cf, bd, u, nullptr, y, skip);
  else k_apply2d_lds<kTileRows, false, 0, true, R, VI, VO><<<grd2, LX * kTileRows, 0, s>>>(g, sc, cf, bd, u, nullptr, y, skip);
  return true;
}

template bool launch_apply_pre<double, double, double>(int, bool, const Geom&, const Scheme&, const Coefs<double>&,
                                                       const Bdry&, const double*, double*, hipStream_t, const int*);
template bool launch_apply_pre<float, double, double>(int, bool, const Geom&, const Scheme&, const Coefs<float>&,
                                                      const Bdry&, const double*, double*, hipStream_t, const int*);
template bool launch_apply_pre<float, float, float>(int, bool, const Geom&, const Scheme&, const Coefs<float>&,
                                                    const Bdry&, const float*, float*, hipStream_t, const int*);

// ----------------------------------------------------------------------------
// Explicit and semi-implicit time steps (Sect. 3.1), one fused kernel per step:
// the residual R(U^n) of the scheme evaluated at U^k = U^n (closure, HLL speeds
// and alpha of the time-n state, computed on the fly, no stored face
// coefficients), then the per-cell update from b = -R(U^n).  There R(U^n) is
// the flux divergence H plus the source part S(U^n), so U^n - H = U^n + b + S(U^n):
//   explicit:      U = U^n + b on the radiation rows, T = T^n + b_T/(rho c_v)
//   semi-implicit: sources at the new level, per cell (centred flux source):
//     F_m = (F_m^n - H_Fm)/(1 + k), k = c dt sigma
//     E   = (E^n - H_E)/(1 + k) with absorption, E^n - H_E without a source
//     coupled: E* = E^n - H_E, T the root of rho c_v (T - T^n) + k/(1+k) (a_r T^4 - E*)
//              (Newton from T^n), then E = (E* + k a_r T^4)/(1 + k)
// ----------------------------------------------------------------------------
constexpr int kTNewtonMax = 60;

template <int NR, bool CPL, bool SEMI>
__device__ __forceinline__ void time_update_cell(const Scheme& sc, double sig, double rc, const double* un,
                                                 const double* b, double* out) {
  if (!SEMI) {
#pragma unroll
    for (int q = 0; q < NR; ++q) out[q] = un[q] + b[q];
    if (CPL) out[NR] = un[NR] + b[NR] / rc;
    return;
  }
  const double k = sc.cdt * sig;
  const double inv = 1.0 / (1.0 + k);
#pragma unroll
  for (int q = 1; q < NR; ++q) out[q] = (un[q] + b[q] + k * un[q]) * inv;
  if (CPL) {
    const double En = un[0], Tn = un[NR];
    const double Es = En + b[0] - k * (sc.a_r * Tn * Tn * Tn * Tn - En);
    const double w = k * inv;
    double T = Tn;
    for (int it = 0; it < kTNewtonMax; ++it) {
      const double T3 = T * T * T;
      const double gT = rc * (T - Tn) + w * (sc.a_r * T3 * T - Es);
      const double dT = gT / (rc + 4.0 * w * sc.a_r * T3);
      T -= dT;
      if (fabs(dT) <= 1e-15 * fabs(T)) break;
    }
    out[NR] = T;
    out[0] = (Es + k * sc.a_r * T * T * T * T) * inv;
  } else if (sc.src == SRC_ABS) {
    out[0] = (un[0] + b[0] + k * un[0]) * inv;
  } else {
    out[0] = un[0] + b[0];
  }
}

// What a face along direction d needs from the cell (or ghost) on one side.
template <int ND> struct Side {
  double u[1 + ND];  // E, F
  double q[ND];      // c^2 D_{dm} E, m = 0..ND-1
  double lmax, lmin, f, sig;
};

template <int ND>
__device__ __forceinline__ void make_side(const ClosureState<ND>& cs, const double* u, double sig, int d,
                                          const Scheme& sc, Side<ND>& S) {
#pragma unroll
  for (int c = 0; c < 1 + ND; ++c) S.u[c] = u[c];
#pragma unroll
  for (int m = 0; m < ND; ++m) S.q[m] = c2D<ND>(cs, d, m, sc.c2) * u[0];
  wave_speeds<ND>(cs, d, sc.c, sc.p1, S.lmax, S.lmin);
  S.f = cs.f;
  S.sig = sig;
}

// HLL flux (with alpha on the energy row) through the face between L and R along d
template <int ND>
__device__ __forceinline__ void face_flux(const Side<ND>& L, const Side<ND>& R, int d, const Scheme& sc, double& FE,
                                          double* FP) {
  const FaceCoef fc = face_coef(L.lmax, L.lmin, R.lmax, R.lmin, 0.5 * (L.sig + R.sig), 0.5 * (L.f + R.f), sc);
  const double b = 1.0 - fc.a;
  FE = fc.alpha * (fc.a * L.u[1 + d] + b * R.u[1 + d] + fc.dd * (R.u[0] - L.u[0]));
#pragma unroll
  for (int m = 0; m < ND; ++m) FP[m] = fc.a * L.q[m] + b * R.q[m] + fc.dd * (R.u[1 + m] - L.u[1 + m]);
}

// residual contributions of direction d (fluxes and the well-balanced source)
template <int ND>
__device__ __forceinline__ void add_direction(const Side<ND>& Lf, const Side<ND>& S, const Side<ND>& Rt, int d,
                                              const Scheme& sc, double* ys) {
  double FEp, FEm, FPp[ND], FPm[ND];
  face_flux<ND>(S, Rt, d, sc, FEp, FPp);
  face_flux<ND>(Lf, S, d, sc, FEm, FPm);
  ys[0] += sc.s * (FEp - FEm);
#pragma unroll
  for (int m = 0; m < ND; ++m) ys[1 + m] += sc.s * (FPp[m] - FPm[m]);
  if (sc.wb)
    ys[1 + d] += 0.25 * sc.cdt * (0.5 * (S.sig + Rt.sig) * (S.u[1 + d] + Rt.u[1 + d]) +
                                  0.5 * (S.sig + Lf.sig) * (Lf.u[1 + d] + S.u[1 + d]));
}

// sources of the residual at U^k = U^n, then the update of one cell
template <int ND, bool CPL, bool SEMI>
__device__ __forceinline__ void finish_cell(const Scheme& sc, double sig, double rc, const double* xs, double* ys,
                                            double* out) {
  constexpr int NR = 1 + ND;
  constexpr int NU = NR + (CPL ? 1 : 0);
  if (!sc.wb) {
#pragma unroll
    for (int m = 0; m < ND; ++m) ys[1 + m] += sc.cdt * sig * xs[1 + m];
  }
  if (sc.src == SRC_ABS) ys[0] += sc.cdt * sig * xs[0];
  if (CPL) {
    const double T = xs[NU - 1];
    const double exch = sc.cdt * sig * (sc.a_r * T * T * T * T - xs[0]);
    ys[NU - 1] = exch;
    ys[0] -= exch;
  }
  double b[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) b[c] = -ys[c];
  time_update_cell<NR, CPL, SEMI>(sc, sig, rc, xs, b, out);
}

// Direct form (3D, and 2D when the LDS tile is switched off): a thread per cell
// evaluates the closures of its 2 ND neighbours itself.
template <int ND, bool CPL, bool SEMI>
__global__ __launch_bounds__(256) void k_step_direct(Geom g, Scheme sc, const double* __restrict__ sigma,
                                                     const double* __restrict__ rcv, Bdry bd,
                                                     const double* __restrict__ Un, double* __restrict__ Uo) {
  constexpr int NR = 1 + ND;
  constexpr int NU = NR + (CPL ? 1 : 0);
  CellPos p;
  if (!cell_pos(g, p)) return;
  const int64_t N = g.N;
  double xs[NU], ys[NU], out[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) { xs[c] = Un[c * N + p.cell]; ys[c] = 0.0; }
  const double sig = sigma[p.cell];
  const ClosureState<ND> cs = closure<ND>(xs[0], xs + 1, sc.c, sc.p1);
  // neighbour (or ghost) of this cell on side `side` of direction d
  auto side_of = [&](int d, int side, Side<ND>& S) {
    const Nb r = neighbour(g, p, d, side);
    double u[NR];
    double sg;
    if (r.kind == 0) {
#pragma unroll
      for (int c = 0; c < NR; ++c) u[c] = Un[c * N + r.nb];
      sg = sigma[r.nb];
    } else {
      const int face = 2 * d + side;
      ghost_state<ND>(g.bc[face], d, bd.plane[face], bd.mask[face], r.pidx, g.plane_n[d], xs, u);
      sg = sig;
    }
    make_side<ND>(closure<ND>(u[0], u + 1, sc.c, sc.p1), u, sg, d, sc, S);
  };
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    Side<ND> S, Lf, Rt;
    make_side<ND>(cs, xs, sig, d, sc, S);
    side_of(d, 1, Rt);
    side_of(d, 0, Lf);
    add_direction<ND>(Lf, S, Rt, d, sc, ys);
  }
  finish_cell<ND, CPL, SEMI>(sc, sig, CPL ? rcv[p.cell] : 1.0, xs, ys, out);
#pragma unroll
  for (int c = 0; c < NU; ++c) Uo[c * N + p.cell] = out[c];
}

// 2D LDS form: a workgroup owns a 64 x SY tile (XCD-aware tile order, as the
// operator kernel).  Every cell of its (64+2) x (SY+2) halo tile is staged once
// with its closure (state, c^2 D E, speeds along x and y, f, sigma: 12 doubles),
// then each face of the tile gets its HLL flux once, and each cell sums its four
// faces: one closure per cell and one flux per face, instead of one per
// neighbour and two per face.  The face fluxes are kept in registers until the
// closure data is dead, then written over it, so the LDS footprint stays at the
// 12 staged doubles per halo cell (38 KB at SY = 4).
template <int SY> __host__ __device__ inline int step_tiles(int nx, int ny) {
  return ((nx + LX - 1) / LX) * ((ny + SY - 1) / SY);
}

template <bool CPL, bool SEMI, int SY>
__global__ __launch_bounds__(LX * SY) void k_step2d_lds(Geom g, Scheme sc, const double* __restrict__ sigma,
                                                        const double* __restrict__ rcv, Bdry bd,
                                                        const double* __restrict__ Un, double* __restrict__ Uo) {
  constexpr int NR = 3;
  constexpr int NU = NR + (CPL ? 1 : 0);
  constexpr int SHY = SY + 2;
  constexpr int NT = LX * SY;
  constexpr int PL = SHY * LHX;                       // one staged quantity
  constexpr int NFX = (LX + 1) * SY, NFY = LX * (SY + 1);
  constexpr int KF = (NFX + NFY + NT - 1) / NT;       // faces per thread
  // staged quantities k: 0-2 E, F_x, F_y; 3-5 c^2 D E (xx, xy, yy); 6-9 speeds
  // (x max, x min, y max, y min); 10 f; 11 sigma.  Face fluxes reuse k = 3..10.
  static_assert(3 * (NFX + NFY) <= 8 * PL, "face fluxes must fit over the dead closure data");
  __shared__ double sb[12 * PL];
  auto at = [&](int k, int b, int a) -> double& { return sb[k * PL + b * LHX + a]; };
  double* fx = sb + 3 * PL;          // [3][SY][LX+1]: face a is left of cell column a
  double* fy = fx + 3 * NFX;         // [3][SY+1][LX]: face b is below cell row b
  const int64_t N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  const int gx = (nx + LX - 1) / LX;
  const int gt = step_tiles<SY>(nx, ny);
  const int per = (gt + 7) / 8;
  const int T = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (T >= gt) return;
  const int tbx = T % gx, tby = T / gx;
  const int i0 = tbx * LX - 1, j0 = tby * SY - 1;
  // ---- stage the halo tile with its closures ----
  for (int t = threadIdx.x; t < PL; t += NT) {
    const int li = t % LHX, lj = t / LHX;
    int gi = i0 + li, gj = j0 + lj;
    const bool outx = gi < 0 || gi >= nx, outy = gj < 0 || gj >= ny;
    double u[NR] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0}, lam[4] = {0.0, 0.0, 0.0, 0.0}, f = 0.0, sg = 0.0;
    // halo corners and cells beyond the ghost layer stay zero (their faces are not used)
    if (!(outx && outy) && gi < nx + 1 && gj < ny + 1) {
      int face = -1, d = 0;
      if (outx) {
        d = 0;
        if (g.bc[0] == BC_PERIODIC) gi = (gi + nx) % nx;
        else { face = gi < 0 ? 0 : 1; gi = gi < 0 ? 0 : nx - 1; }
      } else if (outy) {
        d = 1;
        if (g.bc[2] == BC_PERIODIC) gj = (gj + ny) % ny;
        else { face = gj < 0 ? 2 : 3; gj = gj < 0 ? 0 : ny - 1; }
      }
      const int64_t cell = (int64_t)gj * nx + gi;
#pragma unroll
      for (int c = 0; c < NR; ++c) u[c] = Un[c * N + cell];
      sg = sigma[cell];
      if (face >= 0) {
        double ub[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) ub[c] = u[c];
        const int64_t pidx = d == 0 ? (int64_t)gj : (int64_t)gi;
        ghost_state<2>(g.bc[face], d, bd.plane[face], bd.mask[face], pidx, g.plane_n[d], ub, u);
      }
      const ClosureState<2> cs = closure<2>(u[0], u + 1, sc.c, sc.p1);
      q[0] = c2D<2>(cs, 0, 0, sc.c2) * u[0];
      q[1] = c2D<2>(cs, 0, 1, sc.c2) * u[0];
      q[2] = c2D<2>(cs, 1, 1, sc.c2) * u[0];
      wave_speeds<2>(cs, 0, sc.c, sc.p1, lam[0], lam[1]);
      wave_speeds<2>(cs, 1, sc.c, sc.p1, lam[2], lam[3]);
      f = cs.f;
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) at(c, lj, li) = u[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) at(3 + c, lj, li) = q[c];
#pragma unroll
    for (int c = 0; c < 4; ++c) at(6 + c, lj, li) = lam[c];
    at(10, lj, li) = f;
    at(11, lj, li) = sg;
  }
  __syncthreads();
  auto load = [&](int d, int a, int b, Side<2>& S) {
#pragma unroll
    for (int c = 0; c < NR; ++c) S.u[c] = at(c, b, a);
    S.q[0] = at(3 + d, b, a);
    S.q[1] = at(4 + d, b, a);
    S.lmax = at(6 + 2 * d, b, a);
    S.lmin = at(7 + 2 * d, b, a);
    S.f = at(10, b, a);
    S.sig = at(11, b, a);
  };
  // ---- one flux per face, held in registers ----
  double ff[KF][3];
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int t = threadIdx.x + k * NT;
    if (t < NFX + NFY) {
      Side<2> L, R;
      if (t < NFX) {
        const int a = t % (LX + 1), r = t / (LX + 1);
        load(0, a, r + 1, L);
        load(0, a + 1, r + 1, R);
        face_flux<2>(L, R, 0, sc, ff[k][0], &ff[k][1]);
      } else {
        const int v = t - NFX;
        const int a = v % LX, b = v / LX;
        load(1, a + 1, b, L);
        load(1, a + 1, b + 1, R);
        face_flux<2>(L, R, 1, sc, ff[k][0], &ff[k][1]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int t = threadIdx.x + k * NT;
    if (t < NFX) {
#pragma unroll
      for (int c = 0; c < 3; ++c) fx[c * NFX + t] = ff[k][c];
    } else if (t < NFX + NFY) {
#pragma unroll
      for (int c = 0; c < 3; ++c) fy[c * NFY + (t - NFX)] = ff[k][c];
    }
  }
  __syncthreads();
  // ---- each cell: divergence of its four faces, sources, update ----
  const int tx = threadIdx.x % LX, ty = threadIdx.x / LX;
  const int i = tbx * LX + tx, j = tby * SY + ty;
  if (i >= nx || j >= ny) return;
  const int64_t cell = (int64_t)j * nx + i;
  const int li = tx + 1, lj = ty + 1;
  double xs[NU], ys[NU], out[NU];
#pragma unroll
  for (int c = 0; c < NR; ++c) xs[c] = at(c, lj, li);
  if (CPL) xs[NU - 1] = Un[(NU - 1) * N + cell];
#pragma unroll
  for (int c = 0; c < NU; ++c) ys[c] = 0.0;
  const double sig = at(11, lj, li);
  // x: faces tx (minus) and tx + 1 (plus) of row ty; y: faces ty and ty + 1 of column tx
  const int xm = ty * (LX + 1) + tx, ym = ty * LX + tx;
#pragma unroll
  for (int c = 0; c < 3; ++c) ys[c] += sc.s * (fx[c * NFX + xm + 1] - fx[c * NFX + xm]);
  if (sc.wb)
    ys[1] += 0.25 * sc.cdt * (0.5 * (sig + at(11, lj, li + 1)) * (xs[1] + at(1, lj, li + 1)) +
                              0.5 * (sig + at(11, lj, li - 1)) * (at(1, lj, li - 1) + xs[1]));
#pragma unroll
  for (int c = 0; c < 3; ++c) ys[c] += sc.s * (fy[c * NFY + ym + LX] - fy[c * NFY + ym]);
  if (sc.wb)
    ys[2] += 0.25 * sc.cdt * (0.5 * (sig + at(11, lj + 1, li)) * (xs[2] + at(2, lj + 1, li)) +
                              0.5 * (sig + at(11, lj - 1, li)) * (at(2, lj - 1, li) + xs[2]));
  finish_cell<2, CPL, SEMI>(sc, sig, CPL ? rcv[cell] : 1.0, xs, ys, out);
#pragma unroll
  for (int c = 0; c < NU; ++c) Uo[c * N + cell] = out[c];
}

// tile height of the 2D step kernel (cells per tile 64 x sy; M1_STEP_TILE_Y = 4 or 8)
static int step_tile_y() {
  static int sy = 0;
  if (!sy) {
    const char* e = getenv("M1_STEP_TILE_Y");
    sy = (e && atoi(e) == 4) ? 4 : 8;
  }
  return sy;
}

void launch_time_step(int nd, bool cpl, bool semi, const Geom& g, const Scheme& sc, const Coefs<double>& cf,
                      const Bdry& bd, const double* Un, double* Uo, hipStream_t s) {
  if (nd == 2 && use_lds_2d()) {
    const int sy = step_tile_y();
#define M1_TS(CPL_, SEMI_, SY_)                                                                       \
  k_step2d_lds<CPL_, SEMI_, SY_><<<dim3(8 * ((step_tiles<SY_>(g.n[0], g.n[1]) + 7) / 8)), LX * SY_, 0, s>>>( \
      g, sc, cf.sigma, cf.rcv, bd, Un, Uo)
#define M1_TS_Y(CPL_, SEMI_) \
  if (sy == 4) M1_TS(CPL_, SEMI_, 4); else M1_TS(CPL_, SEMI_, 8)
    if (cpl) { if (semi) { M1_TS_Y(true, true); } else { M1_TS_Y(true, false); } }
    else { if (semi) { M1_TS_Y(false, true); } else { M1_TS_Y(false, false); } }
#undef M1_TS_Y
#undef M1_TS
    return;
  }
  const CellLaunch L = cell_launch(g);
#define M1_TD(ND_, CPL_, SEMI_) k_step_direct<ND_, CPL_, SEMI_><<<L.grd, L.blk, 0, s>>>(L.g, sc, cf.sigma, cf.rcv, bd, Un, Uo)
  if (nd == 2) {
    if (cpl) { if (semi) M1_TD(2, true, true); else M1_TD(2, true, false); }
    else { if (semi) M1_TD(2, false, true); else M1_TD(2, false, false); }
  } else {
    if (cpl) { if (semi) M1_TD(3, true, true); else M1_TD(3, true, false); }
    else { if (semi) M1_TD(3, false, true); else M1_TD(3, false, false); }
  }
#undef M1_TD
}

// ----------------------------------------------------------------------------
// Velocity-dependent sources (Sect. 2.3), added explicitly after the radiation
// step (Sect. 3.2, step 3), cell-centred:
//   S_E(u) = sigma/c [u.F + E u.u + u.(u.P)]
//   S_F(u) = sigma u.P + sigma a_r T^4 u + sigma/c^2 u (u.F),   P = D(E, F) E
//   E += dt S_E,  F += dt c S_F;  other rows copied (without a T row there is no
//   emission term).  U -> V, distinct buffers.
// ----------------------------------------------------------------------------
template <int ND, bool CPL>
__global__ __launch_bounds__(256) void k_velocity_sources(int64_t N, Scheme sc, const double* __restrict__ sigma,
                                                          const double* __restrict__ U, const double* __restrict__ ux,
                                                          const double* __restrict__ uy, const double* __restrict__ uz,
                                                          double dt, double* __restrict__ V) {
  constexpr int NU = 1 + ND + (CPL ? 1 : 0);
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  const double E = U[cell];
  double F[ND], u[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) F[m] = U[(1 + m) * N + cell];
  u[0] = ux[cell];
  u[1] = uy[cell];
  if (ND == 3) u[ND - 1] = uz[cell];
  const double sig = sigma[cell];
  const ClosureState<ND> cs = closure<ND>(E, F, sc.c, sc.p1);
  const double iso = 0.5 * (1.0 - cs.chi), aniso = 0.5 * (3.0 * cs.chi - 1.0);
  double un = 0.0, uF = 0.0, uu = 0.0;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    un += u[m] * cs.nv[m];
    uF += u[m] * F[m];
    uu += u[m] * u[m];
  }
  double uP[ND], uuP = 0.0;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    uP[m] = E * (iso * u[m] + aniso * un * cs.nv[m]);
    uuP += u[m] * uP[m];
  }
  double emis = 0.0;
  if (CPL) {
    const double T = U[(NU - 1) * N + cell];
    emis = sc.a_r * T * T * T * T;
    V[(NU - 1) * N + cell] = T;
  }
  V[cell] = E + dt * (sig / sc.c * (uF + E * uu + uuP));
#pragma unroll
  for (int m = 0; m < ND; ++m)
    V[(1 + m) * N + cell] = F[m] + dt * sc.c * (sig * uP[m] + sig * emis * u[m] + sig / sc.c2 * u[m] * uF);
}

void launch_velocity_sources(int nd, bool cpl, const Geom& g, const Scheme& sc, const double* sigma, const double* U,
                             const double* const* u, double dt, double* V, hipStream_t s) {
  const int64_t grd = (g.N + 255) / 256;
  if (nd == 2) {
    if (cpl) k_velocity_sources<2, true><<<grd, 256, 0, s>>>(g.N, sc, sigma, U, u[0], u[1], nullptr, dt, V);
    else k_velocity_sources<2, false><<<grd, 256, 0, s>>>(g.N, sc, sigma, U, u[0], u[1], nullptr, dt, V);
  } else {
    if (cpl) k_velocity_sources<3, true><<<grd, 256, 0, s>>>(g.N, sc, sigma, U, u[0], u[1], u[2], dt, V);
    else k_velocity_sources<3, false><<<grd, 256, 0, s>>>(g.N, sc, sigma, U, u[0], u[1], u[2], dt, V);
  }
}

// explicit instantiations
template void launch_apply<double, double, double>(int, bool, int, const Geom&, const Scheme&, const Coefs<double>&,
                                                   const Bdry&, const double*, const double*, double*, hipStream_t, const int*);
template void launch_apply<float, float, double>(int, bool, int, const Geom&, const Scheme&, const Coefs<float>&,
                                                 const Bdry&, const float*, const double*, double*, hipStream_t, const int*);
template void launch_apply<float, float, float>(int, bool, int, const Geom&, const Scheme&, const Coefs<float>&,
                                                const Bdry&, const float*, const double*, float*, hipStream_t, const int*);
template void launch_apply<float, double, double>(int, bool, int, const Geom&, const Scheme&, const Coefs<float>&,
                                                  const Bdry&, const double*, const double*, double*, hipStream_t, const int*);
template void launch_apply<double, double, float>(int, bool, int, const Geom&, const Scheme&, const Coefs<double>&,
                                                  const Bdry&, const double*, const double*, float*, hipStream_t, const int*);
template void launch_bj<double, double, double>(int, bool, const Geom&, const Coefs<double>&, const double*, double*,
                                                hipStream_t, const int*);
template void launch_bj<float, double, float>(int, bool, const Geom&, const Coefs<float>&, const double*, float*,
                                              hipStream_t, const int*);
template void launch_bj<float, float, float>(int, bool, const Geom&, const Coefs<float>&, const float*, float*,
                                             hipStream_t, const int*);

}  // namespace m1
