// Device-side building blocks of the implicit M1 step for gfx950.
//
// Closure (Sect. 2.2): f = |F|/(cE) clamped to 1, chi = (3+4f^2)/(5+2 xi),
// xi = sqrt(4-3f^2), D = (1-chi)/2 I + (3chi-1)/2 n n.  Wave speeds: Eq.
// "eigenvalues" (Sect. 3.1.1) with the transverse part f_perp^2.  HLL weights and
// the asymptotic correction alpha: Sect. 3.1.1 and Eq. "asymptoticCorrection".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m1 {

constexpr int kMaxRestart = 48;
constexpr double kDegenerate = 1e-14;     // lambda+ - lambda- <= kDegenerate*c: degenerate face
constexpr double kEFloor = 1e-300;        // E <= 0 in an iterate: f evaluated with this E
constexpr double kFgt1 = 1.0 + 1e-12;     // diagnostic threshold for |F| > c E

enum Bc { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_DIRICHLET = 2, BC_REFLECT = 3 };
enum Src { SRC_NONE = 0, SRC_ABS = 1, SRC_COUPLED = 2 };

template <int ND> struct Dims {
  static constexpr int nd = ND;
  static constexpr int nrad = 1 + ND;              // E, F_0..F_{ND-1}
  static constexpr int npair = ND * (ND + 1) / 2;   // independent entries of the symmetric P
  static constexpr int njac = npair * (1 + ND);     // dP_pair / d(E, F_l)
};

// index of the symmetric pair (d, m) in 0..npair-1
template <int ND> __host__ __device__ constexpr int pair_index(int d, int m) {
  return d <= m ? d * ND - d * (d - 1) / 2 + (m - d) : m * ND - m * (m - 1) / 2 + (d - m);
}

// Geometry shared by all kernels (passed by value).
struct Geom {
  int n[3];          // nx, ny, nz (nz = 1 in 2D)
  int rows;          // ny * nz
  int64_t N;         // cells
  int64_t stride[3]; // 1, nx, nx*ny
  int bc[6];
  int plane_n[3];    // number of cells on a plane normal to d
  int order3d;       // launch order of the cell kernels in 3D (set by the launchers; 0 rows, 1 pencils)
};

// Scheme constants and per-step scalars (passed by value).
struct Scheme {
  double c, c2, a_r, dx, dt;
  double s;          // dt/dx
  double cdt;        // c*dt
  double lambda_floor;
  int src;           // Src
  int wb;            // 1 well-balanced flux source, 0 centred
  int ap;            // asymptotic correction on/off
  int p1;            // P1 closure
  int newton;        // differentiate the tensor (1) or freeze it (0)
  double psi;        // pseudo-transient shift of the linear operator (0: none)
  double dx_c;       // dx / c (the asymptotic correction's scale)
  int wbb;           // well-balanced boundary closure (Eq. "boundaryCondition") on non-periodic faces
  double inv_cdx;    // 1 / (c dx)
};

__device__ __forceinline__ int64_t plane_index(int d, int i, int j, int k, const Geom& g) {
  return d == 0 ? (int64_t)k * g.n[1] + j : (d == 1 ? (int64_t)k * g.n[0] + i : (int64_t)j * g.n[0] + i);
}

// --- closure -----------------------------------------------------------------
template <int ND> struct ClosureState {
  double f;          // clamped |f|
  double nv[ND];     // unit direction (0 if F = 0)
  double chi;
  bool clamped;      // |F| >= cE (or E <= 0 with F != 0): f fixed at 1
  double geoE;       // (3chi-1)/2 * E/|F|: 3f/(c(2+xi)) unclamped, E/|F| clamped, 0 if F = 0
  double xi;         // sqrt(4 - 3 f^2)
  double rxi;        // 1 / (xi (xi + 2))
};

template <int ND>
__device__ __forceinline__ ClosureState<ND> closure(double E, const double* F, double c, int p1) {
  ClosureState<ND> s;
  double F2 = 0.0;
#pragma unroll
  for (int m = 0; m < ND; ++m) F2 += F[m] * F[m];
  const double Fm = sqrt(F2);
  const double Ep = fmax(E, kEFloor);
  const double fr = Fm / (c * Ep);
  s.clamped = !(fr < 1.0);
  s.f = s.clamped ? 1.0 : fr;
  // one reciprocal for the direction; divide where 1/|F| would overflow (subnormal |F|)
  if (Fm > 1e-300) {
    const double inv = 1.0 / Fm;
#pragma unroll
    for (int m = 0; m < ND; ++m) s.nv[m] = F[m] * inv;
  } else {
#pragma unroll
    for (int m = 0; m < ND; ++m) s.nv[m] = Fm > 0.0 ? F[m] / Fm : 0.0;
  }
  const double xi = sqrt(4.0 - 3.0 * s.f * s.f);
  s.xi = xi;
  s.rxi = 1.0 / (xi * (xi + 2.0));
  // 3chi - 1 = 6f^2/(2+xi) exactly, so (3chi-1)/2 E/|F| = 3f/(c(2+xi)) without the
  // cancellation of the literal product at small f
  s.geoE = s.clamped ? (Fm > 0.0 ? E / Fm : 0.0) : 3.0 * s.f / (c * (2.0 + xi));
  if (p1) {
    s.chi = 1.0 / 3.0;
  } else {
    s.chi = (3.0 + 4.0 * s.f * s.f) / (5.0 + 2.0 * xi);
  }
  return s;
}

// c^2 D_{dm} (the Eddington tensor times c^2)
template <int ND>
__device__ __forceinline__ double c2D(const ClosureState<ND>& s, int d, int m, double c2) {
  const double iso = 0.5 * (1.0 - s.chi);
  const double aniso = 0.5 * (3.0 * s.chi - 1.0);
  return c2 * ((d == m ? iso : 0.0) + aniso * s.nv[d] * s.nv[m]);
}

// Jacobian of c^2 P = c^2 D(E, F) E with respect to (E, F_0..F_{ND-1}), one row per
// symmetric pair.  Differentiating P_dm = E (1-chi)/2 delta_dm + E (3chi-1)/2 n_d n_m
// with f = |F|/(cE), n = F/|F|:
//   d/dE   : D_dm - f chi' (3/2 n_d n_m - delta_dm/2)
//   d/dF_l : chi'/c n_l (3/2 n_d n_m - delta_dm/2) + (3chi-1)/2 (E/|F|)(delta_dl n_m + delta_ml n_d - 2 n_d n_m n_l)
// chi' = dchi/df = (8f(5+2xi) + 6f(3+4f^2)/xi) / (5+2xi)^2, zero where f is clamped.
// With newton = 0 (tensor frozen) the rows reduce to (c^2 D_dm, 0, ..., 0).
template <int ND>
__device__ __forceinline__ void pressure_jacobian(const ClosureState<ND>& s, double c, double c2, int p1,
                                                  int newton, double* J /* npair*(1+ND) */) {
  double dchi = 0.0;
  if (!p1 && newton && !s.clamped) {
    const double f = s.f;
    const double xi = s.xi;
    const double den = 5.0 + 2.0 * xi;
    dchi = (8.0 * f * den + 6.0 * f * (3.0 + 4.0 * f * f) / xi) / (den * den);
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
#pragma unroll
    for (int m = d; m < ND; ++m) {
      const int p = pair_index<ND>(d, m);
      double* row = J + p * (1 + ND);
      const double shape = 1.5 * s.nv[d] * s.nv[m] - (d == m ? 0.5 : 0.0);
      if (!newton || p1) {
        row[0] = c2D<ND>(s, d, m, c2);
#pragma unroll
        for (int l = 0; l < ND; ++l) row[1 + l] = 0.0;
        continue;
      }
      row[0] = c2D<ND>(s, d, m, c2) - c2 * s.f * dchi * shape;
#pragma unroll
      for (int l = 0; l < ND; ++l) {
        const double geo = (d == l ? s.nv[m] : 0.0) + (m == l ? s.nv[d] : 0.0) - 2.0 * s.nv[d] * s.nv[m] * s.nv[l];
        row[1 + l] = c2 * (dchi / c * s.nv[l] * shape + s.geoE * geo);
      }
    }
  }
}

// Largest / smallest wave speed along direction d (Eq. "eigenvalues").
template <int ND>
__device__ __forceinline__ void wave_speeds(const ClosureState<ND>& s, int d, double c, int p1, double& lmax,
                                            double& lmin) {
  if (p1) {
    lmax = c * 0.57735026918962576451;
    lmin = -lmax;
    return;
  }
  const double f = s.f;
  const double fn = f * s.nv[d];
  const double fperp2 = fmax(f * f - fn * fn, 0.0);
  const double xi = s.xi;
  const double q = (xi - 1.0) * (xi + 2.0);
  // sqrt(2) sqrt(q (2q + 3 fperp^2)) / (sqrt(3) xi (xi+2)); fn / xi = fn (xi+2) / (xi (xi+2))
  const double root = 0.81649658092772603273 * sqrt(q * (2.0 * q + 3.0 * fperp2)) * s.rxi;
  const double adv = fn * (xi + 2.0) * s.rxi;
  lmax = c * (adv + root);
  lmin = c * (adv - root);
}

// HLL weights a = l+/(l+ - l-), dd = l+ l-/(l+ - l-) (b = 1 - a) and alpha.
struct FaceCoef {
  double a, dd, alpha;
};

__device__ __forceinline__ FaceCoef face_coef(double lmaxL, double lminL, double lmaxR, double lminR,
                                              double sigf, double fbar, const Scheme& sc) {
  double lp = fmax(0.0, fmax(lmaxL, lmaxR));
  double lm = fmin(0.0, fmin(lminL, lminR));
  if (sc.lambda_floor > 0.0) {
    lp = fmax(lp, sc.lambda_floor * sc.c);
    lm = fmin(lm, -sc.lambda_floor * sc.c);
  }
  FaceCoef fc;
  const double den = lp - lm;
  if (den <= kDegenerate * sc.c) {
    fc.a = 0.5;
    fc.dd = 0.0;
  } else {
    const double inv = 1.0 / den;
    fc.a = lp * inv;
    fc.dd = lp * lm * inv;
  }
  fc.alpha = sc.ap ? 1.0 / (1.0 - 3.0 * sigf * sc.dx_c * (1.0 - fbar * fbar) * fc.dd) : 1.0;
  return fc;
}

// --- ghost cells ----------------------------------------------------------------
// State of the ghost beside boundary cell (i,j,k) on face (d, side): outflow copy,
// reflect (normal flux negated) or Dirichlet plane (blended with the copy by mask).
template <int ND>
__device__ __forceinline__ void ghost_state(int bc, int d, const double* plane, const double* mask, int64_t pidx,
                                            int64_t pn, const double* Uin /* E,F */, double* Ug) {
#pragma unroll
  for (int c = 0; c < 1 + ND; ++c) Ug[c] = Uin[c];
  if (bc == BC_REFLECT) {
    Ug[1 + d] = -Ug[1 + d];
  } else if (bc == BC_DIRICHLET) {
    const double w = mask ? mask[pidx] : 1.0;
#pragma unroll
    for (int c = 0; c < 1 + ND; ++c) Ug[c] = w * plane[c * pn + pidx] + (1.0 - w) * Uin[c];
  }
}

// Linear map from a boundary cell's perturbation to its ghost's perturbation
// (diagonal): weight of component comp (0 = E, 1+m = F_m).
__device__ __forceinline__ double ghost_weight(int bc, int d, int comp, const double* mask, int64_t pidx) {
  if (bc == BC_REFLECT) return comp == 1 + d ? -1.0 : 1.0;
  if (bc == BC_DIRICHLET) return mask ? 1.0 - mask[pidx] : 0.0;
  return 1.0;  // outflow
}

// --- small dense blocks ----------------------------------------------------------
// Inverse of an NU x NU block by Gauss-Jordan elimination with partial pivoting
// (A is overwritten); false if a pivot is zero.
template <int NU>
__device__ __forceinline__ bool invert_block(double (&A)[NU][NU], double (&Ai)[NU][NU]) {
#pragma unroll
  for (int r = 0; r < NU; ++r)
#pragma unroll
    for (int c = 0; c < NU; ++c) Ai[r][c] = r == c ? 1.0 : 0.0;
  bool ok = true;
#pragma unroll
  for (int col = 0; col < NU; ++col) {
    // partial pivoting (rows col..NU-1)
    int piv = col;
    double best = fabs(A[col][col]);
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      const double v = fabs(A[r][col]);
      if (v > best) { best = v; piv = r; }
    }
    ok = ok && best > 0.0;
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      if (r == piv) {
#pragma unroll
        for (int c = 0; c < NU; ++c) {
          double t = A[col][c]; A[col][c] = A[r][c]; A[r][c] = t;
          t = Ai[col][c]; Ai[col][c] = Ai[r][c]; Ai[r][c] = t;
        }
      }
    }
    const double inv = 1.0 / A[col][col];
#pragma unroll
    for (int c = 0; c < NU; ++c) { A[col][c] *= inv; Ai[col][c] *= inv; }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
#pragma unroll
      for (int c = 0; c < NU; ++c) { A[r][c] -= f * A[col][c]; Ai[r][c] -= f * Ai[col][c]; }
    }
  }
  return ok;
}

}  // namespace m1
