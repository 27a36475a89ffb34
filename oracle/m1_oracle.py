"""CPU FP64 oracle for one backward-Euler step of the AP / well-balanced M1 scheme.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the GPU
path is checked against.  Only tests, the smoke entry and the benchmark's CPU
baseline may import it; the product path never calls it and shares no code
with it (the only common module is ``workloads``, which draws inputs).

What it computes (Bloch et al., "An asymptotic-preserving and well-balanced
scheme for the M1 model", A&A 2021):

* M1 closure: reduced flux f = |F|/(cE), Eddington factor
  chi = (3 + 4f^2) / (5 + 2 sqrt(4 - 3f^2)), Eddington tensor
  D = (1-chi)/2 I + (3chi-1)/2 n n  (Sect. 2.2).  f > 1 is clamped to 1 inside
  the tensor (Sect. 6, ionisation-front test).
* Wave speeds of the moment system (Eq. "eigenvalues", Sect. 3.1.1), HLL
  speeds lambda+ = max(0, lambda_max), lambda- = min(0, lambda_min).
* HLL numerical fluxes F* and P* (Sect. 3.1.1) with the asymptotic correction
  alpha on the energy flux (Eq. "asymptoticCorrection", Sect. 3.1.3).
* The flux source term {sigma F}: centred (Eq. "wb_naive") or well balanced
  (Eq. "wb_smart", face averages of sigma and F, Sect. 3.1.2).
* Radiation/matter exchange c sigma (a_r T^4 - E) on the energy and gas
  internal-energy rows (Eqs. "momentModel", "internalEnergyEqua").
* The implicit system of Sect. 3.1.1 solved by Newton iterations (Sect. 3.3.1)
  with the closure frozen at each iterate and T^4 linearised, each linear
  system solved by restarted, right-preconditioned GMRES (Sect. 3.3.2 for
  right preconditioning) with modified Gram-Schmidt and a block-Jacobi
  preconditioner (the exact diagonal n_u x n_u block of the operator).

Readings where the paper is silent are listed in the module docstring of each
function and collected in the design notes: Davis two-sided speed estimate,
iterate-level closure for the speeds in alpha, |f^n| averaged for alpha,
3D speeds with f_perp^2, F_m's source on the faces normal to m, ghost-cell
boundaries, degenerate faces (lambda+ = lambda- = 0 -> a = b = 1/2, dd = 0).

Array layout: grids are numpy arrays shaped (ny, nx) or (nz, ny, nx); states
are component-major (n_u, *grid) with components (E, F_x, F_y[, F_z][, T]).
Direction d (0 = x, 1 = y, 2 = z) is grid axis ndim-1-d.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEGENERATE_REL = 1e-14     # lambda+ - lambda- <= this * c  ->  degenerate face
E_FLOOR_CLOSURE = 1e-300   # E <= 0 in an iterate: f computed with this floor
F_GT_1_REL = 1.0 + 1e-12   # diagnostic: a cell counts as f > 1 when |F| > (1 + 1e-12) c E


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass
class Scheme:
    n: tuple
    dx: float = 1.0
    c: float = 1.0
    a_r: float = 1.0
    source: str = "none"          # none | absorption | coupled_t
    flux_source: str = "wb"       # wb | centered
    closure: str = "m1"           # m1 | p1
    ap: bool = True
    lambda_floor: float = 0.0
    linearization: str = "newton"  # newton (tensor differentiated) | picard (tensor frozen)
    bc: tuple = ("periodic",) * 6
    wb_boundary: bool = False     # Eq. "boundaryCondition" at non-periodic faces (well-balanced source only)
    ghost: dict = field(default_factory=dict)       # face -> (1+ndim, *plane)
    ghost_mask: dict = field(default_factory=dict)  # face -> plane weights

    @property
    def ndim(self):
        return len(self.n)

    @property
    def nrad(self):
        return 1 + self.ndim

    @property
    def nu(self):
        return self.nrad + (1 if self.source == "coupled_t" else 0)

    @property
    def shape(self):
        return tuple(int(v) for v in reversed(self.n))

    def axis(self, d):
        return self.ndim - 1 - d

    @staticmethod
    def from_problem(p):
        return Scheme(n=tuple(p["n"]), dx=p["dx"], c=p["c"], a_r=p["a_r"],
                      source=p["source"], flux_source=p["flux_source"],
                      closure=p.get("closure", "m1"), ap=p["ap"],
                      lambda_floor=p["lambda_floor"], bc=tuple(p["bc"]),
                      linearization=p.get("linearization", "newton"),
                      wb_boundary=bool(p.get("wb_boundary", False)),
                      ghost=dict(p.get("ghost", {})),
                      ghost_mask=dict(p.get("ghost_mask", {})))


def state_from_problem(p, which="U"):
    """Stack the (E, F[, T]) fields of a problem dict into one (n_u, *grid) array."""
    sch = Scheme.from_problem(p)
    if which == "U":
        E, F, T = p["E"], p["F"], p.get("T")
    else:
        E, F, T = p["En"], p["Fn"], p.get("Tn")
    comps = [E] + [F[m] for m in range(sch.ndim)]
    if sch.source == "coupled_t":
        comps.append(T)
    return np.stack([np.asarray(c, dtype=np.float64) for c in comps])


# ---------------------------------------------------------------------------
# Closure and wave speeds
# ---------------------------------------------------------------------------
def closure(E, F, c, kind="m1"):
    """M1 closure (Sect. 2.2).

    Returns (f, nvec, chi, D): the clamped reduced-flux magnitude f <= 1, the
    unit direction n (0 where F = 0), the Eddington factor chi and the Eddington
    tensor D[m][l] (nested lists of arrays).  f > 1 is clamped to 1 with n kept
    unit (Sect. 6); an iterate with E <= 0 uses E = 1e-300 for f.
    With kind="p1" the P1 closure D = I/3 is used (chi = 1/3).
    """
    ndim = len(F)
    Fmag = np.sqrt(sum(F[m] * F[m] for m in range(ndim)))
    Epos = np.maximum(E, E_FLOOR_CLOSURE)
    f = np.minimum(Fmag / (c * Epos), 1.0)
    safe = np.where(Fmag > 0.0, Fmag, 1.0)
    nvec = [np.where(Fmag > 0.0, F[m] / safe, 0.0) for m in range(ndim)]
    if kind == "p1":
        chi = np.full_like(f, 1.0 / 3.0)
    else:
        xi = np.sqrt(4.0 - 3.0 * f * f)
        chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * xi)
    D = [[(0.5 * (1.0 - chi) if m == l else 0.0) + 0.5 * (3.0 * chi - 1.0) * nvec[m] * nvec[l]
          for l in range(ndim)] for m in range(ndim)]
    return f, nvec, chi, D


def wave_speeds(f, nvec, d, c, kind="m1"):
    """Largest and smallest wave speed of the M1 system along direction d.

    Eq. "eigenvalues" with xi = sqrt(4 - 3 f^2), f_x -> the component of the
    reduced flux along d and f_y^2 -> the squared transverse part (in 3D the
    sum of both transverse components).  P1: +-c/sqrt(3).
    """
    if kind == "p1":
        s = c / math.sqrt(3.0)
        return np.full_like(f, s), np.full_like(f, -s)
    fn = f * nvec[d]
    fperp2 = np.maximum(f * f - fn * fn, 0.0)
    xi = np.sqrt(4.0 - 3.0 * f * f)
    q = (xi - 1.0) * (xi + 2.0)
    root = math.sqrt(2.0) * np.sqrt(q * (2.0 * q + 3.0 * fperp2)) / (math.sqrt(3.0) * xi * (xi + 2.0))
    return c * (fn / xi + root), c * (fn / xi - root)


def pressure_jacobian(E, F, c, kind="m1"):
    """Derivative of the radiative pressure P = D(E, F) E with respect to (E, F).

    Returns J[d][m] = [dP_dm/dE, dP_dm/dF_0, ..., dP_dm/dF_{ndim-1}] (arrays).
    From P_dm = E (1-chi)/2 delta_dm + E (3chi-1)/2 n_d n_m (Sect. 2.2):
      dP_dm/dE   = D_dm - f chi'(f) (-delta_dm/2 + 3/2 n_d n_m)
      dP_dm/dF_l = chi'(f)/c n_l (-delta_dm/2 + 3/2 n_d n_m)
                   + (3chi-1)/2 (E/|F|) (delta_dl n_m + delta_ml n_d - 2 n_d n_m n_l)
    with chi'(f) = [8f(5+2xi) + 6f(3+4f^2)/xi] / (5+2xi)^2.  Where f is clamped to 1
    (|F| > cE, or E <= 0) the derivatives of f vanish; F = 0 gives dP/dF = 0.
    P1: P = E I/3, so dP/dE = I/3 and dP/dF = 0.

    The factor (3chi-1)/2 (E/|F|) of the direction term is evaluated without
    cancellation: from chi = (3+4f^2)/(5+2xi) and xi^2 = 4 - 3f^2 one gets
    3chi - 1 = 6f^2/(2+xi) exactly, so (3chi-1)/2 (E/|F|) = 3f/(c(2+xi)) where f
    is not clamped (bounded as F -> 0, where the literal product is rounding
    noise times an unbounded E/|F|); where f is clamped, chi = 1 and the factor
    is E/|F| <= 1/c.
    """
    ndim = len(F)
    f, nvec, chi, D = closure(E, F, c, kind)
    Fmag = np.sqrt(sum(F[m] * F[m] for m in range(ndim)))
    zero = np.zeros_like(f)
    if kind == "p1":
        return [[[D[d][m]] + [zero] * ndim for m in range(ndim)] for d in range(ndim)]
    xi = np.sqrt(4.0 - 3.0 * f * f)
    dchi = (8.0 * f * (5.0 + 2.0 * xi) + 6.0 * f * (3.0 + 4.0 * f * f) / xi) / (5.0 + 2.0 * xi) ** 2
    Epos = np.maximum(E, E_FLOOR_CLOSURE)
    clamped = Fmag >= c * Epos
    dchi = np.where(clamped, 0.0, dchi)
    E_over_F = np.where(Fmag > 0.0, E / np.where(Fmag > 0.0, Fmag, 1.0), 0.0)
    geo_factor = np.where(clamped, E_over_F, 3.0 * f / (c * (2.0 + xi)))
    J = []
    for d in range(ndim):
        row = []
        for m in range(ndim):
            shape_dm = (-0.5 if d == m else 0.0) + 1.5 * nvec[d] * nvec[m]
            dE = D[d][m] - f * dchi * shape_dm
            dF = []
            for l in range(ndim):
                t1 = dchi / c * nvec[l] * shape_dm
                geo = ((nvec[m] if d == l else 0.0) + (nvec[d] if m == l else 0.0)
                       - 2.0 * nvec[d] * nvec[m] * nvec[l])
                t2 = geo_factor * geo
                dF.append(t1 + t2)
            row.append([dE] + dF)
        J.append(row)
    return J


def hll_coefficients(lmax_L, lmin_L, lmax_R, lmin_R, c, lambda_floor=0.0):
    """HLL weights of a face from the speeds on its two sides.

    lambda+ = max(0, lmax_L, lmax_R) and lambda- = min(0, lmin_L, lmin_R)
    (Sect. 3.1.1, two-sided reading), optionally floored to +-floor*c as in the
    shadow test (Sect. 5.4).  Returns a = l+/(l+ - l-), b = 1 - a and
    dd = l+ l- / (l+ - l-); a degenerate face (l+ - l- <= 1e-14 c, both speeds
    zero) takes a = b = 1/2, dd = 0.
    """
    lp = np.maximum(0.0, np.maximum(lmax_L, lmax_R))
    lm = np.minimum(0.0, np.minimum(lmin_L, lmin_R))
    if lambda_floor > 0.0:
        lp = np.maximum(lp, lambda_floor * c)
        lm = np.minimum(lm, -lambda_floor * c)
    den = lp - lm
    deg = den <= DEGENERATE_REL * c
    safe = np.where(deg, 1.0, den)
    a = np.where(deg, 0.5, lp / safe)
    dd = np.where(deg, 0.0, lp * lm / safe)
    return a, 1.0 - a, dd


def ap_alpha(sigma_face, dx, fbar, dd, c):
    """Asymptotic correction of the energy flux (Eq. "asymptoticCorrection").

    alpha = 1 / (1 - 3 sigma_{i+1/2} dx (1 - fbar^2) dd / c), dd = l+ l- /(l+ - l-)
    and fbar the mean of |f^n| over the two cells.
    """
    return 1.0 / (1.0 - 3.0 * sigma_face * dx * (1.0 - fbar * fbar) * dd / c)


# ---------------------------------------------------------------------------
# Ghost cells (one layer) -- boundary reading: periodic wrap, outflow copy,
# reflect (normal flux negated), Dirichlet (given plane, optional mask that
# blends it with the outflow copy).
# ---------------------------------------------------------------------------
def _take(a, ax, idx):
    """The slab a[..., idx, ...] along axis ax, keeping the axis (extent 1)."""
    return np.take(a, [idx], axis=ax)


def ghost_layer(sch, X, d, side, mode):
    """Ghost layer of a component-major field X (n, *grid) on one side of direction d.

    mode 'state': the boundary values of a state (Dirichlet planes inserted);
    mode 'linear': the same map applied to a perturbation (Dirichlet -> 0 on the
    masked part).  Returns an array with extent 1 along the direction's axis.
    """
    ax = sch.axis(d) + 1
    face = 2 * d + side
    bc = sch.bc[face]
    N = X.shape[ax]
    if bc == "periodic":
        return _take(X, ax, N - 1 if side == 0 else 0).copy()
    inner = _take(X, ax, 0 if side == 0 else N - 1).copy()
    if bc == "outflow":
        return inner
    if bc == "reflect":
        inner[1 + d] *= -1.0
        return inner
    if bc == "dirichlet":
        w = sch.ghost_mask.get(face)
        w = np.ones(inner.shape[1:]) if w is None else np.expand_dims(np.asarray(w, float), sch.axis(d))
        out = inner * (1.0 - w)[None]
        if mode == "state":
            plane = np.expand_dims(np.asarray(sch.ghost[face], float), ax)
            out[: sch.nrad] += w[None] * plane
        return out
    raise ValueError(f"unknown boundary {bc}")


def padded(sch, X, d, mode):
    """X with one ghost layer on each side along direction d."""
    ax = sch.axis(d) + 1
    return np.concatenate([ghost_layer(sch, X, d, 0, mode), X,
                           ghost_layer(sch, X, d, 1, mode)], axis=ax)


def padded_scalar(sch, s, d):
    """A per-cell coefficient (sigma) extended to the ghosts: wrap if periodic, else copy."""
    ax = sch.axis(d)
    N = s.shape[ax]
    lo_bc, hi_bc = sch.bc[2 * d], sch.bc[2 * d + 1]
    lo = _take(s, ax, N - 1 if lo_bc == "periodic" else 0)
    hi = _take(s, ax, 0 if hi_bc == "periodic" else N - 1)
    return np.concatenate([lo, s, hi], axis=ax)


def _slice(a, ax, start, stop):
    sl = [slice(None)] * a.ndim
    sl[ax] = slice(start, stop)
    return a[tuple(sl)]


# ---------------------------------------------------------------------------
# Linearisation: every coefficient that is frozen during one Newton iterate
# ---------------------------------------------------------------------------
@dataclass
class Linearization:
    sch: Scheme
    dt: float
    Ulin: np.ndarray
    Un: np.ndarray
    sigma: np.ndarray
    rho_cv: np.ndarray | None
    faces: list            # per direction: dict(a, b, dd, alpha, sigf) over N+1 faces
    Dpad: list             # per direction: c^2 D[d][m] on the padded grid along d
    Jpad: list             # per direction: c^2 dP_dm/d(E, F_l) on the padded grid along d
    kappa: np.ndarray | None   # 4 a_r T_k^3 (coupled mode)


def reduced_flux_magnitude(sch, U):
    """|f| = min(1, |F|/(cE)) per cell (the quantity alpha averages)."""
    f, _, _, _ = closure(U[0], [U[1 + m] for m in range(sch.ndim)], sch.c, sch.closure)
    return f


def linearize(sch, sigma, rho_cv, Ulin, Un, dt):
    """Freeze the closure, the HLL weights and alpha at the iterate Ulin.

    The speeds and Eddington tensor use the iterate (they are the scheme's
    nonlinearities, Sect. 3.3.1); alpha's reduced flux uses time n (Sect. 3.1.3).
    """
    ndim, c = sch.ndim, sch.c
    faces, Dpad, Jpad = [], [], []
    for d in range(ndim):
        ax = sch.axis(d)
        P = padded(sch, Ulin, d, "state")
        Pn = padded(sch, Un, d, "state")
        f, nv, chi, D = closure(P[0], [P[1 + m] for m in range(ndim)], c, sch.closure)
        fn_abs = reduced_flux_magnitude(sch, Pn)
        lmax, lmin = wave_speeds(f, nv, d, c, sch.closure)
        N = Ulin.shape[ax + 1]
        L = lambda a: _slice(a, ax, 0, N + 1)
        R = lambda a: _slice(a, ax, 1, N + 2)
        a, b, dd = hll_coefficients(L(lmax), L(lmin), R(lmax), R(lmin), c, sch.lambda_floor)
        sp = padded_scalar(sch, sigma, d)
        sigf = 0.5 * (L(sp) + R(sp))
        if sch.ap:
            alpha = ap_alpha(sigf, sch.dx, 0.5 * (L(fn_abs) + R(fn_abs)), dd, c)
        else:
            alpha = np.ones_like(a)
        faces.append(dict(a=a, b=b, dd=dd, alpha=alpha, sigf=sigf))
        Dpad.append([[c * c * np.broadcast_to(D[m][l], f.shape) for l in range(ndim)]
                     for m in range(ndim)])
        Jd = pressure_jacobian(P[0], [P[1 + m] for m in range(ndim)], c, sch.closure)
        Jpad.append([[c * c * np.broadcast_to(v, f.shape) for v in Jd[d][m]] for m in range(ndim)])
    kappa = None
    if sch.source == "coupled_t":
        kappa = 4.0 * sch.a_r * Ulin[sch.nrad] ** 3
    return Linearization(sch, float(dt), Ulin, Un, sigma, rho_cv, faces, Dpad, Jpad, kappa)


# ---------------------------------------------------------------------------
# The discrete operator.  One routine evaluates
#   mode 'residual' : R(X) with the frozen coefficients, X a state (ghost = BC values)
#   mode 'linear'   : A X, the derivative with the coefficients frozen
#   mode 'diag'     : A X keeping only couplings of a cell with itself (the
#                     diagonal blocks; neighbours contribute only through a
#                     ghost derived from the same cell or a one-cell period)
# ---------------------------------------------------------------------------
def _neighbour_mask(sch, d, N, side):
    """1 where the neighbour on `side` of a cell is the cell itself or its own ghost."""
    m = np.zeros(N)
    bc = sch.bc[2 * d + side]
    if bc == "periodic":
        if N == 1:
            m[:] = 1.0
    else:
        m[0 if side == 0 else N - 1] = 1.0
    return m


def operator(lin, X, mode):
    sch, dt = lin.sch, lin.dt
    ndim, c, nrad = sch.ndim, sch.c, sch.nrad
    s = dt / sch.dx
    Y = np.zeros_like(X)
    gmode = "state" if mode == "residual" else "linear"
    # time derivative
    if mode == "residual":
        Y[:nrad] = X[:nrad] - lin.Un[:nrad]
    else:
        Y[:nrad] = X[:nrad]
    for d in range(ndim):
        ax = sch.axis(d)
        N = X.shape[ax + 1]
        P = padded(sch, X, d, gmode)
        Xl = _slice(P, ax + 1, 0, N)        # left neighbour (or ghost)
        Xr = _slice(P, ax + 1, 2, N + 2)    # right neighbour (or ghost)
        if mode == "diag":
            shp = [1] * X.ndim
            shp[ax + 1] = N
            Xl = Xl * _neighbour_mask(sch, d, N, 0).reshape(shp)
            Xr = Xr * _neighbour_mask(sch, d, N, 1).reshape(shp)
        fc = lin.faces[d]
        plus = {k: _slice(v, ax, 1, N + 1) for k, v in fc.items()}
        minus = {k: _slice(v, ax, 0, N) for k, v in fc.items()}
        # c^2 P_dm of each cell: the pressure itself (residual, tensor from the
        # evaluated state) or its linearisation (Newton: dP/dU . X; Picard: D X_E)
        if mode == "residual":
            _, _, _, Dst = closure(P[0], [P[1 + m] for m in range(ndim)], c, sch.closure)
            qpad = [c * c * Dst[d][m] * P[0] for m in range(ndim)]
            q_self = [_slice(q, ax, 1, N + 1) for q in qpad]
            q_left = [_slice(q, ax, 0, N) for q in qpad]
            q_right = [_slice(q, ax, 2, N + 2) for q in qpad]
        else:
            def lin_pressure(Xs, lo, hi):
                if sch.linearization == "newton":
                    Jp = lin.Jpad[d]
                    return [sum(_slice(Jp[m][k], ax, lo, hi) * Xs[k] for k in range(1 + ndim))
                            for m in range(ndim)]
                return [_slice(lin.Dpad[d][d][m], ax, lo, hi) * Xs[0] for m in range(ndim)]
            q_self = lin_pressure(X, 1, N + 1)
            q_left = lin_pressure(Xl, 0, N)
            q_right = lin_pressure(Xr, 2, N + 2)

        def flux_E(f, L, R):
            return f["alpha"] * (f["a"] * L[1 + d] + f["b"] * R[1 + d] + f["dd"] * (R[0] - L[0]))

        def flux_F(f, L, R, qL, qR, m):
            return f["a"] * qL[m] + f["b"] * qR[m] + f["dd"] * (R[1 + m] - L[1 + m])

        Y[0] += s * (flux_E(plus, X, Xr) - flux_E(minus, Xl, X))
        for m in range(ndim):
            Y[1 + m] += s * (flux_F(plus, X, Xr, q_self, q_right, m) - flux_F(minus, Xl, X, q_left, q_self, m))
        if sch.flux_source == "wb":
            # {sigma F_d}_i = 1/2 (sigma_{i+1/2} F_{i+1/2} + sigma_{i-1/2} F_{i-1/2}),
            # F_{i+1/2} = (F_i + F_{i+1}) / 2, faces normal to d (Eq. "wb_smart");
            # below, hi and lo are twice the face values sigma F of the two faces
            hi = plus["sigf"] * (X[1 + d] + Xr[1 + d])
            lo = minus["sigf"] * (Xl[1 + d] + X[1 + d])
            if sch.wb_boundary:
                # Eq. "boundaryCondition": on a face between a cell and a ghost, sigma F is
                # -c (P_dd(inside) - P_dd(outside)) / dx with the pressure of the ghost state
                # (q = c^2 P, so sigma F = -(q_R - q_L) / (c dx))
                shp = [1] * (X.ndim - 1)
                shp[ax] = N
                at_lo = np.zeros(N, bool)
                at_hi = np.zeros(N, bool)
                at_lo[0] = sch.bc[2 * d] != "periodic"
                at_hi[N - 1] = sch.bc[2 * d + 1] != "periodic"
                lo = np.where(at_lo.reshape(shp), -2.0 * (q_self[d] - q_left[d]) / (c * sch.dx), lo)
                hi = np.where(at_hi.reshape(shp), -2.0 * (q_right[d] - q_self[d]) / (c * sch.dx), hi)
            Y[1 + d] += c * dt * 0.25 * (hi + lo)
    sig = lin.sigma
    if sch.flux_source == "centered":
        for m in range(ndim):
            Y[1 + m] += c * dt * sig * X[1 + m]          # Eq. "wb_naive"
    if sch.source == "absorption":
        Y[0] += c * sig * dt * X[0]
    elif sch.source == "coupled_t":
        T = X[nrad]
        if mode == "residual":
            exch = c * sig * dt * (sch.a_r * T ** 4 - X[0])
            Y[0] -= exch
            Y[nrad] = lin.rho_cv * (T - lin.Un[nrad]) + exch
        else:
            exch = c * sig * dt * (lin.kappa * T - X[0])
            Y[0] -= exch
            Y[nrad] = lin.rho_cv * T + exch
    return Y


def residual(lin, U=None):
    """R(U) of the backward-Euler scheme, coefficients frozen at lin (default U = Ulin)."""
    return operator(lin, lin.Ulin if U is None else U, "residual")


def apply_operator(lin, x):
    """y = A x with A the linearised operator at lin; x, y flat (n_u*N,) or (n_u, *grid)."""
    shp = (lin.sch.nu,) + lin.sch.shape
    return operator(lin, np.asarray(x, float).reshape(shp), "linear").reshape(np.shape(x))


def diagonal_blocks(lin):
    """The exact diagonal n_u x n_u block of A at every cell, shape (N, n_u, n_u)."""
    nu = lin.sch.nu
    shp = (nu,) + lin.sch.shape
    cols = []
    for k in range(nu):
        e = np.zeros(shp)
        e[k] = 1.0
        cols.append(operator(lin, e, "diag").reshape(nu, -1))
    B = np.stack(cols, axis=-1)           # (nu, N, nu): row comp, cell, column comp
    return np.transpose(B, (1, 0, 2))


class BlockJacobi:
    """z = M^{-1} r with M the block diagonal of A (one dense solve per cell).

    shift (optional, shape (n_u, N)) is added to the diagonal of every block:
    the block diagonal of A + diag(shift), used by pseudo-transient continuation."""

    def __init__(self, lin, shift=None):
        self.nu = lin.sch.nu
        self.blocks = diagonal_blocks(lin)
        if shift is not None:
            idx = np.arange(self.nu)
            self.blocks[:, idx, idx] += np.asarray(shift, float).reshape(self.nu, -1).T
        self.inv = np.linalg.inv(self.blocks)

    def __call__(self, r):
        R = np.asarray(r, float).reshape(self.nu, -1).T          # (N, nu)
        Z = np.einsum("nij,nj->ni", self.inv, R)
        return Z.T.reshape(np.shape(r))


def assemble_dense(lin):
    """A as a dense matrix, column k = A e_k (small grids only)."""
    n = lin.sch.nu * int(np.prod(lin.sch.shape))
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = apply_operator(lin, e)
    return A


# ---------------------------------------------------------------------------
# Restarted right-preconditioned GMRES with modified Gram-Schmidt
# ---------------------------------------------------------------------------
@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    restarts: int
    rel_residual: float
    converged: bool


def gmres(apply, precond, b, restart=30, rtol=1e-10, max_iters=10000, fixed_iters=0):
    """Solve A x = b with x0 = 0, right preconditioning A M^{-1} y = b, x = M^{-1} y.

    Convergence is judged on the true residual ||b - A x|| / ||b|| at every
    restart and at exit; inside a cycle the least-squares residual decides when
    to end the cycle.  fixed_iters > 0 runs exactly that many iterations
    (restarting every `restart`) with no early exit.
    """
    b = np.asarray(b, float)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return GmresResult(x, 0, 0, 0.0, True)
    budget = fixed_iters if fixed_iters > 0 else max_iters
    total, cycles = 0, 0
    r = b.copy()
    beta = bnorm
    while True:
        if fixed_iters <= 0 and beta <= rtol * bnorm:
            return GmresResult(x, total, max(cycles - 1, 0), beta / bnorm, True)
        if total >= budget:
            return GmresResult(x, total, max(cycles - 1, 0), beta / bnorm,
                               fixed_iters > 0 or beta <= rtol * bnorm)
        cycles += 1
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        k = 0
        for j in range(restart):
            w = apply(precond(V[j]))
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            k = j + 1
            total += 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)
            est = float(np.linalg.norm(e1 - H[: k + 1, :k] @ y))
            breakdown = H[j + 1, j] <= 1e-14 * beta
            if breakdown or total >= budget or (fixed_iters <= 0 and est <= rtol * bnorm):
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)
        x = x + precond(sum(y[i] * V[i] for i in range(k)))
        r = b - apply(x)
        beta = float(np.linalg.norm(r))


# ---------------------------------------------------------------------------
# One implicit step
# ---------------------------------------------------------------------------
@dataclass
class StepResult:
    U: np.ndarray
    converged: bool
    newton_iters: int
    krylov_iters: int
    restarts: int
    nonlinear_rel: float
    cells_f_gt_1: int
    history: list


def mass_diagonal(sch, rho_cv):
    """Coefficient of U^{n+1} in each row of the backward-Euler residual: 1 on
    the E and F rows, rho c_v on the T row; shape (n_u, N)."""
    N = int(np.prod(sch.shape))
    m = np.ones((sch.nu, N))
    if sch.source == "coupled_t":
        m[sch.nrad] = np.asarray(rho_cv, float).reshape(-1)
    return m


def implicit_step(sch, sigma, rho_cv, Un, dt, *, restart=30, rtol=1e-10, max_iters=20000,
                  newton_max=20, newton_rtol=None, fixed_iters=0, pc="bj",
                  psi0=0.0, ptc_rtol=0.0, line_search=False, clip=0.0, forcing=0.0, mg_opts=None):
    """Advance Un by one backward-Euler step (Sect. 3.1, Sect. 3.3.1).

    Newton loop: linearise at U^k, b = -R(U^k); stop when
    ||R(U^k)|| <= newton_rtol ||R(U^0)||; else solve A^k delta = b by GMRES and
    set U^{k+1} = U^k + delta.  With fixed_iters > 0 exactly newton_max linear
    solves of exactly fixed_iters GMRES iterations are made (no early exit).

    pc: "bj" (block-Jacobi), "mg" (the aggregation multigrid V-cycle of
    m1_multigrid, options mg_opts) or "none".

    Four optional additions change the path to the root, never the root
    itself (the residual R is untouched).  They are solver additions; the
    paper's Newton iteration has none of them:

    * psi0 > 0: pseudo-transient continuation (Kelley and Keyes, SIAM J. Numer.
      Anal. 35, 1998).  Iteration k solves (A^k + psi_k M) delta = -R(U^k),
      M = mass_diagonal (the coefficient of U^{n+1} in each row); block-Jacobi
      takes the shifted diagonal blocks.  psi follows switched evolution
      relaxation (Mulder and van Leer, 1985): psi_{k+1} = psi_k ||R_{k+1}||/||R_k||
      when the residual fell, 2 psi_k when it did not, and 0 once below
      1e-6 psi0.  While psi > 0 and ptc_rtol > 0 the linear tolerance is
      max(rtol, min(ptc_rtol, psi/psi0)): loose while far from the root,
      tightening with the residual.
    * forcing > 0: inexact Newton; iteration k solves to max(rtol, min(0.1,
      forcing ||R_k||/||R_0||)) (with PTC the looser of the two tolerances).
    * clip in (0, 1): before the update, dE (and dT with the T row) is raised to
      at least -clip E (-clip T) per cell: the energy and temperature of a cell
      drop by at most that fraction in one update.
    * line_search (not with fixed_iters): U^{k+1} = U^k + lam delta with the
      first lam in 1, 1/2, ..., 1/128 whose residual satisfies
      ||R|| <= (1 - 1e-4 lam) ||R(U^k)|| (Armijo test).  If none does: with
      psi0 > 0 the step is rejected (U^{k+1} = U^k) and psi becomes
      max(10 psi, 1e-3 psi0); without, the trial with the smallest ||R|| is
      taken (the earliest on ties).
    """
    if newton_rtol is None:
        newton_rtol = rtol
    U = np.array(Un, dtype=float, copy=True)
    mass = mass_diagonal(sch, rho_cv)
    psi = float(psi0)
    r0 = None
    kry = rst = 0
    hist = []
    rel = 1.0
    converged = False
    it = 0
    lin = linearize(sch, sigma, rho_cv, U, Un, dt)
    R = residual(lin)
    rn = float(np.linalg.norm(R))
    while True:
        if r0 is None:
            r0 = rn
        rel = rn / r0 if r0 > 0 else 0.0
        hist.append(rn)
        if fixed_iters > 0:
            if it >= newton_max:
                converged = True
                break
        elif rn == 0.0 or (it > 0 and rel <= newton_rtol):
            converged = True
            break
        elif it >= newton_max:
            break
        if not np.isfinite(rn):
            break
        shift = psi * mass if psi > 0 else None
        if pc == "bj":
            M = BlockJacobi(lin, shift)
        elif pc == "mg":
            from .m1_multigrid import Multigrid
            M = Multigrid(lin, shift=shift, **(mg_opts or {}))
        else:
            M = lambda v: v
        if shift is None:
            op = lambda v: apply_operator(lin, v)
        else:
            op = lambda v, sh=shift.reshape(-1): apply_operator(lin, v) + sh * v
        lin_tol = rtol
        if forcing > 0:
            lin_tol = max(lin_tol, min(0.1, forcing * rel))
        if psi > 0 and ptc_rtol > 0:
            lin_tol = max(lin_tol, min(ptc_rtol, psi / psi0))
        res = gmres(op, M, -R.reshape(-1), restart=restart, rtol=lin_tol, max_iters=max_iters,
                    fixed_iters=fixed_iters)
        kry += res.iters
        rst += res.restarts
        delta = res.x.reshape(U.shape)
        if clip > 0:
            delta = delta.copy()
            delta[0] = np.maximum(delta[0], -clip * U[0])
            if sch.source == "coupled_t":
                delta[sch.nrad] = np.maximum(delta[sch.nrad], -clip * U[sch.nrad])
        rejected = False
        if line_search and fixed_iters == 0:
            ref = rn
            lam, best, passed = 1.0, None, False
            for _ in range(8):
                lin_t = linearize(sch, sigma, rho_cv, U + lam * delta, Un, dt)
                R_t = residual(lin_t)
                r_t = float(np.linalg.norm(R_t))
                if best is None or (np.isfinite(r_t) and not r_t >= best[0]):
                    best = (r_t, lam, lin_t, R_t)
                if np.isfinite(r_t) and r_t <= (1.0 - 1e-4 * lam) * ref:
                    best = (r_t, lam, lin_t, R_t)
                    passed = True
                    break
                lam *= 0.5
            if passed or psi0 <= 0:
                r_new, lam, lin, R = best
                U = U + lam * delta
            else:
                rejected = True          # keep U^k, lin and R; raise the shift
                r_new = rn
        else:
            U = U + delta
            lin = linearize(sch, sigma, rho_cv, U, Un, dt)
            R = residual(lin)
            r_new = float(np.linalg.norm(R))
        if rejected:
            psi = max(10.0 * psi, 1e-3 * psi0)
        elif psi > 0:
            psi = psi * r_new / rn if r_new < rn else 2.0 * psi
            if psi < 1e-6 * psi0:
                psi = 0.0
        rn = r_new
        it += 1
    Fmag = np.sqrt(sum(U[1 + m] ** 2 for m in range(sch.ndim)))
    nf = int(np.count_nonzero(Fmag > F_GT_1_REL * sch.c * U[0]))
    return StepResult(U, converged, it, kry, rst, rel, nf, hist)


def explicit_step(sch, sigma, rho_cv, Un, dt):
    """Forward-Euler step of the same spatial operator (coefficients at time n)."""
    lin = linearize(sch, sigma, rho_cv, Un, Un, dt)
    R = residual(lin)              # = dt * (divergence + sources) evaluated at U^n
    U = Un - R
    if sch.source == "coupled_t":
        U[sch.nrad] = Un[sch.nrad] - R[sch.nrad] / rho_cv
    return U


def source_terms(sch, sigma, rho_cv, U, dt):
    """The source part of the residual at state U, row by row (the terms the
    semi-implicit step treats implicitly): c dt sigma F_m on the flux rows
    (centred form, Eq. "wb_naive"); c dt sigma E on the energy row with
    absorption; with the T row, -c dt sigma (a_r T^4 - E) on the energy row and
    +c dt sigma (a_r T^4 - E) on the T row."""
    if sch.flux_source != "centered":
        raise ValueError("the source part is separable per cell only for the centred flux source")
    S = np.zeros_like(U)
    c, nrad = sch.c, sch.nrad
    for m in range(sch.ndim):
        S[1 + m] = c * dt * sigma * U[1 + m]
    if sch.source == "absorption":
        S[0] = c * dt * sigma * U[0]
    elif sch.source == "coupled_t":
        exch = c * dt * sigma * (sch.a_r * U[nrad] ** 4 - U[0])
        S[0] = -exch
        S[nrad] = exch
    return S


def semi_implicit_step(sch, sigma, rho_cv, Un, dt, t_newton=60):
    """Semi-implicit step (Sect. 3.1: sources implicit, hyperbolic part explicit).

    H = R(U^n) - S(U^n) is the flux divergence of the scheme at time n (closure,
    speeds and alpha from U^n); the new state solves, cell by cell,
        U - U^n + H + S(U) = 0,
    i.e. F_m = (F_m^n - H_Fm)/(1 + c dt sigma); with absorption
    E = (E^n - H_E)/(1 + c dt sigma), without a source E = E^n - H_E; with the T
    row, E = (E* + k a_r T^4)/(1 + k) (k = c dt sigma, E* = E^n - H_E) and T the
    root of rho c_v (T - T^n) + k (a_r T^4 - E) = 0, found by Newton from T^n
    (t_newton iterations, stopping once the update is below 1e-15 T).  Only the
    centred flux source (Eq. "wb_naive") keeps the sources local to a cell.
    """
    lin = linearize(sch, sigma, rho_cv, Un, Un, dt)
    H = residual(lin) - source_terms(sch, sigma, rho_cv, Un, dt)
    c, nrad, k = sch.c, sch.nrad, sch.c * dt * sigma
    U = np.array(Un, dtype=float, copy=True)
    for m in range(sch.ndim):
        U[1 + m] = (Un[1 + m] - H[1 + m]) / (1.0 + k)
    if sch.source == "absorption":
        U[0] = (Un[0] - H[0]) / (1.0 + k)
    elif sch.source == "coupled_t":
        Es = Un[0] - H[0]
        rc = np.asarray(rho_cv, float)
        T = np.array(Un[nrad], dtype=float, copy=True)
        # eliminate E: g(T) = rc (T - T^n) + k (a_r T^4 - (Es + k a_r T^4)/(1 + k))
        #                  = rc (T - T^n) + k/(1+k) (a_r T^4 - Es)
        w = k / (1.0 + k)
        for _ in range(t_newton):
            g = rc * (T - Un[nrad]) + w * (sch.a_r * T ** 4 - Es)
            dg = rc + 4.0 * w * sch.a_r * T ** 3
            dT = g / dg
            T = T - dT
            if np.all(np.abs(dT) <= 1e-15 * np.abs(T)):
                break
        U[nrad] = T
        U[0] = (Es + k * sch.a_r * T ** 4) / (1.0 + k)
    else:
        U[0] = Un[0] - H[0]
    return U


def discrete_diffusion_step(sigma, E, dt, c=1.0, dx=1.0):
    """Backward-Euler step of the discrete diffusion limit (Eq. "discreteDiffusionEqua").

    E^{n+1} - E^n = c dt/(3 dx^2) sum_d [ (E_{i+1}-E_i)/sigma_{i+1/2} - (E_i-E_{i-1})/sigma_{i-1/2} ]
    on a periodic grid (E at n+1 on the right), sigma_{i+1/2} the arithmetic face
    mean of the two cells; solved with a sparse direct solver.
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    shape = E.shape
    N = E.size
    idx = np.arange(N).reshape(shape)
    k = c * dt / (3.0 * dx * dx)
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [np.ones(N)]
    for ax in range(E.ndim):
        nb = np.roll(idx, -1, axis=ax).ravel()
        w = (k / (0.5 * (sigma + np.roll(sigma, -1, axis=ax)))).ravel()
        i = idx.ravel()
        rows += [i, nb, i, nb]
        cols += [i, nb, nb, i]
        vals += [w, w, -w, -w]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return spla.spsolve(A.tocsc(), E.ravel()).reshape(shape)


def equilibrium_diffusion_step(T, Tn, dt, sigma, rho_cv, c=1.0, a_r=1.0, dx=1.0, left=None, right="outflow",
                               newton_max=60):
    """Backward-Euler step of the equilibrium diffusion limit (Eq. "diffusionEqua") on a 1D row.

    The total energy E + rho c_v T with E = a_r T^4 obeys
        (E_i + rho_cv_i T_i) - (E_i^n + rho_cv_i T_i^n)
            = dt/dx^2 [k_{i+1/2} (E_{i+1} - E_i) - k_{i-1/2} (E_i - E_{i-1})],
    k = c / (3 sigma_face) with sigma_face the arithmetic mean of the two cells
    (the face opacity of the scheme's asymptotic correction).  Boundaries: `left`
    a temperature held in a ghost cell one cell beyond the first (with the first
    cell's sigma), or None for no flux; `right` "outflow" (no diffusive flux);
    left = "periodic" wraps both ends.  T is the Newton starting guess (usually
    T^n); Newton on T with the tridiagonal Jacobian, stopping once |dT| <= 1e-14 T.
    """
    from scipy.linalg import solve_banded

    T = np.array(T, dtype=float, copy=True)
    Tn = np.asarray(Tn, float)
    sig = np.asarray(sigma, float)
    rc = np.broadcast_to(np.asarray(rho_cv, float), T.shape)
    n = T.size
    periodic = isinstance(left, str) and left == "periodic"
    if periodic:
        kr = c / (3.0 * 0.5 * (sig + np.roll(sig, -1)))          # face i+1/2, i = 0..n-1 (wraps)
    else:
        kr = np.zeros(n)
        kr[:-1] = c / (3.0 * 0.5 * (sig[:-1] + sig[1:]))         # right face closed: outflow, no flux
    kl = np.roll(kr, 1)
    if not periodic:
        kl[0] = c / (3.0 * sig[0]) if left is not None else 0.0
    lam = dt / (dx * dx)
    total_n = a_r * Tn ** 4 + rc * Tn
    Eg = a_r * float(left) ** 4 if (left is not None and not periodic) else 0.0
    for _ in range(newton_max):
        E = a_r * T ** 4
        dE = 4.0 * a_r * T ** 3
        Er = np.roll(E, -1)
        El = np.roll(E, 1)
        if not periodic:
            Er[-1] = E[-1]
            El[0] = Eg
        g = E + rc * T - total_n - lam * (kr * (Er - E) - kl * (E - El))
        diag = dE + rc + lam * (kr + kl) * dE
        up = -lam * kr * np.roll(dE, -1)      # d g_i / d T_{i+1}
        lo = -lam * kl * np.roll(dE, 1)       # d g_i / d T_{i-1}
        if periodic:
            J = np.diag(diag) + np.diag(up[:-1], 1) + np.diag(lo[1:], -1)
            J[-1, 0] += up[-1]
            J[0, -1] += lo[0]
            d = np.linalg.solve(J, g)
        else:
            ab = np.zeros((3, n))
            ab[0, 1:] = up[:-1]
            ab[1] = diag
            ab[2, :-1] = lo[1:]
            d = solve_banded((1, 1), ab, g)
        T = T - d
        if np.all(np.abs(d) <= 1e-14 * np.abs(T)):
            break
    return T


def velocity_sources(sch, sigma, U, u):
    """The velocity-dependent source terms (Sect. 2.3), per cell, with P = D(E, F) E:
        S_E(u) = sigma/c [u.F + E u.u + u.(u.P)]
        S_F(u) = sigma u.P + sigma a_r T^4 u + sigma/c^2 u (u.F)
    T is the gas-temperature row when the state has one; without it there is no
    emission term (a_r T^4 -> 0).  u: (ndim, *grid).  Returns (S_E, S_F)."""
    c, nd = sch.c, sch.ndim
    E = U[0]
    F = U[1:1 + nd]
    D = closure(E, F, c, sch.closure)[3]
    u = np.asarray(u, float)
    uP = [E * sum(u[l] * D[l][m] for l in range(nd)) for m in range(nd)]   # (u.P)_m
    uF = sum(u[m] * F[m] for m in range(nd))
    uu = sum(u[m] * u[m] for m in range(nd))
    uuP = sum(u[m] * uP[m] for m in range(nd))
    SE = sigma / c * (uF + E * uu + uuP)
    emis = sch.a_r * U[sch.nrad] ** 4 if sch.source == "coupled_t" else 0.0
    SF = np.stack([sigma * uP[m] + sigma * emis * u[m] + sigma / c ** 2 * u[m] * uF for m in range(nd)])
    return SE, SF


def velocity_source_step(sch, sigma, U, u, dt):
    """Step 3 of the splitting (Sect. 3.2): the velocity-dependent sources added
    explicitly to the radiation, E += dt S_E(u), F += dt c S_F(u); the gas rows are
    left to the hydrodynamics."""
    SE, SF = velocity_sources(sch, sigma, U, u)
    V = np.array(U, dtype=float, copy=True)
    V[0] = U[0] + dt * SE
    V[1:1 + sch.ndim] = U[1:1 + sch.ndim] + dt * sch.c * SF
    return V
