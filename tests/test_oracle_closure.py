"""Pins of the oracle's pointwise formulas against facts fixed independently of it.

closure (Sect. 2.2), wave speeds (Eq. "eigenvalues", checked against a brute
force eigen-decomposition of the flux Jacobian), the asymptotic correction
(Eq. "asymptoticCorrection" and its P1 form, Appendix C), the AP flux identity
(Appendix C with the WB face relation of Sect. 3.1.2) and the von Neumann bound
of the WB source (Appendix B).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import m1_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _rand_states(rng, n, ndim, fmax=1.0):
    E = rng.uniform(0.1, 3.0, n)
    f = rng.uniform(0, fmax, n)
    v = rng.standard_normal((ndim, n))
    v /= np.linalg.norm(v, axis=0)
    return E, E[None] * f[None] * v


def test_chi_limits_and_tensor():
    g = golden()
    E = np.array([1.0, 1.0, 2.0])
    F = [np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 2.0]), np.array([0.0, 0.0, 0.0])]
    f, n, chi, D = O.closure(E, F, 1.0)
    assert chi[0] == pytest.approx(g["chi_f0"]["value"], abs=1e-15)      # P1 limit 1/3
    assert chi[1] == pytest.approx(g["chi_f1"]["value"], abs=1e-15)      # free streaming
    assert chi[2] == pytest.approx(1.0, abs=1e-15)
    # f = 0: D = I/3 (P1 limit)
    for m in range(3):
        for l in range(3):
            assert D[m][l][0] == pytest.approx(1 / 3 if m == l else 0.0, abs=1e-16)
    # f = 1 along x: D = n n
    assert D[0][0][1] == pytest.approx(1.0)
    assert D[1][1][1] == pytest.approx(0.0, abs=1e-16)


def test_eddington_tensor_spectrum_3d():
    rng = np.random.default_rng(5)
    E, F = _rand_states(rng, 200, 3)
    f, n, chi, D = O.closure(E, list(F), 1.0)
    for k in range(200):
        M = np.array([[D[m][l][k] for l in range(3)] for m in range(3)])
        assert np.trace(M) == pytest.approx(1.0, abs=1e-14)
        ev = np.sort(np.linalg.eigvalsh(M))
        want = np.sort([(1 - chi[k]) / 2, (1 - chi[k]) / 2, chi[k]])
        assert np.allclose(ev, want, atol=1e-14)
        assert ev[0] >= -1e-15                        # D is positive semidefinite
        assert 1 / 3 - 1e-15 <= chi[k] <= 1 + 1e-15   # realisability of the closure


def test_clamp_f_above_one():
    E = np.array([1.0])
    F = [np.array([3.0]), np.array([4.0])]          # |F| = 5 > cE
    f, n, chi, D = O.closure(E, F, 1.0)
    assert f[0] == 1.0 and chi[0] == pytest.approx(1.0)
    assert n[0][0] ** 2 + n[1][0] ** 2 == pytest.approx(1.0)


def _flux_jacobian_speeds(E, F, d, c, h=1e-6):
    """Brute force: eigenvalues of the central-difference Jacobian of the 1D flux along d."""
    ndim = len(F)
    U0 = np.concatenate([[E], F])

    def flux(U):
        f, n, chi, D = O.closure(np.array([U[0]]), [np.array([U[1 + m]]) for m in range(ndim)], c)
        return np.array([U[1 + d]] + [c * c * D[d][m][0] * U[0] for m in range(ndim)])

    J = np.zeros((ndim + 1, ndim + 1))
    for k in range(ndim + 1):
        e = np.zeros(ndim + 1)
        e[k] = h * max(1.0, abs(U0[k]))
        J[:, k] = (flux(U0 + e) - flux(U0 - e)) / (2 * e[k])
    ev = np.linalg.eigvals(J)
    return ev.real.max(), ev.real.min()


@pytest.mark.parametrize("ndim", [2, 3])
def test_wave_speeds_match_flux_jacobian(ndim):
    rng = np.random.default_rng(11 + ndim)
    for _ in range(150):
        E, F = _rand_states(rng, 1, ndim, fmax=0.95)
        f, n, chi, D = O.closure(E, list(F), 1.0)
        for d in range(ndim):
            lmax, lmin = O.wave_speeds(f, n, d, 1.0)
            bmax, bmin = _flux_jacobian_speeds(E[0], F[:, 0], d, 1.0)
            assert lmax[0] == pytest.approx(bmax, abs=5e-7)
            assert lmin[0] == pytest.approx(bmin, abs=5e-7)


def test_wave_speed_special_cases():
    g = golden()
    c = 2.0
    f = np.array([0.0, 1.0, 1.0])
    n = [np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])]
    lmax, lmin = O.wave_speeds(f, n, 0, c)
    s = g["p1_speed_over_c"]["value"]
    assert lmax[0] == pytest.approx(s * c, rel=1e-15) and lmin[0] == pytest.approx(-s * c, rel=1e-15)
    assert lmax[1] == pytest.approx(c) and lmin[1] == pytest.approx(c)       # normal beam: upwind
    assert lmax[2] == pytest.approx(0.0, abs=1e-15) and lmin[2] == pytest.approx(0.0, abs=1e-15)
    rng = np.random.default_rng(3)
    E, F = _rand_states(rng, 1000, 3)
    f, n, _, _ = O.closure(E, list(F), c)
    for d in range(3):
        lmax, lmin = O.wave_speeds(f, n, d, c)
        assert np.all(np.abs(lmax) <= c * (1 + 1e-14)) and np.all(np.abs(lmin) <= c * (1 + 1e-14))
        assert np.all(lmax >= lmin)


def test_alpha_p1_closed_form():
    g = golden()
    s = 1 / math.sqrt(3)
    a, b, dd = O.hll_coefficients(np.array([s]), np.array([-s]), np.array([s]), np.array([-s]), 1.0)
    assert a[0] == pytest.approx(0.5) and b[0] == pytest.approx(0.5)
    for sdx in [1e-3, 0.5, 1.0, 25.0, 1e3, 1e6]:
        al = O.ap_alpha(np.array([sdx]), 1.0, np.array([0.0]), dd, 1.0)[0]
        closed = 1.0 / (1.0 + math.sqrt(3.0) * sdx / 2.0)
        assert al == pytest.approx(closed, rel=2e-15)
        assert 0.0 < al <= 1.0
    al25 = O.ap_alpha(np.array([25.0]), 1.0, np.array([0.0]), dd, 1.0)[0]
    assert al25 == pytest.approx(g["alpha_p1_sigma_dx_25"]["value"], rel=1e-12)
    # alpha -> 1 as sigma dx -> 0 (HLL recovered), and as fbar -> 1
    assert O.ap_alpha(np.array([1e-12]), 1.0, np.array([0.0]), dd, 1.0)[0] == pytest.approx(1.0)
    assert O.ap_alpha(np.array([1e4]), 1.0, np.array([1.0]), dd, 1.0)[0] == 1.0


def test_ap_flux_identity_p1():
    """With P1 speeds, a state satisfying the WB face relation sigma_f F_f = -c (P_R - P_L)/dx
    gives alpha F* = -c (E_R - E_L) / (3 sigma dx) exactly (Appendix C, Sect. 3.1.2)."""
    s = 1 / math.sqrt(3)
    rng = np.random.default_rng(0)
    for sdx in [0.01, 0.3, 1.0, 25.0, 1e2, 1e4]:
        EL, ER = rng.uniform(0.5, 2, 2)
        Ff = -(ER - EL) / (3.0 * sdx)                  # c = dx = 1, P = E/3
        FL = Ff + rng.uniform(-1, 1) * 1e-3
        FR = 2 * Ff - FL                               # face mean equals Ff
        a, b, dd = O.hll_coefficients(np.array([s]), np.array([-s]), np.array([s]), np.array([-s]), 1.0)
        al = O.ap_alpha(np.array([sdx]), 1.0, np.array([0.0]), dd, 1.0)
        Fstar = a * FL + b * FR + dd * (ER - EL)
        assert (al * Fstar)[0] == pytest.approx(-(ER - EL) / (3.0 * sdx), rel=1e-12)


def test_degenerate_face():
    a, b, dd = O.hll_coefficients(np.array([0.0]), np.array([0.0]), np.array([0.0]), np.array([0.0]), 1.0)
    assert a[0] == 0.5 and b[0] == 0.5 and dd[0] == 0.0


def _source_only_linearization(sigma):
    n = sigma.shape[0]
    sch = O.Scheme(n=(n, 1), bc=("periodic",) * 4)
    U = np.zeros((3, 1, n))
    U[0] = 1.0
    lin = O.linearize(sch, sigma.reshape(1, n), None, U, U, 1.0)
    for fc in lin.faces:                     # switch the hyperbolic part off
        fc["a"][:] = 0
        fc["b"][:] = 0
        fc["dd"][:] = 0
    for row in lin.Dpad:
        for r in row:
            for k in range(len(r)):
                r[k] = np.zeros_like(r[k])
    return lin


def test_wb_source_fourier_symbol():
    """Constant sigma: the periodic WB source operator has eigenvalues 1 + 2r(1 + cos 2 pi k/N),
    r = c sigma dt / 4, so every amplification factor is <= 1 (Appendix B; the
    paper's (1 - cos) is read as (1 + cos), which is what its discretisation gives)."""
    N, sig = 16, 3.7
    lin = _source_only_linearization(np.full(N, sig))
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros((3, 1, N))
        e[1, 0, k] = 1.0
        A[:, k] = O.operator(lin, e, "linear")[1, 0]
    r = sig / 4.0
    want = np.sort(1 + 2 * r * (1 + np.cos(2 * np.pi * np.arange(N) / N)))
    assert np.allclose(np.sort(np.linalg.eigvals(A).real), want, rtol=1e-13)
    # variable sigma: the inverse is a contraction in the 2-norm
    lin = _source_only_linearization(10 ** np.random.default_rng(1).uniform(-2, 3, N))
    for k in range(N):
        e = np.zeros((3, 1, N))
        e[1, 0, k] = 1.0
        A[:, k] = O.operator(lin, e, "linear")[1, 0]
    assert np.linalg.norm(np.linalg.inv(A), 2) <= 1.0 + 1e-12


def test_pressure_jacobian_small_flux_is_bounded_and_matches_the_limit():
    """Near F = 0 the Jacobian of P = D(E, F) E with respect to F tends to 0:
    chi'(f) ~ f and (3chi - 1)/2 E/|F| = 3f/(c(2+xi)) ~ 3f/(4c).  The literal product
    (3chi-1)/2 * E/|F| is rounding noise times an unbounded E/|F| (a plausible
    evaluation mistake); the Jacobian must stay finite and of order f."""
    c = 1.0
    for Fx in (1e-12, 1e-100, 1e-300):
        E = np.array([1e-6])
        F = [np.array([Fx]), np.array([0.5 * Fx])]
        J = O.pressure_jacobian(E, F, c)
        f = np.hypot(Fx, 0.5 * Fx) / (c * 1e-6)
        for d in range(2):
            for m in range(2):
                for l in range(2):
                    v = J[d][m][1 + l][0]
                    assert np.isfinite(v)
                    assert abs(v) <= 3.0 * f + 1e-300
    # the identity behind it, at moderate f where the literal form is accurate
    f = np.linspace(1e-3, 1.0, 200)
    xi = np.sqrt(4.0 - 3.0 * f * f)
    chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * xi)
    assert np.allclose(3.0 * chi - 1.0, 6.0 * f * f / (2.0 + xi), rtol=1e-10, atol=1e-15)


def test_pressure_jacobian_matches_high_precision_derivative_at_small_f():
    """At f = 1e-9 and 1e-12 the Jacobian dP/dF equals the central difference of
    P = D(E, F) E evaluated in 60-digit decimal arithmetic from the closure's
    definition (Sect. 2.2).  In double precision the literal (3chi - 1) is 0 or
    rounding noise there, so an evaluation through it misses the direction term
    (~3f/(4c)) entirely."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    c = 1.0

    def P_dec(E, F):
        Fm = (F[0] * F[0] + F[1] * F[1]).sqrt()
        f = Fm / (Decimal(c) * E)
        xi = (Decimal(4) - 3 * f * f).sqrt()
        chi = (3 + 4 * f * f) / (5 + 2 * xi)
        n = [F[0] / Fm, F[1] / Fm]
        return [[((1 - chi) / 2 if d == m else Decimal(0)) * E + (3 * chi - 1) / 2 * n[d] * n[m] * E
                 for m in range(2)] for d in range(2)]

    for fmag in (1e-9, 1e-12):
        E0 = 1.5
        F0 = [0.6 * fmag * c * E0, -0.8 * fmag * c * E0]
        J = O.pressure_jacobian(np.array([E0]), [np.array([F0[0]]), np.array([F0[1]])], c)
        for l in range(2):
            h = Decimal(fmag) * Decimal("1e-20")
            Fp = [Decimal(F0[0]), Decimal(F0[1])]
            Fq = list(Fp)
            Fp[l] += h
            Fq[l] -= h
            Pp, Pq = P_dec(Decimal(E0), Fp), P_dec(Decimal(E0), Fq)
            for d in range(2):
                for m in range(2):
                    ref = float((Pp[d][m] - Pq[d][m]) / (2 * h))
                    got = J[d][m][1 + l][0]
                    assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-30 * fmag, (fmag, l, d, m, got, ref)


def test_pressure_jacobian_matches_finite_difference_at_small_f():
    """At f = 1e-4 (where a central difference is still accurate) the Jacobian
    equals the finite difference of c^2-free P = D(E, F) E."""
    c = 1.0
    E0, F0 = 2.0, np.array([1.2e-4, -0.7e-4])

    def P(E, Fv):
        _, _, _, D = O.closure(np.array([E]), [np.array([Fv[0]]), np.array([Fv[1]])], c)
        return np.array([[D[d][m][0] * E for m in range(2)] for d in range(2)])

    J = O.pressure_jacobian(np.array([E0]), [np.array([F0[0]]), np.array([F0[1]])], c)
    h = 1e-9
    for l in range(2):
        e = np.zeros(2)
        e[l] = h
        fd = (P(E0, F0 + e) - P(E0, F0 - e)) / (2 * h)
        for d in range(2):
            for m in range(2):
                assert abs(J[d][m][1 + l][0] - fd[d, m]) <= 1e-6 * max(1.0, abs(fd[d, m])) + 1e-9
