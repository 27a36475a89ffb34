"""Pins of the oracle's explicit and semi-implicit steps (sources implicit,
hyperbolic part explicit, Sect. 3.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import m1_oracle as O

BC2 = ("outflow", "reflect", "dirichlet", "outflow")


def _p(src, seed, n=(14, 11), bc=BC2, dt=0.4, fmax=0.6):
    return W.random_problem(n, seed, source=src, flux_source="centered", bc=bc, dt=dt, fmax=fmax)


@pytest.mark.parametrize("src", ["none", "absorption"])
def test_semi_implicit_equals_explicit_without_opacity(src):
    """sigma = 0: no source acts, so the semi-implicit step is the explicit one."""
    p = _p(src, 31)
    p["sigma"] = np.zeros_like(p["sigma"])
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    a = O.semi_implicit_step(sch, p["sigma"], None, Un, p["dt"])
    b = O.explicit_step(sch, p["sigma"], None, Un, p["dt"])
    assert np.allclose(a, b, rtol=0, atol=1e-14 * np.abs(Un).max())


def test_uniform_state_closed_forms():
    """A spatially uniform periodic state has no flux divergence: the step is the
    source solve alone, F^{n+1} = F^n/(1 + c dt sigma), and with absorption
    E^{n+1} = E^n/(1 + c dt sigma)."""
    for src in ("none", "absorption"):
        p = _p(src, 32, bc=("periodic",) * 4)
        ny, nx = p["sigma"].shape
        p["sigma"] = np.full((ny, nx), 3.7)
        Un = np.stack([np.full((ny, nx), 1.3), np.full((ny, nx), 0.4), np.full((ny, nx), -0.2)])
        sch = O.Scheme.from_problem(p)
        U = O.semi_implicit_step(sch, p["sigma"], None, Un, p["dt"])
        k = p["c"] * p["dt"] * 3.7
        assert np.allclose(U[1:], Un[1:] / (1 + k), rtol=1e-14, atol=0)
        expect_E = Un[0] / (1 + k) if src == "absorption" else Un[0]
        assert np.allclose(U[0], expect_E, rtol=1e-14, atol=0)


def test_coupled_uniform_state_conserves_energy_and_keeps_equilibrium():
    p = _p("coupled_t", 33, bc=("periodic",) * 4, dt=50.0)
    ny, nx = p["sigma"].shape
    rng = np.random.default_rng(5)
    sig = float(rng.uniform(0.5, 5.0))
    p["sigma"] = np.full((ny, nx), sig)
    rc = np.full((ny, nx), 0.8)
    sch = O.Scheme.from_problem(p)
    # out of equilibrium: a_r T^4 != E; the exchange moves energy, E + rho c_v T is kept
    Un = np.stack([np.full((ny, nx), 0.2), np.zeros((ny, nx)), np.zeros((ny, nx)), np.full((ny, nx), 1.1)])
    U = O.semi_implicit_step(sch, p["sigma"], rc, Un, p["dt"])
    tot0 = Un[0] + rc * Un[3]
    tot1 = U[0] + rc * U[3]
    assert np.allclose(tot1, tot0, rtol=1e-13)
    # the implicit exchange relaxes toward a_r T^4 = E without overshoot
    gap0 = sch.a_r * Un[3] ** 4 - Un[0]
    gap1 = sch.a_r * U[3] ** 4 - U[0]
    assert np.all(np.abs(gap1) < np.abs(gap0)) and np.all(np.sign(gap1) == np.sign(gap0))
    # equilibrium is a fixed point
    Te = 0.9
    Ueq = np.stack([np.full((ny, nx), sch.a_r * Te ** 4), np.zeros((ny, nx)), np.zeros((ny, nx)),
                    np.full((ny, nx), Te)])
    Ue = O.semi_implicit_step(sch, p["sigma"], rc, Ueq, p["dt"])
    assert np.allclose(Ue, Ueq, rtol=1e-14, atol=1e-15)


def test_semi_implicit_free_streaming_moves_the_pulse_by_c_dt():
    """Vacuum, a pulse with F = cE along x (f = 1): with lambda+ = c, lambda- = 0 the
    flux is upwind, and one step moves the energy centroid by exactly c dt and
    keeps the total energy (no boundary flux while the pulse is inside)."""
    p = W.base_problem((40, 6), dt=0.5, flux_source="centered", bc=["outflow"] * 4)
    nx, ny = 40, 6
    x = np.arange(nx) + 0.5
    prof = 1e-12 + np.exp(-((x - 20.0) / 2.5) ** 2)
    E = np.tile(prof, (ny, 1))
    Un = np.stack([E, p["c"] * E, np.zeros_like(E)])
    sigma = np.zeros((ny, nx))
    sch = O.Scheme.from_problem(p)
    U = O.semi_implicit_step(sch, sigma, None, Un, p["dt"])
    c0 = (Un[0] * x).sum() / Un[0].sum()
    c1 = (U[0] * x).sum() / U[0].sum()
    assert abs(U[0].sum() - Un[0].sum()) <= 1e-12 * Un[0].sum()
    assert abs((c1 - c0) - p["c"] * p["dt"]) <= 1e-9


def test_semi_implicit_approaches_explicit_as_dt_shrinks():
    """Both are first-order steps of the same equation: their difference is O(dt^2)."""
    p = _p("absorption", 34, dt=1.0)
    p["sigma"] = np.random.default_rng(1).uniform(0.1, 1.0, size=p["sigma"].shape)
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    diffs = []
    for dt in (2.0 ** -7, 2.0 ** -8, 2.0 ** -9):
        a = O.semi_implicit_step(sch, p["sigma"], None, Un, dt)
        b = O.explicit_step(sch, p["sigma"], None, Un, dt)
        diffs.append(np.linalg.norm(a - b))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_semi_implicit_rejects_the_well_balanced_source():
    p = W.random_problem((6, 5), 35, source="none", flux_source="wb", bc=BC2)
    sch = O.Scheme.from_problem(p)
    with pytest.raises(ValueError):
        O.semi_implicit_step(sch, p["sigma"], None, O.state_from_problem(p, "n"), p["dt"])


def beam_width_at_mid_height(E, e_bg):
    """Full width at half maximum, in cells, of E - E_background along the
    horizontal cut at mid-height (mean of the two middle rows)."""
    n = E.shape[0]
    cut = 0.5 * (E[n // 2 - 1] + E[n // 2]) - e_bg
    return int(np.sum(cut > 0.5 * cut.max())), int(np.argmax(cut))


def test_beam45_width_computed_versus_fixed_eigenvalues():
    """Sect. 5.3: a beam sampled over 8 cells enters a 128^2 vacuum box at 45
    degrees.  The paper reports a width at mid-height of about 24 cells with the
    computed eigenvalues and about 30 cells with fixed +-c.  The width is read
    as the full width at half maximum of E above the background; the oracle's
    steady state (500 explicit steps at the CFL limit, sigma = 0 so the
    semi-implicit step is the same) gives 22 and 28.  The pin brackets the
    printed figures with the reading's slack and requires the ordering; the
    beam centre must sit on the 45-degree line (x = 51.5 at mid-height)."""
    widths = {}
    for floor in (0.0, 1.0):
        p = W.beam45(lambda_floor=floor)
        sch = O.Scheme.from_problem(p)
        U = np.stack([p["E"], p["F"][0], p["F"][1]])
        for _ in range(500):
            U = O.semi_implicit_step(sch, p["sigma"], None, U, p["dt"])
        assert np.isfinite(U).all()
        widths[floor], centre = beam_width_at_mid_height(U[0], p["E"][0, 0])
        assert abs(centre - 51.5) <= 2.0
    computed, fixed = widths[0.0], widths[1.0]
    assert 20 <= computed <= 26
    assert 26 <= fixed <= 33
    assert fixed - computed >= 4


def test_semi_implicit_hll_keeps_realizability_without_the_asymptotic_factor():
    """The HLL scheme keeps |F| <= cE under the 2D CFL bound c dt <= dx/2 (the
    realizability property of the M1 HLL flux).  On the Voronoi workload at 512^2
    (fronts running into sigma ~ 1e-3..1e4 cells) 20 semi-implicit steps at the
    bound keep every cell realizable and E positive when the asymptotic factor
    alpha is off.  (With alpha on, alpha scales only the energy flux and the
    same run loses realizability within a dozen steps; that is a property of
    the scheme, not pinned here.)"""
    p = W.voronoi_opacity(seed=1000)
    p["flux_source"] = "centered"
    p["ap"] = False
    sch = O.Scheme.from_problem(p)
    U = np.stack([p["E"], p["F"][0], p["F"][1]])
    worst = 0.0
    for _ in range(20):
        U = O.semi_implicit_step(sch, p["sigma"], None, U, 0.5)
        assert U[0].min() > 0.0
        worst = max(worst, float((np.sqrt(U[1] ** 2 + U[2] ** 2) / (p["c"] * U[0])).max()))
    print(f"max |F|/cE over the run: {worst:.4f}")
    assert 0.5 < worst <= 1.0 + 1e-12
