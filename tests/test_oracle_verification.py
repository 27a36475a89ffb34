"""Pins of the 1D verification references (Sect. 5.1 Marshak wave, Sect. 5.2
steady state across an opacity jump): the equilibrium diffusion step of Eq.
"diffusionEqua" that the Marshak comparison is measured against."""
import numpy as np
from scipy.special import erfc

from oracle import m1_oracle as O


def test_equilibrium_diffusion_small_perturbation_is_the_erfc_profile():
    """A small temperature step dT held at the boundary of a uniform medium: the
    linearised equation is the heat equation with diffusivity
    kappa = (c/3 sigma) 4 a_r T^3 / (4 a_r T^3 + rho c_v), whose half-space solution
    is dT erfc(x / 2 sqrt(kappa t)) (x measured from the ghost cell's centre)."""
    n, T0, dT, sig, rc = 400, 1.0, 1e-4, 25.0, 3.0
    Tn = np.full(n, T0)
    dt, steps = 200.0, 200
    for _ in range(steps):
        Tn = O.equilibrium_diffusion_step(Tn, Tn, dt, np.full(n, sig), rc, left=T0 + dT)
    kap = (1.0 / (3.0 * sig)) * 4.0 * T0 ** 3 / (4.0 * T0 ** 3 + rc)
    x = np.arange(n) + 1.0
    ref = dT * erfc(x / (2.0 * np.sqrt(kap * dt * steps)))
    assert np.linalg.norm((Tn - T0) - ref) / np.linalg.norm(ref) < 3e-3


def test_equilibrium_diffusion_conserves_total_energy_without_boundary_flux():
    rng = np.random.default_rng(5)
    T = 0.5 + rng.random(50)
    s = 10.0 ** rng.uniform(-1, 2, 50)
    r = 0.5 + rng.random(50)
    tot0 = (T ** 4 + r * T).sum()
    for left in (None, "periodic"):
        T1 = O.equilibrium_diffusion_step(T, T, 30.0, s, r, left=left)
        assert abs((T1 ** 4 + r * T1).sum() - tot0) <= 1e-13 * tot0
        assert np.abs(T1 - T).max() > 1e-3


def test_equilibrium_diffusion_without_heat_capacity_is_the_linear_diffusion_step():
    """rho c_v = 0 leaves E = a_r T^4 alone: one step equals the backward-Euler
    step of the linear diffusion limit of E (periodic), a separate routine."""
    rng = np.random.default_rng(6)
    T = 0.5 + rng.random(40)
    s = 10.0 ** rng.uniform(-1, 2, 40)
    Te = O.equilibrium_diffusion_step(T, T, 30.0, s, 0.0, left="periodic")
    Ed = O.discrete_diffusion_step(s[None, :], (T ** 4)[None, :], 30.0)[0]
    assert np.abs(Te ** 4 - Ed).max() <= 1e-12 * Ed.max()
