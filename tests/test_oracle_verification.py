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


def test_marshak_wave_asymptotic_preserving_scheme_reaches_the_diffusion_reference():
    """Sect. 5.1 (nondimensional): 400 cells at sigma dx = 25, gas coupled (rho c_v = 1),
    a source at T = 1 lit on the left of a medium at 0.3.  Ten implicit steps of the
    scheme with the asymptotic correction (dt = 1e4, c sigma dt = 2.5e5) against ten
    backward-Euler steps of the equilibrium diffusion limit: the gas temperature agrees
    to 1e-3 in relative L2 and the wave front (T = 0.65) sits in the same cell.  A
    dropped or mis-scaled alpha moves the front by a hundred cells (plain HLL: 214
    against 45)."""
    import workloads as W
    n, dt, nsteps, T0 = 400, 1e4, 10, 0.3
    Tref = np.full(n, T0)
    for _ in range(nsteps):
        Tref = O.equilibrium_diffusion_step(Tref, Tref, dt, np.full(n, 25.0), 1.0, left=1.0)
    p = W.marshak_1d(dt=dt, ap=True)
    sch = O.Scheme.from_problem(p)
    U = np.stack([p["E"], p["F"][0], p["F"][1], p["T"]])
    for _ in range(nsteps):
        r = O.implicit_step(sch, p["sigma"], p["rho_cv"], U, dt, rtol=1e-10, newton_rtol=1e-8, newton_max=30,
                            max_iters=40000)
        assert r.converged
        U = r.U
    Tg = U[3, 0]
    assert np.linalg.norm(Tg - Tref) / np.linalg.norm(Tref) <= 1e-3
    assert int(np.argmax(Tg < 0.65)) == int(np.argmax(Tref < 0.65)) == 45
