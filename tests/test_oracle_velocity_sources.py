"""Pins of the oracle's velocity-dependent source terms (Sect. 2.3) and of the
explicit step that adds them after the implicit radiation step (Sect. 3.2)."""
import numpy as np
import pytest

import workloads as W
from oracle import m1_oracle as O


def _sch(ndim, source):
    n = (6, 5) if ndim == 2 else (4, 3, 5)
    p = W.base_problem(n, dt=1.0, source=source, c=3.0, a_r=0.7)
    return O.Scheme.from_problem(p), W.grid_shape(n)


@pytest.mark.parametrize("ndim,source", [(2, "coupled_t"), (3, "absorption")])
def test_no_velocity_no_source(ndim, source):
    sch, g = _sch(ndim, source)
    rng = np.random.default_rng(1)
    U = np.concatenate([rng.uniform(0.5, 2, (1,) + g), rng.uniform(-0.3, 0.3, (ndim,) + g)]
                       + ([rng.uniform(0.5, 2, (1,) + g)] if source == "coupled_t" else []))
    V = O.velocity_source_step(sch, rng.uniform(0.1, 3, g), U, np.zeros((ndim,) + g), 0.7)
    assert np.array_equal(V, U)


def test_isotropic_state_closed_forms():
    """F = 0: P = E/3 I, so S_E = (4/3)(sigma/c) E u.u and S_F = sigma u (E/3 + a_r T^4)."""
    sch, g = _sch(2, "coupled_t")
    rng = np.random.default_rng(2)
    E = rng.uniform(0.5, 2, g)
    T = rng.uniform(0.5, 2, g)
    sig = rng.uniform(0.1, 3, g)
    u = rng.uniform(-0.2, 0.2, (2,) + g)
    U = np.stack([E, np.zeros(g), np.zeros(g), T])
    SE, SF = O.velocity_sources(sch, sig, U, u)
    uu = u[0] ** 2 + u[1] ** 2
    assert np.allclose(SE, 4.0 / 3.0 * sig / sch.c * E * uu, rtol=1e-14, atol=0)
    for m in range(2):
        assert np.allclose(SF[m], sig * u[m] * (E / 3.0 + sch.a_r * T ** 4), rtol=1e-14, atol=0)


def test_comoving_equilibrium_has_no_first_order_flux_source():
    """Radiation in equilibrium with gas moving at u = beta c d carries F = (4/3) E u in
    the laboratory frame at first order.  The flux equation's total source
    -c sigma F + c S_F(u) then cancels at first and second order (u.P = E u/3 up to
    the closure's O(f^2) anisotropy, and u (u.F) is itself O(beta^3)): halving u
    divides it by eight.  S_E(u) = (sigma/c)(4/3 + 1 + 1/3) E u.u = (8/3) beta^2 c sigma E
    at leading order."""
    sch, g = _sch(3, "coupled_t")
    rng = np.random.default_rng(3)
    T = rng.uniform(0.5, 2, g)
    E = sch.a_r * T ** 4
    sig = rng.uniform(0.1, 3, g)
    d = rng.standard_normal((3,) + g)
    d /= np.sqrt((d ** 2).sum(0))
    out = []
    for beta in (1e-3, 5e-4):
        u = beta * sch.c * d
        F = 4.0 / 3.0 * E * u
        SE, SF = O.velocity_sources(sch, sig, np.concatenate([E[None], F, T[None]]), u)
        scale = sch.c * sig * E
        net = np.abs((-sch.c * sig * F + sch.c * SF) / scale).max()
        out.append(net)
        assert net < 10 * beta ** 3
        assert np.allclose(SE / scale, 8.0 / 3.0 * beta ** 2, rtol=1e-5, atol=0)
    assert 7.0 < out[0] / out[1] < 9.0
