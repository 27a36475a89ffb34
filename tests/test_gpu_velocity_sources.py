"""GPU parity of the velocity-dependent sources (Sect. 2.3; step 3 of the splitting,
Sect. 3.2) against the oracle: the change of the state, per component, to 1e-12
relative.  Full size: the 192^3 ionisation-front workload with its solenoidal
velocity field, checked on 100 000 sampled cells (the step is cell-local, so the
oracle evaluates exactly those cells)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import m1_oracle as O

pytestmark = pytest.mark.gpu

BC2 = ("outflow", "reflect", "dirichlet", "outflow")
BC3 = ("outflow", "dirichlet", "reflect", "outflow", "periodic", "periodic")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _state(p):
    comps = [p["E"]] + [p["F"][m] for m in range(p["ndim"])]
    if p["source"] == "coupled_t":
        comps.append(p["T"])
    return np.stack(comps)


@pytest.mark.parametrize("n,src", [((131, 37), "coupled_t"), ((131, 37), "none"), ((23, 19, 11), "coupled_t"),
                                   ((23, 19, 11), "absorption")])
def test_velocity_sources_parity(n, src):
    import paper_2011_13926_amd as P
    _say("velocity sources", n, src)
    bc = BC2 if len(n) == 2 else BC3
    p = W.random_problem(n, 41, source=src, bc=bc, fmax=0.9)
    rng = np.random.default_rng(42)
    u = rng.uniform(-0.05, 0.05, (len(n),) + W.grid_shape(n)) * p["c"]
    U0 = _state(p)
    sch = O.Scheme.from_problem(p)
    ref = O.velocity_source_step(sch, p["sigma"], U0, u, 0.7)
    s = P.Solver(p)
    try:
        U = s.to_device(U0)
        st, stats = s.velocity_sources(U, u, dt=0.7)
        assert st == P.M1_OK
        got = U.cpu().numpy()
    finally:
        s.close()
    for c in range(U0.shape[0]):
        if np.any(ref[c] != U0[c]):
            assert _rel(got[c] - U0[c], ref[c] - U0[c]) <= 1e-12, c
            # worst element against the largest change (not diluted by the grid)
            assert np.max(np.abs(got[c] - ref[c])) <= 1e-11 * np.max(np.abs(ref[c] - U0[c])), c
        else:
            assert np.array_equal(got[c], U0[c]), c


def test_velocity_sources_error_paths_leave_the_state():
    import torch
    import paper_2011_13926_amd as P
    p = W.random_problem((40, 33), 43, source="coupled_t", bc=BC2)
    U0 = _state(p)
    s = P.Solver(p)
    try:
        U = s.to_device(U0)
        before = U.clone()
        u = np.zeros((2,) + W.grid_shape((40, 33)))
        u[1, 3, 4] = np.nan
        st, _ = s.velocity_sources(U, u, dt=0.5, raise_on_fail=False)
        assert st == P.M1_ERR_NONFINITE and torch.equal(U, before)
        st, _ = s.velocity_sources(U, np.zeros_like(u), dt=-1.0, raise_on_fail=False)
        assert st == P.M1_ERR_INVALID_ARG and torch.equal(U, before)
    finally:
        s.close()


def test_ionization_front_192_velocity_sources_sampled():
    import paper_2011_13926_amd as P
    _say("ionisation front 192^3 with velocity")
    p = W.ionization_front(with_velocity=True)
    # a state with flux: the front's own initial state has F = 0 and E = floor
    rng = np.random.default_rng(44)
    g = W.grid_shape(p["n"])
    p["E"] = 10.0 ** rng.uniform(-6, 0, g)
    f = rng.uniform(0, 0.95, g)
    d = rng.standard_normal((3,) + g)
    d /= np.sqrt((d ** 2).sum(0))
    p["F"] = p["c"] * p["E"][None] * f[None] * d
    U0 = _state(p)
    dt = 100.0
    s = P.Solver(p, restart=1)
    try:
        U = s.to_device(U0)
        st, stats = s.velocity_sources(U, p["velocity"], dt=dt)
        assert st == P.M1_OK
        got = U.cpu().numpy().reshape(U0.shape[0], -1)
    finally:
        s.close()
    idx = np.random.default_rng(45).choice(U0[0].size, 100000, replace=False)
    sch = O.Scheme.from_problem(p)
    Us = U0.reshape(U0.shape[0], -1)[:, idx]
    ref = O.velocity_source_step(sch, p["sigma"].reshape(-1)[idx], Us, p["velocity"].reshape(3, -1)[:, idx], dt)
    for c in range(4):
        assert _rel(got[c, idx] - Us[c], ref[c] - Us[c]) <= 1e-12, c
        assert np.max(np.abs(got[c, idx] - ref[c])) <= 1e-11 * np.max(np.abs(ref[c] - Us[c])), c
    _say(f"  max relative change of E {np.abs((got[0, idx] - Us[0]) / Us[0]).max():.2e}, "
         f"{stats['seconds'] * 1e3:.1f} ms")
