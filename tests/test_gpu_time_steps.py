"""GPU parity of the explicit and semi-implicit steps (Sect. 3.1) through the C ABI.

Each case runs the HIP step and the oracle's step on the same seeded input and
compares the state change U^{n+1} - U^n component by component: 1e-12 relative
for the explicit step (one residual evaluation, FP64), 1e-10 for the
semi-implicit step (the per-cell temperature Newton solve stops per cell on
the GPU and for the whole grid in the oracle).  Full sizes: the 2D workloads
against the whole-grid oracle; the 256^3 coupled workload on interior windows,
where the oracle runs on the window plus a one-cell halo (the scheme's stencil
has radius one, so the window's own boundary only reaches the halo)."""
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


def _state(p, which="n"):
    if which == "n":
        comps = [p["En"]] + [p["Fn"][m] for m in range(p["ndim"])]
        if p["source"] == "coupled_t":
            comps.append(p["Tn"])
    else:
        comps = [p["E"]] + [p["F"][m] for m in range(p["ndim"])]
        if p["source"] == "coupled_t":
            comps.append(p["T"])
    return np.stack(comps)


def _gpu_step(p, Un, kind, **kw):
    import paper_2011_13926_amd as P
    s = P.Solver(p, **kw)
    try:
        U = s.to_device(Un)
        st, stats = getattr(s, kind)(U)
        return st, stats, U.cpu().numpy()
    finally:
        s.close()


def _oracle_step(p, Un, kind):
    sch = O.Scheme.from_problem(p)
    f = O.explicit_step if kind == "explicit_step" else O.semi_implicit_step
    return f(sch, p["sigma"], p.get("rho_cv"), Un, p["dt"])


def _check(got, ref, Un, tol):
    """Each component's increment over the step against the oracle's: relative L2 within
    tol, and the worst element within 10 tol of the largest increment, so that an error
    confined to a boundary row is not diluted by the rest of the grid."""
    for c in range(got.shape[0]):
        assert _rel(got[c] - Un[c], ref[c] - Un[c]) <= tol, c
        scale = np.max(np.abs(ref[c] - Un[c]))
        assert np.max(np.abs(got[c] - ref[c])) <= 10 * tol * max(scale, 1e-300), c


CASES = []
for _src in ("none", "absorption", "coupled_t"):
    CASES.append(((131, 37), BC2, _src, "centered"))
    CASES.append(((23, 19, 11), BC3, _src, "centered"))
CASES += [((131, 37), BC2, "coupled_t", "wb"), ((23, 19, 11), BC3, "none", "wb"),
          ((1, 5), ("periodic", "periodic", "reflect", "dirichlet"), "absorption", "centered"),
          ((64, 1), ("outflow", "outflow", "periodic", "periodic"), "none", "centered")]


@pytest.mark.parametrize("n,bc,src,fs", CASES)
def test_explicit_step_parity(n, bc, src, fs):
    _say("explicit step", n, bc, src, fs)
    p = W.random_problem(n, 21, source=src, flux_source=fs, bc=bc, dt=0.3, fmax=0.8)
    Un = _state(p)
    st, stats, got = _gpu_step(p, Un, "explicit_step")
    assert st == 0 and stats["newton_iters"] == 0 and stats["krylov_iters"] == 0
    _check(got, _oracle_step(p, Un, "explicit_step"), Un, 1e-12)


@pytest.mark.parametrize("n,bc,src,fs", [c for c in CASES if c[3] == "centered"])
def test_semi_implicit_step_parity(n, bc, src, fs):
    """sigma spans 1e-2..1e2 per cell, so c dt sigma reaches 30: the stiff source
    regime the semi-implicit step exists for."""
    _say("semi-implicit step", n, bc, src, fs)
    p = W.random_problem(n, 22, source=src, flux_source=fs, bc=bc, dt=0.3, fmax=0.8)
    Un = _state(p)
    st, stats, got = _gpu_step(p, Un, "semi_implicit_step")
    assert st == 0
    _check(got, _oracle_step(p, Un, "semi_implicit_step"), Un, 1e-10)


@pytest.mark.parametrize("src", ["none", "absorption", "coupled_t"])
def test_semi_implicit_without_opacity_is_the_explicit_step_bitwise(src):
    """sigma = 0: the source solve is the identity (k = 0), on the GPU to the bit."""
    import paper_2011_13926_amd as P
    _say("sigma = 0", src)
    p = W.random_problem((70, 9), 23, source=src, flux_source="centered", bc=BC2, dt=0.3)
    p["sigma"] = np.zeros_like(p["sigma"])
    Un = _state(p)
    s = P.Solver(p)
    try:
        Ua = s.to_device(Un)
        Ub = s.to_device(Un)
        s.explicit_step(Ua)
        s.semi_implicit_step(Ub)
        assert np.array_equal(Ua.cpu().numpy(), Ub.cpu().numpy())
    finally:
        s.close()


@pytest.mark.parametrize("src,n", [("coupled_t", (70, 9)), ("absorption", (23, 19, 11))])
def test_nsteps_in_one_call_equals_single_steps_bitwise(src, n):
    import torch
    import paper_2011_13926_amd as P
    _say("nsteps", src, n)
    bc = BC2 if len(n) == 2 else BC3
    p = W.random_problem(n, 26, source=src, flux_source="centered", bc=bc, dt=0.2, fmax=0.5,
                         sigma_range=(1e-2, 1e0))
    Un = _state(p)
    s = P.Solver(p)
    try:
        for kind in ("explicit_step", "semi_implicit_step"):
            Ua = s.to_device(Un)
            Ub = s.to_device(Un)
            getattr(s, kind)(Ua, nsteps=7)
            for _ in range(7):
                getattr(s, kind)(Ub)
            assert torch.equal(Ua, Ub), kind
    finally:
        s.close()


def test_time_step_keeps_the_linearisation():
    """A time step between m1_linearize and m1_residual does not change R."""
    import paper_2011_13926_amd as P
    _say("linearisation kept")
    p = W.random_problem((40, 33), 27, source="absorption", flux_source="centered", bc=BC2, dt=0.3)
    U = _state(p, "0")
    Un = _state(p)
    s = P.Solver(p, U_lin=U, U_n=Un)
    try:
        R0 = s.residual().cpu().numpy()
        V = s.to_device(Un)
        s.semi_implicit_step(V, nsteps=3)
        s.explicit_step(V)
        R1 = s.residual().cpu().numpy()
        assert np.array_equal(R0, R1)
    finally:
        s.close()


def test_semi_implicit_rejects_the_well_balanced_source_and_bad_input():
    import torch
    import paper_2011_13926_amd as P
    _say("semi-implicit error paths")
    p = W.random_problem((40, 33), 24, source="absorption", flux_source="wb", bc=BC2, dt=0.3)
    Un = _state(p)
    s = P.Solver(p)
    try:
        U = s.to_device(Un)
        before = U.clone()
        st, _ = s.semi_implicit_step(U, raise_on_fail=False)
        assert st == P.M1_ERR_INVALID_ARG and torch.equal(U, before)
        for bad_dt in (0.0, -1.0, float("nan")):
            st, _ = s.explicit_step(U, dt=bad_dt, raise_on_fail=False)
            assert st == P.M1_ERR_INVALID_ARG and torch.equal(U, before)
        for bad_n in (0, -3):
            st, _ = s.explicit_step(U, nsteps=bad_n, raise_on_fail=False)
            assert st == P.M1_ERR_INVALID_ARG and torch.equal(U, before)
        U[0, 3, 4] = -1.0
        st, _ = s.explicit_step(U, raise_on_fail=False)
        assert st == P.M1_ERR_INVALID_ARG
        U[0, 3, 4] = float("inf")
        st, _ = s.explicit_step(U, raise_on_fail=False)
        assert st == P.M1_ERR_NONFINITE
    finally:
        s.close()


def test_time_steps_agree_with_the_implicit_step_as_dt_shrinks():
    """Explicit, semi-implicit and (converged) implicit steps are all first-order
    in time and share the spatial operator: their differences fall like dt^2."""
    import paper_2011_13926_amd as P
    _say("dt -> 0")
    diffs = []
    for dt in (2.0 ** -6, 2.0 ** -7, 2.0 ** -8):
        p = W.random_problem((40, 33), 25, source="coupled_t", flux_source="centered", bc=BC2, dt=dt,
                             fmax=0.6, sigma_range=(1e-2, 1e0))
        Un = _state(p)
        out = {}
        for kind in ("explicit_step", "semi_implicit_step", "implicit_step"):
            s = P.Solver(p, rtol=1e-13, newton_rtol=1e-13, newton_max=40)
            try:
                U = s.to_device(Un)
                st, _ = getattr(s, kind)(U)
                assert st == 0
                out[kind] = U.cpu().numpy()
            finally:
                s.close()
        d_semi = np.abs(out["semi_implicit_step"] - out["implicit_step"]).max()
        d_expl = np.abs(out["explicit_step"] - out["implicit_step"]).max()
        diffs.append((d_semi, d_expl))
        _say(f"  dt={dt:.2e} |semi - implicit|={d_semi:.3e} |explicit - implicit|={d_expl:.3e}")
    for a, b in zip(diffs, diffs[1:]):
        assert 3.0 <= a[0] / b[0] <= 5.0
        assert 3.0 <= a[1] / b[1] <= 5.0


def test_beam45_many_steps_matches_oracle_and_paper_widths():
    """The 45-degree beam (Sect. 5.3), 128^2, 500 semi-implicit steps at the CFL
    limit on the GPU: the final state matches the oracle's 500 steps, and the
    widths at mid-height reproduce the ordering the paper reports (about 24 cells
    with computed eigenvalues, about 30 with fixed +-c; full width at half
    maximum of E above the background)."""
    import paper_2011_13926_amd as P
    widths = {}
    for floor in (0.0, 1.0):
        _say("beam45, lambda floor", floor)
        p = W.beam45(lambda_floor=floor)
        U0 = np.stack([p["E"], p["F"][0], p["F"][1]])
        s = P.Solver(p)
        try:
            U = s.to_device(U0)
            s.semi_implicit_step(U, nsteps=500)
            got = U.cpu().numpy()
        finally:
            s.close()
        sch = O.Scheme.from_problem(p)
        ref = U0
        for _ in range(500):
            ref = O.semi_implicit_step(sch, p["sigma"], None, ref, p["dt"])
        _check(got, ref, U0, 1e-10)
        n = got.shape[1]
        cut = 0.5 * (got[0, n // 2 - 1] + got[0, n // 2]) - p["E"][0, 0]
        widths[floor] = int(np.sum(cut > 0.5 * cut.max()))
        _say(f"  width at mid-height {widths[floor]} cells")
    assert 20 <= widths[0.0] <= 26 and 26 <= widths[1.0] <= 33 and widths[1.0] - widths[0.0] >= 4


@pytest.mark.parametrize("name,make,kind", [
    ("beam_shadow_1024", lambda: W.beam_shadow(dt=0.5), "semi_implicit_step"),
    ("voronoi_512_centred", lambda: dict(W.voronoi_opacity(seed=1000, dt=0.5), flux_source="centered"),
     "semi_implicit_step"),
    ("voronoi_512_wb", lambda: W.voronoi_opacity(seed=1000, dt=0.5), "explicit_step"),
])
def test_full_size_2d_step_against_whole_grid_oracle(name, make, kind):
    _say("full size", name, kind)
    p = make()
    Un = _state(p, "0")
    st, stats, got = _gpu_step(p, Un, kind)
    assert st == 0
    _say(f"  {stats['seconds'] * 1e3:.2f} ms (first call), f>1 cells {stats['cells_f_gt_1']}")
    _check(got, _oracle_step(p, Un, kind), Un, 1e-10)


def _window(p, lo, size):
    """The sub-problem on cells lo - 1 .. lo + size (a one-cell halo), outflow faces."""
    sl = tuple(slice(l - 1, l + size + 1) for l in reversed(lo))
    n = tuple(size + 2 for _ in lo)
    q = W.base_problem(n, dt=p["dt"], source=p["source"], flux_source=p["flux_source"],
                       ap=p["ap"], lambda_floor=p["lambda_floor"], bc=["outflow"] * (2 * len(lo)))
    q["sigma"] = p["sigma"][sl]
    q["rho_cv"] = None if p["rho_cv"] is None else p["rho_cv"][sl]
    q["E"] = p["E"][sl]
    q["F"] = p["F"][(slice(None),) + sl]
    q["T"] = None if p["T"] is None else p["T"][sl]
    return q, sl


def test_coupled_lognormal_256_semi_implicit_on_interior_windows():
    """256^3 with the gas-temperature row, centred flux source, dt = 0.3 (below
    the 3D CFL limit 1/3): the GPU step on the whole grid; the oracle on three
    interior 24^3 windows."""
    _say("coupled lognormal 256^3 semi-implicit")
    p = W.coupled_lognormal(dt=0.3)
    p["flux_source"] = "centered"
    Un = _state(p, "0")
    st, stats, got = _gpu_step(p, Un, "semi_implicit_step", restart=1)
    assert st == 0
    # total energy E + rho c_v T is conserved on the periodic box
    rc = p["rho_cv"]
    tot0 = Un[0].sum() + (rc * Un[-1]).sum()
    tot1 = got[0].sum() + (rc * got[-1]).sum()
    assert abs(tot1 - tot0) <= 1e-12 * tot0
    for lo in ((1, 1, 1), (100, 37, 200), (231, 231, 231)):
        q, sl = _window(p, lo, 24)
        Uq = _state(q, "0")
        ref = _oracle_step(q, Uq, "semi_implicit_step")
        inner = (slice(None),) + (slice(1, -1),) * 3
        gsl = (slice(None),) + tuple(slice(s.start + 1, s.stop - 1) for s in sl)
        _check(got[gsl], ref[inner], Uq[inner], 1e-10)
