"""GPU parity of the aggregation multigrid preconditioner (pc = M1_PC_MULTIGRID)
against the oracle's multigrid (oracle/m1_multigrid.py), through the C ABI.

One V-cycle z = M^{-1} r (m1_precondition) element by element at 1e-12 (the
coarsest level is an exact solve on both sides: a dense inverse on the GPU, a
sparse LU in the oracle, so the cycles agree to rounding times the coarse
condition number); fixed-iteration and converged implicit steps with the
multigrid preconditioner at 1e-10; the mixed-precision form within 1e-8 of the
FP64 oracle; and the iteration reduction on a Voronoi field."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import m1_multigrid as MG
from oracle import m1_oracle as O

pytestmark = pytest.mark.gpu

BC2 = {
    "periodic": ("periodic",) * 4,
    "mixed": ("outflow", "reflect", "dirichlet", "outflow"),
    "walls": ("dirichlet", "dirichlet", "reflect", "reflect"),
}
BC3 = {
    "mixed": ("outflow", "dirichlet", "reflect", "outflow", "periodic", "periodic"),
    "open": ("outflow", "outflow", "reflect", "reflect", "dirichlet", "outflow"),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _maxabs_by_component(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return max(float(np.max(np.abs(a[c] - b[c])) / max(np.max(np.abs(b[c])), 1e-300)) for c in range(b.shape[0]))


# (grid, bc, source, flux source, nu1, nu2, nmin, nu1 coarse, nu2 coarse) -- odd and even
# extents, several levels, a grid already at the coarsest size, 3D with 4x4 and 5x5
# blocks, other sweep counts below the finest level (-1: the same)
CYCLE_CASES = [
    ((40, 33), BC2["mixed"], "none", "wb", 1, 1, 0, -1, -1),
    ((64, 48), BC2["periodic"], "absorption", "centered", 2, 1, 0, -1, -1),
    ((37, 29), BC2["walls"], "coupled_t", "wb", 1, 2, 0, -1, -1),
    ((33, 7), BC2["periodic"], "none", "wb", 0, 1, 4, -1, -1),
    ((30, 31), BC2["mixed"], "absorption", "wb", 1, 0, 8, -1, -1),
    ((8, 6), BC2["mixed"], "none", "wb", 1, 1, 0, -1, -1),
    ((17, 13, 11), BC3["mixed"], "none", "wb", 1, 1, 0, -1, -1),
    ((12, 10, 9), BC3["open"], "coupled_t", "wb", 1, 1, 0, -1, -1),
    ((16, 16, 16), ("periodic",) * 6, "absorption", "centered", 2, 2, 4, -1, -1),
    ((72, 40), BC2["mixed"], "none", "wb", 3, 3, 0, 1, 1),
    ((45, 64), BC2["walls"], "absorption", "wb", 2, 1, 4, 0, 2),
    ((20, 18, 14), BC3["open"], "coupled_t", "wb", 2, 2, 0, 1, 0),
    # 2D finest-level sweeps fused into the staged operator on 64 x 16 tiles: several
    # tiles with ragged tails, the first two sweeps in one launch (nu1 >= 2), the
    # coupled 4 x 4 blocks
    ((131, 37), BC2["mixed"], "none", "wb", 4, 4, 0, 2, 2),
    ((70, 33), BC2["walls"], "coupled_t", "wb", 2, 3, 0, -1, -1),
    ((66, 18), BC2["periodic"], "absorption", "centered", 3, 1, 0, 1, 1),
    # two sweeps per launch with one periodic and one bounded direction: the halo's
    # corners are grid cells or ghosts of grid cells there
    ((70, 40), ("periodic", "periodic", "outflow", "dirichlet"), "coupled_t", "wb", 3, 2, 0, 1, 1),
    ((70, 40), ("outflow", "reflect", "periodic", "periodic"), "none", "wb", 2, 4, 0, -1, -1),
]


@pytest.mark.parametrize("n,bc,src,fs,nu1,nu2,nmin,nu1c,nu2c", CYCLE_CASES)
def test_vcycle_parity(n, bc, src, fs, nu1, nu2, nmin, nu1c, nu2c):
    import paper_2011_13926_amd as P
    _say("multigrid cycle parity", n, bc, src, fs, nu1, nu2, nmin, nu1c, nu2c)
    p = W.random_problem(n, 21, source=src, flux_source=fs, bc=bc, dt=3.0)
    sch = O.Scheme.from_problem(p)
    U = O.state_from_problem(p, "U")
    Un = O.state_from_problem(p, "n")
    lin = O.linearize(sch, p["sigma"], p.get("rho_cv"), U, Un, p["dt"])
    omin = nmin if nmin else (8 if len(n) == 2 else 4)
    ref_mg = MG.Multigrid(lin, omega=0.7, nu1=nu1, nu2=nu2, nmin=omin, nu1_coarse=None if nu1c < 0 else nu1c,
                          nu2_coarse=None if nu2c < 0 else nu2c)
    x = W.random_vector(U.size, 5).reshape(U.shape)
    z_ref = ref_mg(x)
    s = P.Solver(p, U_lin=U, U_n=Un, dt=p["dt"], pc="mg", mg_omega=0.7, mg_nu1=nu1, mg_nu2=nu2, mg_nmin=nmin,
                 mg_nu1_coarse=nu1c, mg_nu2_coarse=nu2c)
    try:
        z_gpu = s.precondition(x).cpu().numpy()
    finally:
        s.close()
    e = (_rel(z_gpu, z_ref), _maxabs_by_component(z_gpu, z_ref))
    _say(f"  levels={len(ref_mg.levels)} rel={e[0]:.2e} maxabs={e[1]:.2e}")
    assert e[0] <= 1e-12 and e[1] <= 1e-11


STEP_CASES = [
    ((40, 33), BC2["mixed"], "none", "wb"),
    ((40, 33), BC2["walls"], "coupled_t", "centered"),
    ((24, 20), BC2["periodic"], "absorption", "wb"),
    ((12, 10, 9), BC3["open"], "coupled_t", "wb"),
]


@pytest.mark.parametrize("n,bc,src,fs", STEP_CASES)
def test_step_fixed_iterations_multigrid(n, bc, src, fs):
    """Exactly 2 Newton x 12 GMRES iterations with the multigrid preconditioner."""
    import paper_2011_13926_amd as P
    _say("fixed-iteration step, multigrid", n, bc, src, fs)
    p = W.random_problem(n, 11, source=src, flux_source=fs, bc=bc, dt=2.0, fmax=0.6)
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    nmin = 8 if len(n) == 2 else 4
    ref = O.implicit_step(sch, p["sigma"], p.get("rho_cv"), Un, p["dt"], restart=30, newton_max=2, fixed_iters=12,
                          pc="mg", mg_opts=dict(nmin=nmin))
    s = P.Solver(p, restart=30, newton_max=2, fixed_iters=12, pc="mg")
    try:
        U = s.to_device(Un)
        st, stats = s.implicit_step(U)
        assert stats["newton_iters"] == 2 and stats["krylov_iters"] == 24
        got = U.cpu().numpy()
        for c in range(got.shape[0]):
            assert _rel(got[c] - Un[c], ref.U[c] - Un[c]) <= 1e-10, c
    finally:
        s.close()


# the FP32 multigrid cycle of the mixed-precision solver (fused two-sweep launches with
# every staged-input and epilogue form, one-sweep launches for odd counts, FP32
# restriction and coarse levels) on ragged multi-tile grids: a fixed number of GMRES
# iterations must track the FP64 cycle's, which the oracle pins at 1e-10 above.  A
# converged solve would not show a wrong preconditioner (it only converges slower).
MIXED_FIXED_CASES = [
    ((131, 37), BC2["mixed"], "none", "wb", 12),
    ((131, 37), BC2["walls"], "absorption", "centered", 3),
    ((130, 34), BC2["periodic"], "none", "wb", 12),
]


@pytest.mark.parametrize("basis32", [False, True])
@pytest.mark.parametrize("n,bc,src,fs,nu", MIXED_FIXED_CASES)
def test_mixed_multigrid_fixed_iterations_track_fp64(n, bc, src, fs, nu, basis32):
    import paper_2011_13926_amd as P
    _say("mixed multigrid, fixed iterations", n, bc, src, fs, f"V({nu},{nu})", "basis32" if basis32 else "basis64")
    p = W.random_problem(n, 31, source=src, flux_source=fs, bc=bc, dt=2.0, fmax=0.6)
    Un = O.state_from_problem(p, "n")
    mg = dict(pc="mg", mg_nu1=nu, mg_nu2=nu, mg_nu1_coarse=1, mg_nu2_coarse=1, mg_omega=0.9)
    out = {}
    for prec in ("fp64", "mixed"):
        extra = dict(basis_fp32=basis32) if prec == "mixed" else {}
        s = P.Solver(p, restart=30, newton_max=2, fixed_iters=12, precision=prec, **mg, **extra)
        try:
            U = s.to_device(Un)
            st, stats = s.implicit_step(U)
            assert stats["newton_iters"] == 2 and stats["krylov_iters"] == 24
            out[prec] = U.cpu().numpy()
        finally:
            s.close()
    worst, worst_elem = 0.0, 0.0
    for c in range(Un.shape[0]):
        d64, d32 = out["fp64"][c] - Un[c], out["mixed"][c] - Un[c]
        err = _rel(d32, d64)
        elem = float(np.max(np.abs(d32 - d64)) / max(np.max(np.abs(d64)), 1e-300))
        worst, worst_elem = max(worst, err), max(worst_elem, elem)
        # FP32 operator and cycle inside an FP64 (or FP32-stored) Krylov basis:
        # rounding-level drift (measured at most 1.07e-7 in L2 and 8.1e-7 per element
        # over these cases, either basis)
        assert err <= 1e-6 and elem <= 1e-5, (c, err, elem)
    _say(f"  FP32 cycle against FP64, increment: relative L2 {worst:.2e}, worst element {worst_elem:.2e}")


@pytest.mark.parametrize("n,bc,src,fs", STEP_CASES)
def test_step_converged_multigrid(n, bc, src, fs):
    """Converged to 1e-12 with the multigrid preconditioner; the root agrees with the
    oracle's block-Jacobi root to 1e-10 (the preconditioner changes the path only)."""
    import paper_2011_13926_amd as P
    _say("converged step, multigrid", n, bc, src, fs)
    p = W.random_problem(n, 12, source=src, flux_source=fs, bc=bc, dt=2.0, fmax=0.6)
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    ref = O.implicit_step(sch, p["sigma"], p.get("rho_cv"), Un, p["dt"], rtol=1e-12, newton_rtol=1e-12,
                          newton_max=80)
    assert ref.converged
    s = P.Solver(p, rtol=1e-12, newton_rtol=1e-12, newton_max=80, pc="mg")
    try:
        U = s.to_device(Un)
        st, stats = s.implicit_step(U)
        got = U.cpu().numpy()
        for c in range(got.shape[0]):
            assert _rel(got[c], ref.U[c]) <= 1e-10, c
        assert _maxabs_by_component(got, ref.U) <= 1e-9
    finally:
        s.close()


@pytest.mark.parametrize("n,bc,src,fs", STEP_CASES)
@pytest.mark.parametrize("basis32", [False, True])
def test_step_mixed_precision_multigrid(n, bc, src, fs, basis32):
    """FP32 multigrid and operator inside FP64 GMRES with FP64 restarts: within 1e-8
    of the FP64 oracle."""
    import paper_2011_13926_amd as P
    _say("mixed-precision step, multigrid", n, bc, src, fs, "basis32" if basis32 else "basis64")
    p = W.random_problem(n, 12, source=src, flux_source=fs, bc=bc, dt=2.0, fmax=0.6)
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    ref = O.implicit_step(sch, p["sigma"], p.get("rho_cv"), Un, p["dt"], rtol=1e-12, newton_rtol=1e-12,
                          newton_max=80)
    s = P.Solver(p, rtol=1e-10, newton_rtol=1e-10, newton_max=80, pc="mg", precision="mixed", basis_fp32=basis32)
    try:
        U = s.to_device(Un)
        st, stats = s.implicit_step(U)
        got = U.cpu().numpy()
        err = _rel(got, ref.U)
        _say(f"  error against the FP64 oracle: {err:.2e} (newton={stats['newton_iters']} krylov={stats['krylov_iters']})")
        assert err <= 1e-8
    finally:
        s.close()


@pytest.mark.parametrize("n,bc,src,fs", [((131, 37), BC2["mixed"], "none", "wb"),
                                         ((70, 33), BC2["walls"], "coupled_t", "wb")])
def test_step_mixed_precision_multigrid_v44(n, bc, src, fs):
    """The benchmark's cycle, V(4, 4) with 2 + 2 sweeps below the finest level, in FP32
    inside FP64 GMRES: within 1e-8 of the FP64 oracle."""
    import paper_2011_13926_amd as P
    _say("mixed-precision step, multigrid V(4,4)", n, bc, src, fs)
    p = W.random_problem(n, 12, source=src, flux_source=fs, bc=bc, dt=2.0, fmax=0.6)
    sch = O.Scheme.from_problem(p)
    Un = O.state_from_problem(p, "n")
    ref = O.implicit_step(sch, p["sigma"], p.get("rho_cv"), Un, p["dt"], rtol=1e-12, newton_rtol=1e-12,
                          newton_max=80)
    assert ref.converged
    s = P.Solver(p, rtol=1e-10, newton_rtol=1e-10, newton_max=80, pc="mg", precision="mixed", mg_nu1=4, mg_nu2=4,
                 mg_nu1_coarse=2, mg_nu2_coarse=2)
    try:
        U = s.to_device(Un)
        st, stats = s.implicit_step(U)
        got = U.cpu().numpy()
        err = _rel(got, ref.U)
        _say(f"  error against the FP64 oracle: {err:.2e} (newton={stats['newton_iters']} krylov={stats['krylov_iters']})")
        assert err <= 1e-8
    finally:
        s.close()


def test_multigrid_cuts_voronoi_iterations():
    """First Newton system of a 128^2 Voronoi field (8 sites, dt = 100): GMRES(30)
    to 1e-8 with one V(1,1) cycle per iteration needs at most a fifth of the
    block-Jacobi iterations, and both solutions satisfy the tolerance."""
    import paper_2011_13926_amd as P
    p = W.voronoi_opacity(n=(128, 128), nsites=8, seed=1000)
    U = O.state_from_problem(p)
    sch = O.Scheme.from_problem(p)
    lin = O.linearize(sch, p["sigma"], None, U, U, p["dt"])
    b = -O.residual(lin)
    its = {}
    for pc in ["bj", "mg"]:
        s = P.Solver(p, U_lin=U, U_n=U, dt=p["dt"], pc=pc, rtol=1e-8, max_iters=20000)
        try:
            x, st, stats = s.solve_linear(b)
            its[pc] = stats["krylov_iters"]
            r = b - O.apply_operator(lin, x.cpu().numpy())
            assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)
        finally:
            s.close()
    _say(f"  krylov iterations: block-Jacobi {its['bj']}, multigrid {its['mg']}")
    assert its["mg"] * 5 <= its["bj"]
