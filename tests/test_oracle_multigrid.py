"""Pins of the oracle's aggregation multigrid (oracle/m1_multigrid.py).  CPU only.

The multigrid is checked against what its definition fixes, by routes that do
not reuse its own code: the assembled operator against the matrix-free oracle
operator; the block diagonal against the oracle's 'diag' operator mode; the
Galerkin coarse operator against P^T A P evaluated matrix-free; the two-level
coarse-grid correction is a projector annihilated by P^T A; a grid at or below
the coarsest size is solved exactly; the cycle is linear; and as the GMRES
preconditioner it reaches the dense solution."""
import numpy as np
import pytest

import workloads as W
from oracle import m1_multigrid as MG
from oracle import m1_oracle as O


def _lin(p):
    sch = O.Scheme.from_problem(p)
    U = O.state_from_problem(p, "U")
    Un = O.state_from_problem(p, "n")
    return O.linearize(sch, p["sigma"], p.get("rho_cv"), U, Un, p["dt"])


ASM_CASES = [
    ((7, 5), ("periodic",) * 4, "none", "wb"),
    ((6, 4), ("outflow", "reflect", "dirichlet", "outflow"), "coupled_t", "centered"),
    ((5, 2), ("dirichlet", "dirichlet", "periodic", "periodic"), "absorption", "wb"),
    ((1, 4), ("periodic", "periodic", "outflow", "reflect"), "none", "centered"),
    ((4, 3, 5), ("outflow", "dirichlet", "reflect", "outflow", "periodic", "periodic"), "coupled_t", "wb"),
    ((3, 3, 2), ("periodic",) * 6, "absorption", "centered"),
]


@pytest.mark.parametrize("n,bc,src,fs", ASM_CASES)
def test_assembled_operator_equals_matrix_free(n, bc, src, fs):
    p = W.random_problem(n, 11, source=src, flux_source=fs, bc=bc)
    lin = _lin(p)
    A = MG.assemble_sparse(lin)
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal(A.shape[0])
        y = O.apply_operator(lin, x)
        assert np.linalg.norm(A @ x - y) <= 1e-14 * np.linalg.norm(y)
    # and against the dense column-by-column assembly
    assert np.abs(A.toarray() - O.assemble_dense(lin)).max() <= 1e-14 * np.abs(A.data).max()


@pytest.mark.parametrize("n,bc,src,fs", ASM_CASES[:3] + ASM_CASES[4:5])
def test_block_diagonal_equals_diag_mode(n, bc, src, fs):
    p = W.random_problem(n, 12, source=src, flux_source=fs, bc=bc)
    lin = _lin(p)
    A = MG.assemble_sparse(lin)
    N = int(np.prod(lin.sch.shape))
    D = MG.block_diagonal(A, lin.sch.nu, N)
    ref = O.diagonal_blocks(lin)
    assert np.abs(D - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("n,bc", [((12, 10), ("periodic",) * 4),
                                  ((11, 9), ("outflow", "reflect", "dirichlet", "outflow")),
                                  ((10, 9, 12), ("outflow", "dirichlet", "reflect", "outflow", "periodic", "periodic"))])
def test_galerkin_operator_is_restricted_matrix_free_product(n, bc):
    p = W.random_problem(n, 13, source="absorption", bc=bc)
    lin = _lin(p)
    m = MG.Multigrid(lin)
    lev0, lev1 = m.levels[0], m.levels[1]
    rng = np.random.default_rng(2)
    xc = rng.standard_normal(lev1["A"].shape[0])
    ref = lev0["P"].T @ O.apply_operator(lin, lev0["P"] @ xc)
    assert np.linalg.norm(lev1["A"] @ xc - ref) <= 1e-13 * np.linalg.norm(ref)
    # aggregates: every fine cell in exactly one, each aggregate 1..2^ndim cells
    Pc = lev0["P"][: lev0["N"], : lev1["N"]]
    assert np.all(np.asarray(Pc.sum(axis=1)).ravel() == 1)
    sizes = np.asarray(Pc.sum(axis=0)).ravel()
    assert sizes.min() >= 1 and sizes.max() == 2 ** len(n)


def test_two_level_correction_is_a_projector():
    # nu1 = nu2 = 0 with one coarse level solved exactly: M^{-1} = P A_c^{-1} P^T,
    # E = I - M^{-1} A is the A-coarse-grid correction: E^2 = E and P^T A E = 0
    p = W.random_problem((12, 10), 14, source="none", bc=("outflow", "outflow", "dirichlet", "reflect"), dt=2.0)
    lin = _lin(p)
    m = MG.Multigrid(lin, nu1=0, nu2=0)
    assert len(m.levels) == 2
    A = O.assemble_dense(lin)
    n = A.shape[0]
    Minv = np.stack([m(e) for e in np.eye(n)], axis=1)
    E = np.eye(n) - Minv @ A
    assert np.abs(E @ E - E).max() <= 1e-10
    PtAE = m.levels[0]["P"].T @ (A @ E)
    assert np.abs(PtAE).max() <= 1e-10 * np.abs(A).max()
    # the correction is not trivial: rank of I - E is the coarse dimension
    assert np.linalg.matrix_rank(np.eye(n) - E, tol=1e-8) == m.levels[1]["A"].shape[0]


@pytest.mark.parametrize("n", [(8, 8), (5, 7), (4, 4, 3)])
def test_coarsest_size_grid_is_solved_exactly(n):
    p = W.random_problem(n, 15, source="coupled_t", bc=("outflow",) * 2 * len(n))
    lin = _lin(p)
    m = MG.Multigrid(lin, nmin=8)
    assert len(m.levels) == 1
    b = np.random.default_rng(3).standard_normal(m.levels[0]["A"].shape[0])
    x = np.linalg.solve(O.assemble_dense(lin), b)
    assert np.linalg.norm(m(b) - x) <= 1e-11 * np.linalg.norm(x)


def test_cycle_is_linear():
    p = W.random_problem((20, 18), 16, source="absorption", bc=("periodic",) * 4)
    lin = _lin(p)
    m = MG.Multigrid(lin, nu1=2, nu2=1)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, m.levels[0]["A"].shape[0]))
    lhs = m(2.5 * u - 0.75 * v)
    rhs = 2.5 * m(u) - 0.75 * m(v)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_shift_enters_every_level():
    p = W.random_problem((12, 12), 17, bc=("periodic",) * 4)
    lin = _lin(p)
    N = 144
    shift = np.full((3, N), 0.5)
    m = MG.Multigrid(lin, shift=shift)
    A0 = MG.assemble_sparse(lin)
    diff = (m.levels[0]["A"] - A0).toarray()
    assert np.allclose(diff, 0.5 * np.eye(3 * N), atol=1e-15)
    # the coarse shift is the aggregate size times the fine one
    Ac0 = MG.Multigrid(lin).levels[1]["A"]
    dc = (m.levels[1]["A"] - Ac0).toarray()
    assert np.allclose(dc, 2.0 * np.eye(dc.shape[0]), atol=1e-13)


def test_gmres_with_multigrid_reaches_the_dense_solution_in_fewer_iterations():
    p = W.voronoi_opacity(n=(32, 32), nsites=4, seed=3, dt=30.0)
    sch = O.Scheme.from_problem(p)
    U = O.state_from_problem(p)
    lin = O.linearize(sch, p["sigma"], None, U, U, p["dt"])
    b = -O.residual(lin).reshape(-1)
    x = np.linalg.solve(O.assemble_dense(lin), b)
    mg = MG.Multigrid(lin, nu1=1, nu2=1)
    r_mg = O.gmres(lambda v: O.apply_operator(lin, v), mg, b, rtol=1e-12, max_iters=5000)
    r_bj = O.gmres(lambda v: O.apply_operator(lin, v), O.BlockJacobi(lin), b, rtol=1e-12, max_iters=5000)
    assert r_mg.converged and r_bj.converged
    assert np.linalg.norm(r_mg.x - x) <= 1e-8 * np.linalg.norm(x)
    assert r_mg.iters * 3 <= r_bj.iters
