"""CPU FP64 oracle of the aggregation multigrid preconditioner.

TEST INFRASTRUCTURE ONLY: tests, the smoke entry and the benchmark's CPU
baseline may import it; the product path never does and shares no code with it.

The method's implicit systems were solved with Trilinos preconditioners; the
best of them was algebraic multigrid, about ten Krylov iterations per solve
against about 250 for damped Jacobi (Sect. 4.1-4.2, weak-scaling study).  The
preconditioner here is a geometric-aggregation multigrid on the Cartesian
grid, written from the textbook definition of a multigrid V-cycle:

* levels 0 (the grid of the step), 1, ...: level l+1 has one cell per 2 x 2
  (x 2) aggregate of level-l cells (the last aggregate along an odd axis holds
  one layer), until every extent is <= nmin;
* prolongation P_l: piecewise constant, every unknown of a cell takes the
  same unknown of its aggregate; restriction P_l^T: the sum over the aggregate;
* coarse operators A_{l+1} = P_l^T A_l P_l (Galerkin products of the
  assembled matrices);
* smoother: damped block-Jacobi, x <- x + omega D_l^{-1} (b - A_l x), with D_l
  the n_u x n_u diagonal block of every cell of A_l;
* V(nu1, nu2) cycle from x = 0 (optionally other sweep counts below the finest
  level); the coarsest level is solved exactly (LU).

The cycle is a fixed linear map of its input, so it serves as the right
preconditioner of GMRES unchanged.  Vectors are component-major, index
comp * N + cell, like the rest of the oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import m1_oracle as O


def _colour_period(n, periodic):
    """Smallest colouring period along one axis such that two cells of the same
    colour never share a stencil neighbour (distance >= 3, also across a wrap)."""
    if not periodic:
        return 3
    for p in range(3, n + 1):
        if n % p == 0:
            return p
    return n


def assemble_sparse(lin, shift=None):
    """The linearised operator A (plus diag(shift) if given) as a CSR matrix.

    Probing: the oracle's matrix-free operator is applied to sums of unit
    vectors whose cells are far enough apart (coloured by position modulo a
    period >= 3 per axis) that every output entry comes from exactly one probed
    cell: the one of that colour within one cell along every axis.
    """
    sch = lin.sch
    nu, shape, nd = sch.nu, sch.shape, sch.ndim
    N = int(np.prod(shape))
    per_ax = []
    for ax in range(nd):
        d = nd - 1 - ax
        per_ax.append(_colour_period(shape[ax], "periodic" in (sch.bc[2 * d], sch.bc[2 * d + 1])))
    idx = np.indices(shape)
    rows, cols, vals = [], [], []
    for col in np.ndindex(*per_ax):
        mask = np.ones(shape, bool)
        for ax in range(nd):
            mask &= (idx[ax] % per_ax[ax]) == col[ax]
        # source cell of every output cell: the probed cell within one step per axis
        src = np.full(shape, -1, dtype=np.int64)
        for off in np.ndindex(*([3] * nd)):
            nb = []
            ok = np.ones(shape, bool)
            for ax in range(nd):
                d = nd - 1 - ax
                j = idx[ax] + (off[ax] - 1)
                if "periodic" in (sch.bc[2 * d], sch.bc[2 * d + 1]):
                    j = j % shape[ax]
                else:
                    ok &= (j >= 0) & (j < shape[ax])
                    j = np.clip(j, 0, shape[ax] - 1)
                nb.append(j)
            hit = ok & mask[tuple(nb)]
            lin_idx = np.ravel_multi_index(tuple(nb), shape)
            src = np.where(hit, lin_idx, src)
        for k in range(nu):
            x = np.zeros((nu,) + shape)
            x[k][mask] = 1.0
            y = O.operator(lin, x, "linear").reshape(nu, N)
            rc, rcell = np.nonzero(y)
            scell = src.reshape(-1)[rcell]
            keep = scell >= 0
            rows.append(rc[keep] * N + rcell[keep])
            cols.append(k * N + scell[keep])
            vals.append(y[rc[keep], rcell[keep]])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nu * N, nu * N))
    if shift is not None:
        A = (A + sp.diags(np.asarray(shift, float).reshape(-1))).tocsr()
    return A


def aggregation(shape):
    """Piecewise-constant prolongation of one unknown from the aggregate grid to
    the grid `shape` (numpy order): an (N x Nc) 0/1 matrix, and the coarse shape."""
    nd = len(shape)
    cshape = tuple((s + 1) // 2 for s in shape)
    idx = np.indices(shape)
    parent = np.ravel_multi_index(tuple(idx[a] // 2 for a in range(nd)), cshape).reshape(-1)
    N = int(np.prod(shape))
    return sp.csr_matrix((np.ones(N), (np.arange(N), parent)), shape=(N, int(np.prod(cshape)))), cshape


def block_diagonal(A, nu, N):
    """The n_u x n_u diagonal block of every cell of a component-major matrix, (N, nu, nu)."""
    D = np.zeros((N, nu, nu))
    A = A.tocsr()
    cells = np.arange(N)
    for r in range(nu):
        for c in range(nu):
            D[:, r, c] = np.asarray(A[r * N + cells, c * N + cells]).reshape(-1)
    return D


class Multigrid:
    """z = M^{-1} r, one V(nu1, nu2) cycle of aggregation multigrid on A(lin) (+ diag(shift))."""

    def __init__(self, lin, *, omega=0.7, nu1=1, nu2=1, nmin=8, shift=None, A=None, nu1_coarse=None,
                 nu2_coarse=None):
        sch = lin.sch
        self.nu = nu = sch.nu
        self.omega, self.nu1, self.nu2, self.nmin = float(omega), int(nu1), int(nu2), int(nmin)
        # sweeps on the levels below the finest (default: the same as on the finest)
        self.nu1c = self.nu1 if nu1_coarse is None else int(nu1_coarse)
        self.nu2c = self.nu2 if nu2_coarse is None else int(nu2_coarse)
        A = assemble_sparse(lin, shift) if A is None else A.tocsr()
        shape = tuple(sch.shape)
        self.levels = []
        while True:
            N = int(np.prod(shape))
            lev = dict(A=A, shape=shape, N=N)
            self.levels.append(lev)
            if max(shape) <= self.nmin:
                lev["lu"] = spla.splu(A.tocsc())
                break
            Dinv = np.linalg.inv(block_diagonal(A, nu, N))
            lev["Dinv"] = Dinv
            Pc, cshape = aggregation(shape)
            P = sp.kron(sp.identity(nu), Pc, format="csr")   # component-major unknowns
            lev["P"] = P
            A = (P.T @ A @ P).tocsr()
            shape = cshape

    def smooth(self, lev, x, b):
        r = (b - lev["A"] @ x).reshape(self.nu, lev["N"]).T              # (N, nu)
        return x + self.omega * np.einsum("nij,nj->ni", lev["Dinv"], r).T.reshape(-1)

    def vcycle(self, l, b):
        lev = self.levels[l]
        if "lu" in lev:
            return lev["lu"].solve(b)
        nu1, nu2 = (self.nu1, self.nu2) if l == 0 else (self.nu1c, self.nu2c)
        x = np.zeros_like(b)
        for _ in range(nu1):
            x = self.smooth(lev, x, b)
        rc = lev["P"].T @ (b - lev["A"] @ x)
        x = x + lev["P"] @ self.vcycle(l + 1, rc)
        for _ in range(nu2):
            x = self.smooth(lev, x, b)
        return x

    def __call__(self, r):
        r = np.asarray(r, float)
        return self.vcycle(0, r.reshape(-1)).reshape(r.shape)
