"""The allocation-free entry point m1_time_steps_noalloc against the context
entry points m1_explicit_step / m1_semi_implicit_step, called through the C ABI.

Both run the same step kernels on the same inputs, so the results must agree
bit for bit (a stricter bar than the oracle tolerances of the step tests).
Two calls in a row on one GPU, the second on a smaller grid (the static work
array keeps the first call's contents); the size limit and argument checks are
rejected on the host."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(p):
    comps = [p["En"]] + [p["Fn"][m] for m in range(p["ndim"])]
    if p["source"] == "coupled_t":
        comps.append(p["Tn"])
    return np.stack(comps)


def _noalloc(P, s, U, dt, nsteps, semi):
    """Call m1_time_steps_noalloc with the config and fields of Solver s (its
    device copies of sigma, rho_cv and the boundary planes) on device tensor U."""
    stats = P.M1Stats()
    st = P.m1_time_steps_noalloc(ctypes.byref(s.cfg), ctypes.byref(s.fields),
                                 ctypes.byref(P.state_struct(U, s.ndim, s.coupled)), float(dt), int(nsteps),
                                 int(semi), ctypes.c_void_p(s.stream.cuda_stream), ctypes.byref(stats))
    return st, stats.as_dict()


CASES = [
    # (grid, seed, source, bc, semi, nsteps) -- the second case is the smaller one
    ((72, 40), 7, "coupled_t", ("outflow", "reflect", "dirichlet", "outflow"), 1, 3),
    ((10, 9, 7), 8, "absorption", ("outflow", "dirichlet", "reflect", "outflow", "periodic", "periodic"), 0, 2),
]


def test_noalloc_matches_context_steps_two_calls():
    import torch
    import paper_2011_13926_amd as P
    for (n, seed, source, bc, semi, nsteps) in CASES:
        _say("noalloc case", n, seed, source, "semi" if semi else "explicit", nsteps)
        p = W.random_problem(n, seed, source=source, flux_source="centered", bc=bc, dt=0.2, fmax=0.6)
        Un = _state(p)
        s = P.Solver(p)
        try:
            U_ref = s.to_device(Un)
            step = s.semi_implicit_step if semi else s.explicit_step
            st, st_ref = step(U_ref, dt=p["dt"], nsteps=nsteps)
            assert st == P.M1_OK
            U = s.to_device(Un)
            st, stats = _noalloc(P, s, U, p["dt"], nsteps, semi)
            torch.cuda.synchronize()
            assert st == P.M1_OK, P.m1_last_error(None).decode()
            assert torch.equal(U, U_ref), float((U - U_ref).abs().max())
            assert not torch.equal(U, s.to_device(Un))
            assert stats["cells_f_gt_1"] == st_ref["cells_f_gt_1"]
            assert stats["newton_iters"] == 0 and stats["krylov_iters"] == 0
        finally:
            s.close()


def test_noalloc_rejects_on_host():
    import torch
    import paper_2011_13926_amd as P
    p = W.random_problem((16, 12), 3, flux_source="centered", dt=0.2)
    s = P.Solver(p)
    try:
        U = s.to_device(_state(p))
        before = U.clone()
        # well-balanced source with the semi-implicit step
        cfg_wb = P.make_config(dict(p, flux_source="wb"))
        stats = P.M1Stats()
        st = P.m1_time_steps_noalloc(ctypes.byref(cfg_wb), ctypes.byref(s.fields),
                                     ctypes.byref(P.state_struct(U, 2, False)), 0.2, 1, 1, None, ctypes.byref(stats))
        assert st == P.M1_ERR_INVALID_ARG and "centred" in P.m1_last_error(None).decode()
        # nsteps and dt
        for dt, ns, semi in [(0.2, 0, 1), (-1.0, 1, 1), (0.2, 1, 2)]:
            st, _ = _noalloc(P, s, U, dt, ns, semi)
            assert st == P.M1_ERR_INVALID_ARG
        # grid above the limit (checked before any device work; U is not read)
        big = P.make_config(dict(p, n=(4096, 2048)))
        st = P.m1_time_steps_noalloc(ctypes.byref(big), ctypes.byref(s.fields),
                                     ctypes.byref(P.state_struct(U, 2, False)), 0.2, 1, 1, None, ctypes.byref(stats))
        assert st == P.M1_ERR_INVALID_ARG and "limit" in P.m1_last_error(None).decode()
        torch.cuda.synchronize()
        assert torch.equal(U, before)
        # non-positive energy in the input leaves U unchanged
        U[0, 3, 3] = -1.0
        before = U.clone()
        st, _ = _noalloc(P, s, U, 0.2, 1, 1)
        assert st == P.M1_ERR_INVALID_ARG
        torch.cuda.synchronize()
        assert torch.equal(U, before)
    finally:
        s.close()
