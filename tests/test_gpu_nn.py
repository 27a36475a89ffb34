"""GPU tests of the learned preconditioner: the BF16-MFMA network forward and
gradients against the FP64 oracle (with BF16 rounding emulated at the same
points), training progress, and flexible GMRES with the network inside."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import m1_oracle as O
from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu
CH = [32, 48, 64, 64]
CIN, COUT = 9, 3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _random_net_params(seed, cin=CIN, ch=CH, cout=COUT):
    rng = np.random.default_rng(seed)
    params = N.init_params(cin, ch, cout, seed=seed, head_scale=1.0)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape) * 0.05
    # the GPU stores 3x3 weights in BF16 and everything else in FP32
    for name, kind, ci, co in N.layer_specs(cin, ch, cout):
        if kind == "conv3":
            params[name + ".w"] = N.bf16_round(params[name + ".w"])
    flat = N.flatten_params(params, cin, ch, cout).astype(np.float32)
    return N.unflatten_params(flat.astype(np.float64), cin, ch, cout), flat


def _oracle(params, x, t, ch, rnd=N.bf16_round):
    """Forward output, loss and per-tensor gradients of the oracle with BF16 rounding
    (or the given rounding) of the input and of every stored activation."""
    y, acts = N.forward(params, x, ch, keep=True, act_round=rnd)
    loss, gy = N.relative_loss(y, t)
    return y, loss, N.backward(params, acts, gy, ch)


def _rounding_spread(params, x, t, ch, trials=3, eps=3e-7):
    """How far the oracle moves from itself when each value is perturbed by a relative
    eps (about an FP32 accumulation error) before its BF16 rounding.  A perturbation
    this small only matters where a value sits next to a BF16 rounding boundary and
    flips to the neighbouring BF16 number; in a deep network such a flip in a
    coarse-level activation reaches most of the output.  The GPU accumulates in FP32
    in another order than the oracle, so it takes such flips too: its distance from
    the oracle is bounded by this spread, not by the FP32 accumulation error alone.
    Returns the forward spread and the per-tensor gradient spreads."""
    y0, _, g0 = _oracle(params, x, t, ch)
    fwd, grad = 0.0, {}
    for k in range(trials):
        rng = np.random.default_rng(1000 + k)
        rnd = lambda v: N.bf16_round(v * (1.0 + eps * rng.standard_normal(np.shape(v))))
        y, _, g = _oracle(params, x, t, ch, rnd)
        fwd = max(fwd, _rel(y, y0))
        for name in g0:
            grad[name] = max(grad.get(name, 0.0), _rel(g[name], g0[name]))
    return fwd, grad


# The weight gradients contract the output gradient rounded to BF16 (the MFMA's operand
# type), which the oracle keeps in FP64: each element carries a relative error up to
# 2^-9 (2^-9/sqrt(3) RMS), so a tensor whose sum over pixels cancels can be off by
# about 1e-3.  Tolerances add 4e-3 for this on top of the rounding-flip spread.
BF16_GRAD_TOL = 4e-3


def _gpu_forward_backward(params_flat, x, t, cin, ch, cout):
    import paper_2011_13926_amd as P
    net = P.Net(cin, cout, ch, Hmax=x.shape[0], Wmax=x.shape[1])
    try:
        net.set_params(params_flat)
        assert np.array_equal(net.get_params(), params_flat)
        y = net.forward(x).cpu().numpy()
        loss = net.backward(x, t)
        g = net.get_grads()
    finally:
        net.close()
    return y, loss, g


def _check_grads(g, gref, cin, ch, cout, bound):
    """Compare the flat GPU gradient with the oracle's per tensor; bound(name) gives
    each tensor's relative L2 tolerance.  Returns the worst error over the bound."""
    k = 0
    worst = 0.0
    for name, kind, ci, co in N.layer_specs(cin, ch, cout):
        for part in ("w", "b"):
            key = f"{name}.{part}"
            ref = gref[key].ravel()
            got = g[k:k + ref.size]
            k += ref.size
            err = _rel(got, ref)
            worst = max(worst, err / bound(key))
            assert err <= bound(key), (key, err, bound(key))
    assert k == g.size
    return worst


def test_mfma_network_forward_matches_oracle():
    import paper_2011_13926_amd as P
    _say("nn forward 32x40")
    params, flat = _random_net_params(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((32, 40, CIN)).astype(np.float32)
    net = P.Net(CIN, COUT, CH, Hmax=32, Wmax=40)
    try:
        net.set_params(flat)
        assert np.array_equal(net.get_params(), flat)
        y = net.forward(x).cpu().numpy()
    finally:
        net.close()
    ref = N.forward(params, x.astype(np.float64), CH, act_round=N.bf16_round)
    spread, _ = _rounding_spread(params, x.astype(np.float64), np.ones((32, 40, COUT)), CH)
    err = _rel(y, ref)
    _say(f"  forward relative L2 vs oracle (BF16 emulated): {err:.2e}, oracle rounding spread {spread:.2e}")
    # both sides round the same activations to BF16; what remains is the FP32
    # accumulation order and the rounding-boundary flips it causes
    assert err <= 2 * spread + 1e-4
    assert np.max(np.abs(y - ref)) <= 1e-2 * np.max(np.abs(ref))


# four levels: 32x32 takes one pixel chunk per layer; 32x40 has rows of 20, 10 and 5
# pixels at the lower levels (the weight-gradient kernel for widths that are not a
# multiple of 8); 72x64 has two pixel chunks at the top level, the second one partial
@pytest.mark.parametrize("H,Wd", [(32, 32), (32, 40), (72, 64)])
def test_mfma_network_gradients_match_oracle(H, Wd):
    _say(f"nn gradients {H}x{Wd}")
    params, flat = _random_net_params(3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((H, Wd, CIN)).astype(np.float32)
    t = rng.standard_normal((H, Wd, COUT)).astype(np.float32)
    _, loss, g = _gpu_forward_backward(flat, x, t, CIN, CH, COUT)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    _, lref, gref = _oracle(params, x64, t64, CH)
    _, spread = _rounding_spread(params, x64, t64, CH)
    assert loss == pytest.approx(lref, rel=1e-3)
    worst = _check_grads(g, gref, CIN, CH, COUT, lambda k: 2 * spread[k] + BF16_GRAD_TOL)
    _say(f"  worst per-tensor gradient error / tolerance: {worst:.2f}")


# one level (no pooling, so no coarse-level flips): the oracle's rounding spread stays
# near 1e-4 and the gradients are held to the BF16 operand rounding.  Odd 33x37 takes the weight-gradient
# kernel for any width; 40x24 and 72x64 the one for widths in whole 8-pixel groups, the
# latter over two pixel chunks; 40 input channels pad to 48 and 80 output channels
# span two 64-channel blocks, both partial; 6 outputs take the head gradient kernel
# for more than 4 output channels.  The convolution narrows its output-channel tile on
# small images; 64x512 and 64x1024 are large enough to keep the 32-, 48- and 64-channel
# tiles (forward and input gradient).
@pytest.mark.parametrize("cin,ch,cout,H,Wd", [(9, [32], 3, 33, 37), (40, [48], 3, 40, 24),
                                              (40, [80], 3, 72, 64), (64, [64], 6, 16, 8),
                                              (9, [32], 3, 64, 512), (9, [48], 3, 64, 1024),
                                              (64, [64], 3, 64, 1024)])
def test_single_level_network_gradients_match_oracle(cin, ch, cout, H, Wd):
    _say(f"nn one-level gradients cin {cin} ch {ch} cout {cout} {H}x{Wd}")
    params, flat = _random_net_params(11, cin, ch, cout)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((H, Wd, cin)).astype(np.float32)
    t = rng.standard_normal((H, Wd, cout)).astype(np.float32)
    y, loss, g = _gpu_forward_backward(flat, x, t, cin, ch, cout)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    yref, lref, gref = _oracle(params, x64, t64, ch)
    fspread, spread = _rounding_spread(params, x64, t64, ch)
    _say(f"  forward {_rel(y, yref):.2e}, oracle rounding spread {fspread:.2e}")
    assert _rel(y, yref) <= 2 * fspread + 1e-4
    assert loss == pytest.approx(lref, rel=1e-4)
    worst = _check_grads(g, gref, cin, ch, cout, lambda k: 2 * spread[k] + BF16_GRAD_TOL)
    _say(f"  worst per-tensor gradient error / tolerance: {worst:.2f}")


# two levels at 64x1024: the top level keeps its 32-, 48- and 64-channel output tiles
# (256 pixel blocks), so the pooling written by the second convolution's epilogue is
# checked on the tile widths the 512^2 network uses
@pytest.mark.parametrize("ch", [[32, 48], [48, 64], [64, 64]])
def test_two_level_network_wide_tiles_match_oracle(ch):
    _say(f"nn two-level {ch} 64x1024")
    params, flat = _random_net_params(21, CIN, ch)
    rng = np.random.default_rng(22)
    x = rng.standard_normal((64, 1024, CIN)).astype(np.float32)
    t = rng.standard_normal((64, 1024, COUT)).astype(np.float32)
    y, loss, g = _gpu_forward_backward(flat, x, t, CIN, ch, COUT)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    yref, lref, gref = _oracle(params, x64, t64, ch)
    fspread, spread = _rounding_spread(params, x64, t64, ch)
    _say(f"  forward {_rel(y, yref):.2e}, oracle rounding spread {fspread:.2e}")
    assert _rel(y, yref) <= 2 * fspread + 1e-4
    assert loss == pytest.approx(lref, rel=1e-3)
    worst = _check_grads(g, gref, CIN, ch, COUT, lambda k: 2 * spread[k] + BF16_GRAD_TOL)
    _say(f"  worst per-tensor gradient error / tolerance: {worst:.2f}")


def test_adam_step_matches_oracle():
    """Two Adam steps on the GPU (FP32 master weights and moments) against the oracle's
    Adam in FP64 fed with the same gradients."""
    import paper_2011_13926_amd as P
    _say("nn adam 16x16")
    params, flat = _random_net_params(9)
    rng = np.random.default_rng(10)
    net = P.Net(CIN, COUT, CH, Hmax=16, Wmax=16)
    ref = N.unflatten_params(flat.astype(np.float64), CIN, CH, COUT)
    state = {}
    try:
        net.set_params(flat)
        for step, lr in enumerate((1e-2, 3e-3)):
            x = rng.standard_normal((16, 16, CIN)).astype(np.float32)
            t = rng.standard_normal((16, 16, COUT)).astype(np.float32)
            before = net.get_params().astype(np.float64)
            net.backward(x, t)
            g = N.unflatten_params(net.get_grads().astype(np.float64), CIN, CH, COUT)
            net.adam_step(lr)
            got = net.get_params().astype(np.float64)
            ref = N.adam_step(ref, g, state, lr=lr)
            want = N.flatten_params(ref, CIN, CH, COUT)
            e_par = _rel(got, want)
            e_upd = _rel(got - before, want - before)
            _say(f"  step {step}: params {e_par:.2e}, update {e_upd:.2e}")
            assert e_par <= 1e-6 and e_upd <= 1e-4
    finally:
        net.close()


def test_library_initial_weights():
    """m1nn_init_params: deterministic in the seed, zero biases, He-normal spread per layer."""
    import paper_2011_13926_amd as P
    _say("nn init")
    net = P.Net(CIN, COUT, CH, Hmax=16, Wmax=16)
    try:
        net.init_params(seed=5, head_scale=0.1)
        a = net.get_params()
        net.init_params(seed=5, head_scale=0.1)
        b = net.get_params()
        net.init_params(seed=6, head_scale=0.1)
        c = net.get_params()
    finally:
        net.close()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    prm = N.unflatten_params(a.astype(np.float64), CIN, CH, COUT)
    for name, kind, ci, co in N.layer_specs(CIN, CH, COUT):
        w = prm[name + ".w"]
        assert np.all(prm[name + ".b"] == 0.0)
        sd = np.sqrt(2.0 / (9 * ci)) if kind == "conv3" else 0.1 / np.sqrt(ci)
        assert abs(w.mean()) <= 5 * sd / np.sqrt(w.size)
        assert abs(w.std() / sd - 1.0) <= 6 / np.sqrt(w.size) + 0.02, name


def test_training_reduces_the_loss():
    import paper_2011_13926_amd as P
    _say("nn training")
    rng = np.random.default_rng(5)
    x = rng.standard_normal((32, 32, CIN)).astype(np.float32)
    t = (0.5 * x[:, :, :3] + 0.1).astype(np.float32)
    net = P.Net(CIN, COUT, CH, Hmax=32, Wmax=32)
    try:
        params = N.init_params(CIN, CH, COUT, seed=6)
        net.set_params(N.flatten_params(params, CIN, CH, COUT).astype(np.float32))
        losses = [net.train_step(x, t, 3e-3) for _ in range(40)]
    finally:
        net.close()
    _say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.5 * losses[0]


def test_learned_fgmres_converges_and_matches_block_jacobi():
    import paper_2011_13926_amd as P
    _say("learned FGMRES 64x64")
    p = W.random_problem((64, 64), 21, bc=("outflow", "reflect", "dirichlet", "outflow"), dt=5.0, fmax=0.5)
    U = O.state_from_problem(p, "U")
    Un = O.state_from_problem(p, "n")
    net = P.Net(CIN, COUT, CH, Hmax=64, Wmax=64)
    params = N.init_params(CIN, CH, COUT, seed=7, head_scale=0.05)
    net.set_params(N.flatten_params(params, CIN, CH, COUT).astype(np.float32))
    s_bj = P.Solver(p, U_lin=U, U_n=Un, rtol=1e-11)
    s_nn = P.Solver(p, U_lin=U, U_n=Un, rtol=1e-11, pc="learned")
    try:
        s_nn.set_network(net)
        b = s_bj.residual()
        x_bj, st1, stats_bj = s_bj.solve_linear(b)
        x_nn, st2, stats_nn = s_nn.solve_linear(b)
        _say(f"  BJ {stats_bj['krylov_iters']} it, learned {stats_nn['krylov_iters']} it, fell_back={stats_nn['fell_back']}")
        assert _rel(x_nn.cpu().numpy(), x_bj.cpu().numpy()) <= 1e-8
        # an implicit step with the learned preconditioner agrees with the oracle
        s_nn2 = P.Solver(p, rtol=1e-11, newton_rtol=1e-11, pc="learned")
        s_nn2.set_network(net)
        Ud = s_nn2.to_device(Un)
        st, stats = s_nn2.implicit_step(Ud)
        ref = O.implicit_step(O.Scheme.from_problem(p), p["sigma"], None, Un, p["dt"], rtol=1e-12, newton_rtol=1e-12)
        assert _rel(Ud.cpu().numpy(), ref.U) <= 1e-8
        s_nn2.close()
    finally:
        s_bj.close()
        s_nn.close()
        net.close()


def test_features_and_target_layout():
    """Features and targets computed on the GPU agree with their definitions
    evaluated with the oracle's block-Jacobi."""
    import paper_2011_13926_amd as P
    _say("features/target")
    p = W.random_problem((16, 24), 8, dt=3.0, fmax=0.5)
    U = O.state_from_problem(p, "U")
    Un = O.state_from_problem(p, "n")
    lin = O.linearize(O.Scheme.from_problem(p), p["sigma"], None, U, Un, p["dt"])
    M = O.BlockJacobi(lin)
    r = W.random_vector(U.size, 1).reshape(U.shape)
    e = W.random_vector(U.size, 2).reshape(U.shape)
    s = P.Solver(p, U_lin=U, U_n=Un)
    try:
        f = s.nn_features(r).cpu().numpy()
        t = s.nn_target(r, e).cpu().numpy()
    finally:
        s.close()
    N_ = 16 * 24
    sc = np.sqrt(3 * N_) / np.linalg.norm(r)
    z = M(r)
    # the diagonal block applied to e (target: s (M e - r)/|r|)
    Me = np.einsum("nij,nj->ni", M.blocks, e.reshape(3, -1).T).T.reshape(e.shape)
    for k in range(3):
        assert np.allclose(f[:, :, k], sc * r[k], rtol=1e-6, atol=1e-6)
        assert np.allclose(f[:, :, 3 + k], sc * z[k], rtol=1e-5, atol=1e-5)
        assert np.allclose(t[:, :, k], sc * (Me[k] - r[k]), rtol=1e-5, atol=1e-5)
    assert np.allclose(f[:, :, 6], np.log10(1 + p["sigma"] * p["dt"]) / 4, rtol=1e-6)
    fx = U[1] / U[0]
    assert np.allclose(f[:, :, 7], fx, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("head_scale", [0.0])
def test_flexible_gmres_with_a_silent_network_matches_block_jacobi(head_scale):
    """With every weight zero the network's correction is exactly zero and the learned
    preconditioner is block-Jacobi: flexible GMRES (standard Arnoldi order, the
    preconditioner applied to the orthonormal basis vector) must take the
    block-Jacobi iteration count and reach the same solution."""
    import paper_2011_13926_amd as P
    import workloads as W
    p = W.diffusive_lognormal(n=(128, 128), seed=1000)
    U0 = np.stack([p["E"], p["F"][0], p["F"][1]])
    net = P.Net(9, 3, (32, 48, 64, 64), Hmax=128, Wmax=128)
    s_bj = P.Solver(p, U_lin=U0, U_n=U0, rtol=1e-8, max_iters=5000)
    s_nn = P.Solver(p, U_lin=U0, U_n=U0, rtol=1e-8, max_iters=5000, pc="learned")
    try:
        if head_scale == 0.0:
            net.set_params(np.zeros(net.param_count, np.float32))
        else:
            prm = N.init_params(CIN, CH, COUT, seed=3, head_scale=head_scale)
            net.set_params(N.flatten_params(prm, CIN, CH, COUT).astype(np.float32))
        s_nn.set_network(net)
        b = -s_bj.residual()
        xb, stb, sb = s_bj.solve_linear(b)
        xl, stl, sl = s_nn.solve_linear(b)
        _say(f"  head scale {head_scale}: block-Jacobi {sb['krylov_iters']} it, learned {sl['krylov_iters']} it")
        assert stb == P.M1_OK and stl == P.M1_OK and sl["fell_back"] == 0
        assert abs(sl["krylov_iters"] - sb["krylov_iters"]) <= max(3, 0.1 * sb["krylov_iters"])
        import torch
        assert float(torch.linalg.vector_norm(xl - xb) / torch.linalg.vector_norm(xb)) <= 1e-6
    finally:
        s_bj.close()
        s_nn.close()
        net.close()
