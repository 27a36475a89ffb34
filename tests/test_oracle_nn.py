"""Pins of the network oracle: every gradient against central finite differences,
layer identities, and the BF16 rounding helper against exact cases.  CPU only."""
import numpy as np
import pytest

from oracle import nn_oracle as N

CH = [4, 6, 5]


def _setup(seed=0, H=8, W=8, cin=3, cout=2):
    rng = np.random.default_rng(seed)
    params = N.init_params(cin, CH, cout, seed=seed, head_scale=1.0)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape) * 0.1
    x = rng.standard_normal((H, W, cin))
    t = rng.standard_normal((H, W, cout))
    return params, x, t


def _loss(params, x, t):
    y = N.forward(params, x, CH)
    return N.relative_loss(y, t)[0]


def test_gradients_match_finite_differences():
    params, x, t = _setup()
    y, acts = N.forward(params, x, CH, keep=True)
    L, gy = N.relative_loss(y, t)
    g = N.backward(params, acts, gy, CH)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k, v in params.items():
        idx = [tuple(rng.integers(0, s) for s in v.shape) for _ in range(4)]
        for i in idx:
            old = v[i]
            v[i] = old + h
            lp = _loss(params, x, t)
            v[i] = old - h
            lm = _loss(params, x, t)
            v[i] = old
            fd = (lp - lm) / (2 * h)
            assert g[k][i] == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, i)
    # input gradient
    for _ in range(6):
        i = tuple(rng.integers(0, s) for s in x.shape)
        old = x[i]
        x[i] = old + h
        lp = _loss(params, x, t)
        x[i] = old - h
        lm = _loss(params, x, t)
        x[i] = old
        assert g["input"][i] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)


def test_conv3_is_a_correlation_with_zero_padding():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, 6, 2))
    w = rng.standard_normal((3, 3, 2, 3))
    b = rng.standard_normal(3)
    y = N.conv3_forward(x, w, b)
    # brute force at every pixel
    for h in range(5):
        for ww in range(6):
            acc = b.copy()
            for dy in range(3):
                for dx in range(3):
                    hh, xx = h + dy - 1, ww + dx - 1
                    if 0 <= hh < 5 and 0 <= xx < 6:
                        acc += x[hh, xx] @ w[dy, dx]
            assert np.allclose(y[h, ww], acc, rtol=1e-14, atol=1e-14)


def test_pool_and_upsample_are_adjoint_up_to_scale():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 6, 2))
    z = rng.standard_normal((4, 3, 2))
    # <pool x, z> = <x, pool^T z> with pool^T = up2 / 4
    assert np.sum(N.avgpool2(x) * z) == pytest.approx(np.sum(x * N.up2(z)) / 4, rel=1e-13)
    assert np.allclose(N.avgpool2_backward(z), N.up2(z) / 4)
    assert np.allclose(N.up2_backward(N.up2(z)), 4 * z)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -2.5, 3.0e38, 1e-40])
    got = N.bf16_round(vals)
    # 1 + 2^-9 is a tie between 1 and 1 + 2^-7... bf16 has 8 mantissa bits (7 stored): spacing 2^-7 at 1
    assert got[0] == 1.0
    assert got[1] == 1.0                      # 2^-8 below half-spacing... rounds to nearest: 1.0
    assert got[2] == 1.0 + 2 ** -7            # 1.5 * 2^-8 > half spacing (2^-8) -> up
    assert got[3] == 1.0                      # below half spacing
    assert got[4] == -2.5
    # representable values are fixed points
    rng = np.random.default_rng(4)
    r = N.bf16_round(rng.standard_normal(1000))
    assert np.array_equal(N.bf16_round(r), r)
    # unit roundoff of bf16 (8 significant bits): 2^-8
    x = rng.standard_normal(10000)
    assert np.max(np.abs(N.bf16_round(x) - x) / np.abs(x)) <= 2 ** -8 + 1e-12


def test_bf16_ties_to_even():
    # 1 + 2^-8 is exactly half-way between 1 and 1 + 2^-7: ties to the even mantissa (1.0)
    assert N.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    # 1 + 3*2^-8 is half-way between 1 + 2^-7 (odd) and 1 + 2^-6 (even): goes up
    assert N.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba 2015, Algorithm 1)
# ---------------------------------------------------------------------------
def test_adam_first_step_moves_each_parameter_by_lr_times_the_gradient_sign():
    """After one step the bias-corrected moments are g and g^2 exactly, so every
    parameter moves by -lr g/(|g| + eps): a dropped bias correction moves it by
    about 3.16 lr instead."""
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    p = {"w": np.array([1.0, 2.0, 3.0, 4.0])}
    N.adam_step(p, {"w": g}, {}, lr=0.01, eps=1e-8)
    assert np.allclose(p["w"], [1.0, 2.0, 3.0, 4.0] - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the corrected moments stay g and g^2 for every t."""
    g = np.array([[0.3, -4.0], [1.0, 2.5]])
    p = {"w": np.zeros((2, 2)), "b": np.ones(3)}
    gb = np.array([1.0, -1.0, 0.25])
    st = {}
    for _ in range(7):
        N.adam_step(p, {"w": g, "b": gb}, st, lr=1e-3, eps=0.0)
    assert st["t"] == 7
    assert np.allclose(p["w"], -7e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(p["b"], 1.0 - 7e-3 * np.sign(gb), rtol=0, atol=1e-15)


def test_adam_two_steps_worked_example():
    """Hand-worked two steps with g1 = 2, g2 = -1, beta1 = 0.9, beta2 = 0.999, eps = 0:
    m2 = 0.9*0.1*2 + 0.1*(-1) = 0.08, corrected by 1 - 0.81 = 0.19;
    v2 = 0.999*0.001*4 + 0.001*1 = 0.004996, corrected by 1 - 0.998001 = 0.001999.
    Swapping the two decay rates or the moments changes the second step."""
    p = {"w": np.array([0.0])}
    st = {}
    N.adam_step(p, {"w": np.array([2.0])}, st, lr=0.1, eps=0.0)
    assert p["w"][0] == pytest.approx(-0.1, abs=1e-15)
    N.adam_step(p, {"w": np.array([-1.0])}, st, lr=0.1, eps=0.0)
    step2 = 0.1 * (0.08 / 0.19) / np.sqrt(0.004996 / 0.001999)
    assert p["w"][0] == pytest.approx(-0.1 - step2, rel=1e-13)
    assert step2 == pytest.approx(0.026633, rel=1e-4)


def test_adam_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(3)
    gs = [rng.standard_normal(5) for _ in range(4)]
    pa, pb, sa, sb = {"w": np.zeros(5)}, {"w": np.zeros(5)}, {}, {}
    for g in gs:
        N.adam_step(pa, {"w": g}, sa, lr=1e-2, eps=0.0)
        N.adam_step(pb, {"w": 1e3 * g}, sb, lr=1e-2, eps=0.0)
    assert np.allclose(pa["w"], pb["w"], rtol=1e-12, atol=0)
