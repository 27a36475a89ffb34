"""CPU FP64 oracle of the learned preconditioner's convolutional network.

TEST INFRASTRUCTURE ONLY (tests, the smoke entry and the benchmark's CPU
baseline may use it; the product path never does).

The network (a small U-Net, written here from its definition):
  level l = 0..L-1 (channels C_l), input of C_in channels, H x W divisible by 2^(L-1)
  encoder:  e_l = relu(conv3(relu(conv3(a_l))))      a_0 = input, a_{l+1} = avgpool2(e_l)
  bottom:   d_{L-1} = e_{L-1}
  decoder:  d_l = relu(conv3(relu(conv3(concat(up2(d_{l+1}), e_l)))))   l = L-2..0
  head:     y = conv1(d_0)                            (C_out channels, no activation)
conv3: 3x3 convolution, stride 1, zero padding 1, bias; conv1: 1x1 with bias;
avgpool2: mean over 2x2 blocks; up2: nearest-neighbour x2; concat along channels
(upsampled first, skip second).  Tensors are HWC (channels last).
Weights of a conv3 are (3, 3, C_in, C_out) indexed [dy, dx, ci, co].

Also: BF16 round-to-nearest-even emulation used when comparing with the GPU's
BF16 kernels.
"""
from __future__ import annotations

import numpy as np

RELU = "relu"


def bf16_round(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    x = np.asarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# layers (forward and backward), plain array code
# ---------------------------------------------------------------------------
def conv3_forward(x, w, b):
    """y[h, w, :] = b + sum_{dy, dx} xpad[h + dy, w + dx, :] @ w[dy, dx]."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (H, W, w.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            y += xp[dy:dy + H, dx:dx + W, :] @ w[dy, dx]
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 with respect to x, w and b given dL/dy."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            gxp[dy:dy + H, dx:dx + W, :] += gy @ w[dy, dx].T
            gw[dy, dx] = xp[dy:dy + H, dx:dx + W, :].reshape(-1, x.shape[2]).T @ gy.reshape(-1, gy.shape[2])
    gb = gy.sum(axis=(0, 1))
    return gxp[1:-1, 1:-1, :], gw, gb


def conv1_forward(x, w, b):
    return x @ w + b


def conv1_backward(x, w, gy):
    H, W, C = x.shape
    return gy @ w.T, x.reshape(-1, C).T @ gy.reshape(-1, gy.shape[2]), gy.sum(axis=(0, 1))


def avgpool2(x):
    H, W, C = x.shape
    return x.reshape(H // 2, 2, W // 2, 2, C).mean(axis=(1, 3))


def avgpool2_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=0), 2, axis=1) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def up2_backward(gy):
    H, W, C = gy.shape
    return gy.reshape(H // 2, 2, W // 2, 2, C).sum(axis=(1, 3))


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def layer_specs(c_in, channels, c_out):
    """List of (name, kind, cin, cout) in execution order."""
    specs = []
    L = len(channels)
    prev = c_in
    for l in range(L):
        specs.append((f"enc{l}a", "conv3", prev, channels[l]))
        specs.append((f"enc{l}b", "conv3", channels[l], channels[l]))
        prev = channels[l]
    for l in range(L - 2, -1, -1):
        specs.append((f"dec{l}a", "conv3", channels[l + 1] + channels[l], channels[l]))
        specs.append((f"dec{l}b", "conv3", channels[l], channels[l]))
    specs.append(("head", "conv1", channels[0], c_out))
    return specs


def init_params(c_in, channels, c_out, seed=0, head_scale=0.1):
    """He-normal weights, zero biases; the head is scaled down (the correction starts small)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, kind, ci, co in layer_specs(c_in, channels, c_out):
        if kind == "conv3":
            w = rng.standard_normal((3, 3, ci, co)) * np.sqrt(2.0 / (9 * ci))
        else:
            w = rng.standard_normal((ci, co)) * np.sqrt(1.0 / ci) * head_scale
        params[name + ".w"] = w
        params[name + ".b"] = np.zeros(co)
    return params


def forward(params, x, channels, keep=False, act_round=None):
    """Network output y (H, W, C_out); with keep=True also the activations for backward.

    act_round (optional) is applied to the input and to every stored activation
    (conv and pooling outputs), e.g. to emulate reduced-precision storage."""
    rnd = act_round if act_round is not None else (lambda v: v)
    L = len(channels)
    acts = {}
    a = rnd(x)
    enc = []
    for l in range(L):
        acts[f"enc{l}a.in"] = a
        h = rnd(np.maximum(conv3_forward(a, params[f"enc{l}a.w"], params[f"enc{l}a.b"]), 0.0))
        acts[f"enc{l}b.in"] = h
        e = rnd(np.maximum(conv3_forward(h, params[f"enc{l}b.w"], params[f"enc{l}b.b"]), 0.0))
        enc.append(e)
        acts[f"enc{l}.out"] = e
        if l < L - 1:
            a = rnd(avgpool2(e))
    d = enc[L - 1]
    for l in range(L - 2, -1, -1):
        cat = np.concatenate([up2(d), enc[l]], axis=2)
        acts[f"dec{l}a.in"] = cat
        h = rnd(np.maximum(conv3_forward(cat, params[f"dec{l}a.w"], params[f"dec{l}a.b"]), 0.0))
        acts[f"dec{l}b.in"] = h
        d = rnd(np.maximum(conv3_forward(h, params[f"dec{l}b.w"], params[f"dec{l}b.b"]), 0.0))
        acts[f"dec{l}.out"] = d
    acts["head.in"] = d
    y = conv1_forward(d, params["head.w"], params["head.b"])
    return (y, acts) if keep else y


def backward(params, acts, gy, channels):
    """Gradients of a scalar loss with respect to every parameter given dL/dy."""
    L = len(channels)
    g = {}
    gd, g["head.w"], g["head.b"] = conv1_backward(acts["head.in"], params["head.w"], gy)
    genc = [None] * L
    # decoder: computed from level L-2 down to 0, so walk it back from level 0 up
    for l in range(0, L - 1):
        out = acts[f"dec{l}.out"]
        gpre = gd * (out > 0)
        gh, g[f"dec{l}b.w"], g[f"dec{l}b.b"] = conv3_backward(acts[f"dec{l}b.in"], params[f"dec{l}b.w"], gpre)
        gpre = gh * (acts[f"dec{l}b.in"] > 0)
        gcat, g[f"dec{l}a.w"], g[f"dec{l}a.b"] = conv3_backward(acts[f"dec{l}a.in"], params[f"dec{l}a.w"], gpre)
        cu = channels[l + 1]
        gup, gskip = gcat[:, :, :cu], gcat[:, :, cu:]
        genc[l] = gskip if genc[l] is None else genc[l] + gskip
        gd = up2_backward(gup)          # gradient of d_{l+1}
    # bottom: d_{L-1} = e_{L-1}
    genc[L - 1] = gd if genc[L - 1] is None else genc[L - 1] + gd
    # encoder, from the bottom level down
    ga_next = None
    for l in range(L - 1, -1, -1):
        ge = genc[l]
        if ga_next is not None:
            ge = ge + avgpool2_backward(ga_next)
        gpre = ge * (acts[f"enc{l}.out"] > 0)
        gh, g[f"enc{l}b.w"], g[f"enc{l}b.b"] = conv3_backward(acts[f"enc{l}b.in"], params[f"enc{l}b.w"], gpre)
        gpre = gh * (acts[f"enc{l}b.in"] > 0)
        ga, g[f"enc{l}a.w"], g[f"enc{l}a.b"] = conv3_backward(acts[f"enc{l}a.in"], params[f"enc{l}a.w"], gpre)
        ga_next = ga
    g["input"] = ga_next
    return g


def flatten_params(params, c_in, channels, c_out):
    """Parameters in definition order: each weight (C order) then its bias."""
    out = []
    for name, kind, ci, co in layer_specs(c_in, channels, c_out):
        out.append(params[name + ".w"].ravel())
        out.append(params[name + ".b"].ravel())
    return np.concatenate(out)


def unflatten_params(flat, c_in, channels, c_out):
    params, k = {}, 0
    for name, kind, ci, co in layer_specs(c_in, channels, c_out):
        shape = (3, 3, ci, co) if kind == "conv3" else (ci, co)
        n = int(np.prod(shape))
        params[name + ".w"] = np.asarray(flat[k:k + n], float).reshape(shape)
        k += n
        params[name + ".b"] = np.asarray(flat[k:k + co], float)
        k += co
    return params


def relative_loss(y, target):
    """L = ||y - t||^2 / ||t||^2 and dL/dy."""
    den = float(np.sum(target * target))
    diff = y - target
    return float(np.sum(diff * diff)) / den, 2.0 * diff / den


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) on FP64 parameters; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m." + k, np.zeros_like(params[k]))
        v = state.setdefault("v." + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
