"""Train the learned preconditioner on residual/error pairs the solver generates.

For each training problem the Newton iteration of the implicit step is replayed
through the C ABI (m1_linearize, m1_residual, m1_solve_linear).  Every linear
system A delta = b gives pairs (r, e): r = b with e = delta (x0 = 0), and the
residual/error after one and after three GMRES(30) cycles.  Each pair becomes a
network input (m1_nn_features) and target (m1_nn_target); training runs the
project's BF16 MFMA forward/backward kernels and Adam (m1nn_train_step).

    python -m paper_2011_13926_amd.train_nn --out weights.bin --train 0-7 --steps 3
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHANNELS = (32, 48, 64, 64)


def _log(*a):
    print("[train_nn]", *a, file=sys.stderr, flush=True)


WORKLOAD = "voronoi"


def problem(seed, n=512, dt=None):
    import workloads as W
    if WORKLOAD == "diffusive":
        return W.diffusive_lognormal(n=(n, n), seed=seed, dt=1000.0 if dt is None else dt)
    return W.voronoi_opacity(n=(n, n), seed=seed, dt=100.0 if dt is None else dt)


def generate_pairs(P, torch, p, steps, newton_max=6, rtol=1e-10, partial=(30, 90)):
    """Replay `steps` implicit steps of problem p; return a list of (features, target) device tensors."""
    s_full = P.Solver(p, rtol=rtol)
    s_part = {k: P.Solver(p, rtol=1e-30, max_iters=k) for k in partial}
    U = s_full.to_device(np.stack([p["E"], p["F"][0], p["F"][1]]))
    pairs = []
    try:
        for step in range(steps):
            Un = U.clone()
            Uk = U.clone()
            r0 = None
            for it in range(newton_max):
                s_full.linearize(Uk, Un)
                b = -s_full.residual()
                rn = float(torch.linalg.vector_norm(b))
                r0 = rn if r0 is None else r0
                if it > 0 and rn <= rtol * r0:
                    break
                delta, st, stats = s_full.solve_linear(b, raise_on_fail=False)
                pairs.append((s_full.nn_features(b), s_full.nn_target(b, delta)))
                for k, sp in s_part.items():
                    sp.linearize(Uk, Un)
                    xk, _, _ = sp.solve_linear(b, raise_on_fail=False)
                    rk = b - sp.apply_operator(xk)
                    pairs.append((s_full.nn_features(rk), s_full.nn_target(rk, delta - xk)))
                Uk = Uk + delta
            U = Uk
    finally:
        s_full.close()
        for sp in s_part.values():
            sp.close()
    return pairs


def train(P, torch, pairs, iters, lr=1e-3, seed=0, net=None, n=512, log_every=100, channels=CHANNELS):
    if net is None:
        net = P.Net(9, 3, channels, Hmax=n, Wmax=n)
        net.init_params(seed=seed, head_scale=0.1)
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        f, t = pairs[int(rng.integers(len(pairs)))]
        step_lr = lr * 0.5 * (1 + np.cos(np.pi * it / iters))   # cosine decay
        loss = net.train_step(f, t, step_lr)
        hist.append(loss)
        if log_every and (it % log_every == 0 or it == iters - 1):
            _log(f"iter {it} loss {np.mean(hist[-log_every:]):.4f}")
    return net, hist


def heldout_loss(torch, net, pairs):
    """Mean relative loss ||NN(x) - t||^2 / ||t||^2 on pairs not used for training."""
    vals = []
    for f, t in pairs:
        y = net.forward(f)
        tt = torch.as_tensor(t, dtype=torch.float32, device=y.device)
        vals.append(float(((y - tt) ** 2).sum() / (tt ** 2).sum().clamp_min(1e-300)))
    return float(np.mean(vals)) if vals else float("nan")


def evaluate(P, torch, net, seeds, n=512, rtol=1e-8, dt=None):
    """GMRES iterations and time to rtol with block-Jacobi vs the learned preconditioner
    on the first Newton linear system of each held-out problem."""
    out = []
    for seed in seeds:
        p = problem(seed, n, dt)
        U0 = np.stack([p["E"], p["F"][0], p["F"][1]])
        s_bj = P.Solver(p, U_lin=U0, U_n=U0, rtol=rtol, max_iters=20000)
        s_nn = P.Solver(p, U_lin=U0, U_n=U0, rtol=rtol, max_iters=20000, pc="learned")
        s_nn.set_network(net)
        b = -s_bj.residual()
        rec = {"seed": seed}
        for name, s in (("bj", s_bj), ("learned", s_nn)):
            s.solve_linear(b, raise_on_fail=False)          # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, stats = s.solve_linear(b, raise_on_fail=False)
            torch.cuda.synchronize()
            rec[name] = {"iters": stats["krylov_iters"], "seconds": time.perf_counter() - t0,
                         "status": st, "fell_back": stats["fell_back"], "rel_residual": stats["rel_residual"]}
        s_bj.close()
        s_nn.close()
        out.append(rec)
        _log(json.dumps(rec))
    return out


def _seeds(spec):
    a, _, b = spec.partition("-")
    return list(range(int(a), int(b) + 1)) if b else [int(a)]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--train", default="0-7")
    ap.add_argument("--heldout", default="1000-1003")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--report", default=None)
    ap.add_argument("--channels", default=",".join(str(c) for c in CHANNELS))
    ap.add_argument("--no-solve-eval", action="store_true", help="skip the FGMRES comparison on held-out seeds")
    ap.add_argument("--workload", default="voronoi", choices=["voronoi", "diffusive"],
                    help="voronoi: workloads.voronoi_opacity at dt = 100; diffusive: workloads.diffusive_lognormal "
                         "at dt = 1000")
    args = ap.parse_args()
    global WORKLOAD
    WORKLOAD = args.workload
    channels = tuple(int(v) for v in args.channels.split(","))
    import torch

    import paper_2011_13926_amd as P

    t0 = time.perf_counter()
    pairs = []
    for seed in _seeds(args.train):
        pairs += generate_pairs(P, torch, problem(seed, args.n), args.steps)
        _log(f"seed {seed}: {len(pairs)} pairs ({time.perf_counter() - t0:.1f}s)")
    held = []
    for seed in _seeds(args.heldout):
        held += generate_pairs(P, torch, problem(seed, args.n), 1, newton_max=2)
    net, hist = train(P, torch, pairs, args.iters, lr=args.lr, n=args.n, channels=channels)
    net.save(args.out)
    _log(f"saved {args.out} after {time.perf_counter() - t0:.1f}s")
    hl = heldout_loss(torch, net, held)
    _log(f"held-out loss {hl:.4f} on {len(held)} pairs")
    ev = [] if args.no_solve_eval else evaluate(P, torch, net, _seeds(args.heldout), args.n)
    rep = {"workload": args.workload, "n": args.n, "pairs": len(pairs), "iters": args.iters, "channels": list(channels),
           "loss_first100": float(np.mean(hist[:100])), "loss_last100": float(np.mean(hist[-100:])),
           "heldout_pairs": len(held), "heldout_loss": hl, "heldout": ev}
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
