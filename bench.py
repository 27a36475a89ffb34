#!/usr/bin/env python3
"""Benchmark: implicit M1 cell-updates/s at 1e-8 residual, plain FP64 vs mixed precision.

Workload: the 2D 1024x1024 beam/shadow problem (background sigma*dx = 1e-3, eight
seeded elliptical clumps with sigma*dx = 1e3, a beam F = cE entering through the
-x face, outflow elsewhere; centred flux source and HLL speeds floored at
+-0.1c as in the paper's shadow test, Sect. 5.4), implicit steps at dt = 50 dx/c
starting from E = 1e-6, F = 0.  One "step" is one complete implicit step: Newton
until ||R(U)|| <= 1e-8 ||R(U^n)||, each Newton iteration a block-Jacobi GMRES(30)
solve (pseudo-transient continuation, positivity clip and non-monotone line
search as globalisation; they leave the root unchanged).  Inputs are resident
in HBM before timing starts.

Prints ONE JSON line.  `value` is the faster of the measured solver variants
that converged on every step; every variant's own numbers are in `variants`.
`roofline` is for the kernel class with the largest share of GPU time (HIP
events on the library's stream over the timed region, algorithmic bytes counted
by the library per launch); `roofline_apply` for the operator apply.
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "implicit M1 cell-updates/s at 1e-8 residual: plain FP64 vs mixed+learned"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--dt", type=float, default=50.0)
    ap.add_argument("--variants", default="fp64,mixed")
    ap.add_argument("--max-iters", type=int, default=3000, help="GMRES iterations per linear solve")
    ap.add_argument("--newton-max", type=int, default=60)
    ap.add_argument("--lin-rtol", type=float, default=1e-3, help="linear tolerance per Newton iteration")
    ap.add_argument("--psi0", type=float, default=1.0, help="pseudo-transient continuation start (0: off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-events", action="store_true", help="do not time kernels with HIP events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, 5 times: 1 GiB read + 1 GiB written per launch.
    Its FETCH_SIZE / WRITE_SIZE counter readings calibrate the counters' units."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "seconds_per_copy": dt,
                      "GBps_read_plus_write": 2 * (1 << 30) / dt / 1e9}), flush=True)


VARIANTS = {
    "fp64": dict(precision="fp64"),
    "mixed": dict(precision="mixed", basis_fp32=False, inner_rtol=1e-6),
    "mixed32": dict(precision="mixed", basis_fp32=True, inner_rtol=1e-6),
}
DTYPES = {"fp64": "f64", "mixed": "f32 operator+preconditioner / f64 Krylov", "mixed32": "f32 storage / f64 accumulation"}


def run_variant(P, torch, p, U0, name, args):
    opts = dict(VARIANTS[name], rtol=args.lin_rtol, newton_rtol=1e-8, restart=30, max_iters=args.max_iters,
                newton_max=args.newton_max, ptc_psi0=args.psi0, ptc_rtol=1e-3, positivity_clip=0.9, line_search=True)
    s = P.Solver(p, **opts)
    try:
        U = s.to_device(U0)
        for _ in range(args.warmup):
            st, _ = s.implicit_step(U, raise_on_fail=False)
            print(f"[bench] {name} warmup step status={st}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        s.profile_enable(not args.no_events)
        stats = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            st, sd = s.implicit_step(U, raise_on_fail=False)
            sd["status"] = st
            stats.append(sd)
            print(f"[bench] {name} step {k} status={st} newton={sd['newton_iters']} krylov={sd['krylov_iters']} "
                  f"{sd['seconds']:.3f}s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = s.profile() if not args.no_events else {}
        s.profile_enable(False)
    finally:
        s.close()
    N = p["n"][0] * p["n"][1]
    ok = all(x["status"] == P.M1_OK for x in stats)
    return dict(
        cell_updates_per_s=N * args.steps / wall,
        ms_per_step=1e3 * wall / args.steps,
        converged_all=ok,
        newton_iters=[x["newton_iters"] for x in stats],
        krylov_iters=[x["krylov_iters"] for x in stats],
        cells_f_gt_1=[x["cells_f_gt_1"] for x in stats],
        kernels=prof,
    )


def roofline(prof):
    if not prof:
        return None, None
    top = max(prof.items(), key=lambda kv: kv[1]["ms"])
    name, v = top

    def entry(nm, e):
        avg_s = e["ms"] / e["launches"] / 1e3
        per_launch = e["bytes"] / e["launches"]
        gbs = per_launch / avg_s / 1e9
        return {"kernel": nm, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches": e["launches"], "share_of_gpu_time": round(e["ms"] / sum(x["ms"] for x in prof.values()), 4)}

    apply = entry("apply", prof["apply"]) if "apply" in prof else None
    return entry(name, v), apply


def cpu_baseline(p, U0, fp64_result, budget_s=25.0):
    """The oracle on a bounded sample of the same workload: one linearisation
    (closure, coefficients, residual, block-Jacobi blocks) and one 30-iteration
    GMRES cycle at full size, scaled by the GPU plain-FP64 iteration counts."""
    from threadpoolctl import threadpool_limits

    import numpy as np
    from oracle import m1_oracle as O

    with threadpool_limits(limits=1):
        sch = O.Scheme.from_problem(p)
        t0 = time.perf_counter()
        lin = O.linearize(sch, p["sigma"], None, U0, U0, p["dt"])
        R = O.residual(lin)
        M = O.BlockJacobi(lin)
        t_setup = time.perf_counter() - t0
        iters = 30
        t0 = time.perf_counter()
        O.gmres(lambda v: O.apply_operator(lin, v), M, -R.reshape(-1), restart=30, fixed_iters=iters)
        t_iter = (time.perf_counter() - t0) / iters
    newton = float(np.mean(fp64_result["newton_iters"]))
    krylov = float(np.mean(fp64_result["krylov_iters"]))
    t_step = (newton + 1) * t_setup + krylov * t_iter
    N = p["n"][0] * p["n"][1]
    return {"value": N / t_step, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle at full size: one linearisation+residual+block-Jacobi setup ({t_setup:.2f}s) and one "
                       f"30-iteration GMRES cycle ({t_iter:.3f}s/iteration), scaled by the GPU plain-FP64 counts "
                       f"({newton:.1f} Newton, {krylov:.0f} Krylov iterations per step); BLAS limited to 1 thread")}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2011_13926_amd as P
    import workloads as W

    p = W.beam_shadow(n=(args.n, args.n), dt=args.dt)
    U0 = np.stack([p["E"], p["F"][0], p["F"][1]])
    results = {}
    for name in [v for v in args.variants.split(",") if v]:
        results[name] = run_variant(P, torch, p, U0, name, args)
    valid = {k: v for k, v in results.items() if v["converged_all"]}
    pick = max(valid or results, key=lambda k: (valid or results)[k]["cell_updates_per_s"])
    head = results[pick]
    roof, roof_apply = roofline(head["kernels"])
    out = {
        "metric": METRIC,
        "value": head["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[pick],
        "data": "synthetic",
        "config": {"workload": f"beam_shadow_{args.n}", "grid": [args.n, args.n], "dt_over_cfl": args.dt,
                   "flux_source": "centered", "lambda_floor": 0.1, "newton_rtol": 1e-8,
                   "linear_rtol": args.lin_rtol, "restart": 30, "preconditioner": "block_jacobi",
                   "ptc_psi0": args.psi0, "ptc_rtol": 1e-3, "positivity_clip": 0.9, "line_search": True,
                   "solver": pick, "seed": 2011},
        "converged": head["converged_all"],
        "variants": {k: {kk: vv for kk, vv in v.items() if kk != "kernels"} for k, v in results.items()},
        "roofline": roof,
        "roofline_apply": roof_apply,
        "kernels": head["kernels"],
    }
    if not args.no_cpu_baseline and "fp64" in results:
        out["cpu_baseline"] = cpu_baseline(p, U0, results["fp64"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
