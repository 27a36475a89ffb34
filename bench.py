#!/usr/bin/env python3
"""Benchmark: implicit M1 cell-updates/s at 1e-8 residual, plain FP64 block-Jacobi vs mixed precision.

One "step" is one complete implicit step of the named workload: Newton until
||R(U)|| <= 1e-8 ||R(U^n)||, every Newton system solved by right-preconditioned
GMRES(30) to a true relative residual of 1e-8.  Inputs are resident in HBM
before timing starts; every timed step restarts from the same U^n.

Workloads (seeded, synthetic; recipes in ``workloads``):

* voronoi_512 (default): 2D 512^2 periodic Voronoi opacity field (64 sites,
  sigma dx log-uniform in 1e-3..1e4), dt = 100 dx/c, well-balanced source,
  held-out seed 1000.  The largest configuration of the set whose implicit
  step converges: the beam/shadow 1024^2, coupled 256^3 and ionisation-front
  192^3 steps stall in the Newton iteration whatever the linear solver (with
  exact sparse-LU solves on reduced instances too).  Its root has E <= 0 in a
  few hundred optically thick cells (the scheme is not positivity preserving);
  the line reports that count and measures the solves anyway (the root is the
  same for every variant).
* diffusive_gaussian_64, beam_shadow_1024, coupled_lognormal_256,
  ionization_front_192 (the last three report converged = false).

Variants: plain FP64 with block-Jacobi (the baseline of the metric), FP64 with
the aggregation multigrid preconditioner, mixed precision (FP32 operator and
preconditioner, FP64 Krylov basis and restarts) with either, and the mixed
multigrid form with an FP32-stored basis (reported as its own variant).
`value` is the fastest mixed-precision variant with an FP64 Krylov basis whose
steps all converged; each variant states its error against the plain-FP64
result.  `roofline` is for
the kernel class with the largest share of GPU time (HIP events on the
library's stream over the timed region, algorithmic bytes counted by the
library per launch); `roofline_apply` for the operator apply.  `cpu_baseline`
runs full oracle implicit steps of a reduced instance of the same generator
at one thread and on every core, and evaluates the oracle's residual of each
variant's GPU result.
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
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2011_13926_amd", "csrc")

# profiler kernel class -> prefixes of the HIP kernels' names (without "void " and "m1::")
CLASS_KERNEL = {
    "apply_bj_fused": ("k_apply2d_lds<16, false, 0, true", "k_apply2d_lds<16, true, 0, true"),
    "apply": ("k_apply2d_lds<16, false, 0, false", "k_apply2d_lds<16, true, 0, false", "k_stencil<2, false, 0",
              "k_stencil<2, true, 0", "k_stencil<3, false, 0", "k_stencil<3, true, 0"),
    "arnoldi_dot": ("k_dot<", "k_dot4<"), "arnoldi_update": ("k_update<", "k_update4<"), "arnoldi_scalar": ("k_scalar",),
    "x_update": ("k_xupdate<",), "block_jacobi": ("k_bj<",),
    "true_residual": ("k_apply2d_lds<16, false, 1", "k_apply2d_lds<16, true, 1", "k_stencil<2, false, 1",
                      "k_stencil<2, true, 1", "k_stencil<3, false, 1", "k_stencil<3, true, 1"),
    "time_step": ("k_step2d_lds<", "k_step_direct<"),
    "mg_fine": ("k_mg_fine_smooth<", "k_mg_restrict_fine<", "k_mg_prolong_fine<", "k_mg_cast<", "k_mg_sweep2d<",
                "k_mg_sweep2d_x2<"),
    "mg_smooth": ("k_mg_smooth<", "k_mg_prolong<"),
    "mg_down": ("k_mg_down_lanes<",),
    "mg_coarse_solve": ("k_mg_coarse_solve<",),
    "mg_setup": ("k_mg_galerkin<", "k_mg_invert<", "k_mg_dense_inverse<", "k_mg_dense_inverse_reg<", "k_setup_bj<2, false, true",
                 "k_setup_bj<2, true, true", "k_setup_bj<3, false, true", "k_setup_bj<3, true, true"),
}


def _kname(nm):
    return nm.split("(")[0].replace("void ", "").replace("m1::", "").strip()


def kernel_class(nm):
    k = _kname(nm)
    for cls, prefs in CLASS_KERNEL.items():
        if any(k.startswith(pf) for pf in prefs):
            return cls
    return k.split("<")[0]


def source_hash():
    """SHA-256 over the HIP sources: byte-counter readings are valid only for the
    kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for fn in sorted(os.listdir(CSRC)):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, fn), "rb") as fh:
                h.update(fn.encode() + b"\0" + fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="voronoi_512", choices=sorted(WORKLOADS))
    ap.add_argument("--variants", default="fp64_bj,mixed_bj,fp64_mg,mixed_mg,mixed32_mg")
    ap.add_argument("--scheme", default="implicit", choices=["implicit", "semi_implicit", "explicit"],
                    help="implicit (the default benchmark) or the explicit / semi-implicit step at the CFL "
                         "time step, advancing the workload's dt per timed step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--newton-max", type=int, default=None,
                    help="override the workload's Newton iteration cap (bounded profiling runs)")
    ap.add_argument("--no-events", action="store_true", help="do not time kernels with HIP events")
    ap.add_argument("--nn", action="store_true",
                    help="time the learned preconditioner's U-Net at 512^2 instead: forward pass and training step "
                         "(forward + backward + Adam) on the BF16 MFMA kernels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="turn rocprofv3 CSV output under DIR/{trace,fetch,write,copy_fetch,copy_write} into "
                         "profiles/<workload>_kernels.md and profiles/<workload>_traffic.json")
    ap.add_argument("--profile-commands", default="", help="text recorded with --summarize-profiles")
    ap.add_argument("--profile-name", default=None,
                    help="label of the summaries written by --summarize-profiles (default: the workload; "
                         "'<workload>_<scheme>' for the explicit and semi-implicit benchmarks)")
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


GLOBALISED = dict(ptc_psi0=1.0, ptc_rtol=1e-3, positivity_clip=0.9, line_search=True)
# every workload: linear and nonlinear tolerance 1e-8 (the metric's)
WORKLOADS = {
    "voronoi_512": dict(make=lambda W: W.voronoi_opacity(seed=1000),
                        solver=dict(rtol=1e-8, newton_rtol=1e-8, max_iters=60000, newton_max=40, line_search=True),
                        # a 48 x 48 window of the same field (three Voronoi sites, sigma dx 0.75..2800),
                        # periodic: 16 Newton iterations like the full grid
                        cpu_sample=lambda W: W.window(W.voronoi_opacity(seed=1000), (100, 100), (48, 48),
                                                      ("periodic",) * 4)),
    "beam_shadow_1024": dict(make=lambda W: W.beam_shadow(),
                             solver=dict(rtol=1e-8, newton_rtol=1e-8, max_iters=600, newton_max=30, **GLOBALISED),
                             cpu_sample=None),
    "diffusive_gaussian_64": dict(make=lambda W: W.diffusive_gaussian(),
                                  solver=dict(rtol=1e-8, newton_rtol=1e-8, max_iters=20000, newton_max=20),
                                  cpu_sample=lambda W: W.diffusive_gaussian()),
    "coupled_lognormal_256": dict(make=lambda W: W.coupled_lognormal(),
                                  solver=dict(rtol=1e-8, newton_rtol=1e-8, max_iters=300, newton_max=30, **GLOBALISED),
                                  cpu_sample=None),
    "ionization_front_192": dict(make=lambda W: W.ionization_front(),
                                 solver=dict(rtol=1e-8, newton_rtol=1e-8, max_iters=300, newton_max=30, **GLOBALISED),
                                 cpu_sample=None),
}
# V(12,12) on the finest level (its sweeps fused into the staged operator, two per
# launch: the cheap part of a cycle), one sweep each way below it, damping 0.9: the
# fastest mixed step of sweeps over fine sweeps 3..16, coarse sweeps 0..3 and damping
# 0.7..1.1 on the 512^2 Voronoi step (0.40 s against 0.45 s for V(8,8) and 0.82 s for
# V(4,4) with 2 coarse sweeps at 0.7; damping 1.0 doubles the iterations, 1.1 diverges)
MG = dict(pc="mg", mg_nu1=12, mg_nu2=12, mg_nu1_coarse=1, mg_nu2_coarse=1, mg_omega=0.9)
VARIANTS = {
    "fp64_bj": dict(precision="fp64", pc="bj"),
    "mixed_bj": dict(precision="mixed", basis_fp32=False, inner_rtol=1e-6, pc="bj"),
    "fp64_mg": dict(precision="fp64", **MG),
    "mixed_mg": dict(precision="mixed", basis_fp32=False, inner_rtol=1e-6, **MG),
    "mixed32_mg": dict(precision="mixed", basis_fp32=True, inner_rtol=1e-6, **MG),
}
DTYPES = {"fp64_bj": "f64", "fp64_mg": "f64",
          "mixed_bj": "f32 operator+preconditioner / f64 Krylov", "mixed_mg": "f32 operator+preconditioner / f64 Krylov",
          "mixed32_mg": "f32 storage / f64 accumulation"}


def state0(p):
    import numpy as np
    comps = [p["E"]] + [p["F"][m] for m in range(p["ndim"])]
    if p["source"] == "coupled_t":
        comps.append(p["T"])
    return np.stack(comps)


def run_variant(P, torch, p, U0, name, args):
    import numpy as np
    solver = dict(WORKLOADS[args.workload]["solver"])
    if args.newton_max is not None:
        solver["newton_max"] = args.newton_max
    opts = dict(VARIANTS[name], restart=30, commit_nonadmissible=True, **solver)
    s = P.Solver(p, **opts)
    try:
        U0d = s.to_device(U0)
        U = U0d.clone()
        for _ in range(args.warmup):
            U.copy_(U0d)
            st, _ = s.implicit_step(U, raise_on_fail=False)
            print(f"[bench] {name} warmup step status={st}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        s.profile_enable(not args.no_events)
        stats = []
        wall = 0.0
        # every timed step is the same implicit step on the same input (restored
        # from U^n outside the timed interval)
        for k in range(args.steps):
            U.copy_(U0d)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, sd = s.implicit_step(U, raise_on_fail=False)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            sd["status"] = st
            stats.append(sd)
            print(f"[bench] {name} step {k} status={st} newton={sd['newton_iters']} krylov={sd['krylov_iters']} "
                  f"nl={sd['nonlinear_residual']:.2e} {sd['seconds']:.3f}s E<=0 cells {sd['cells_e_nonpos']}",
                  file=sys.stderr, flush=True)
        prof = s.profile() if not args.no_events else {}
        s.profile_enable(False)
        U_final = U.cpu().numpy()
    finally:
        s.close()
    N = int(np.prod(p["n"][:p["ndim"]]))
    tol = WORKLOADS[args.workload]["solver"]["newton_rtol"]
    # converged: the nonlinear residual reached the tolerance (M1_OK, or M1_NOT_ADMISSIBLE:
    # converged to a root with E <= 0 somewhere, written back for this measurement)
    conv = all(x["status"] in (P.M1_OK, P.M1_NOT_ADMISSIBLE) and x["nonlinear_residual"] <= tol for x in stats)
    return dict(
        cell_updates_per_s=N * args.steps / wall,
        ms_per_step=1e3 * wall / args.steps,
        converged_all=conv,
        status=[P.m1_status_string(x["status"]).decode() for x in stats],
        admissible=all(x["cells_e_nonpos"] == 0 for x in stats),
        cells_e_nonpos=[x["cells_e_nonpos"] for x in stats],
        newton_iters=[x["newton_iters"] for x in stats],
        krylov_iters=[x["krylov_iters"] for x in stats],
        nonlinear_residual=[x["nonlinear_residual"] for x in stats],
        cells_f_gt_1=[x["cells_f_gt_1"] for x in stats],
        kernels=prof,
        U=U_final,
    )


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _counter_means(d, counter):
    """Mean counter value per dispatch, by kernel name (text before the argument list)."""
    import csv
    agg = {}
    for path in _csvs(d, "counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                nm = r["Kernel_Name"].split("(")[0].strip()
                a = agg.setdefault(nm, [0, 0.0])
                a[0] += 1
                a[1] += float(r["Counter_Value"])
    return {k: (n, tot / n) for k, (n, tot) in agg.items()}


def summarize_profiles(d, workload, commands):
    """Write the committed summaries: kernel statistics per kernel and per class
    and, per kernel, the HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE (KiB)
    scaled by what the same counters read for a plain device copy of known size.
    Without counter CSVs under d the existing traffic summary is reused."""
    import csv
    rows = []
    for path in _csvs(os.path.join(d, "trace"), "kernel_stats.csv"):
        with open(path) as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tpath = os.path.join(PROFILES, f"{workload}_traffic.json")
    if _csvs(os.path.join(d, "fetch"), "counter_collection.csv"):
        cf = _counter_means(os.path.join(d, "copy_fetch"), "FETCH_SIZE")
        cw = _counter_means(os.path.join(d, "copy_write"), "WRITE_SIZE")
        copy_bytes = float(1 << 30)
        kf = max(cf.items(), key=lambda kv: kv[1][1])
        kw = max(cw.items(), key=lambda kv: kv[1][1])
        scale_f = copy_bytes / (kf[1][1] * 1024.0)
        scale_w = copy_bytes / (kw[1][1] * 1024.0)
        fetch = _counter_means(os.path.join(d, "fetch"), "FETCH_SIZE")
        write = _counter_means(os.path.join(d, "write"), "WRITE_SIZE")
        kernels = {}
        for nm in sorted(set(fetch) | set(write)):
            fn, fv = fetch.get(nm, (0, 0.0))
            wn, wv = write.get(nm, (0, 0.0))
            kernels[nm] = {"dispatches": max(fn, wn), "fetch_kib": fv, "write_kib": wv,
                           "hbm_bytes_per_dispatch": fv * 1024.0 * scale_f + wv * 1024.0 * scale_w}
        traffic = {"workload": workload, "source_sha256": source_hash(), "copy_kernel": kf[0],
                   "copy_fetch_kib": kf[1][1], "copy_write_kib": kw[1][1], "scale_fetch": scale_f,
                   "scale_write": scale_w, "kernels": kernels, "commands": commands}
        os.makedirs(PROFILES, exist_ok=True)
        with open(tpath, "w") as fh:
            json.dump(traffic, fh, indent=1)
    traffic = None
    if os.path.exists(tpath):
        with open(tpath) as fh:
            traffic = json.load(fh)
    kernels = traffic["kernels"] if traffic else {}
    fam = {}
    for r in rows:
        cls = kernel_class(r["Name"])
        a = fam.setdefault(cls, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
    tot = sum(v[1] for v in fam.values()) or 1.0
    famb = {}
    for nm, v in kernels.items():
        b = famb.setdefault(kernel_class(nm), [0, 0.0])
        b[0] += v["dispatches"]
        b[1] += v["hbm_bytes_per_dispatch"] * v["dispatches"]
    lines = [f"# rocprofv3 kernel statistics: {workload}", "", "Commands (run from the repository root; `<raw>` is a "
             "scratch directory for rocprofv3's CSV output):", "", "```", commands.strip(), "```", "",
             f"HIP sources SHA-256 when taken: `{traffic['source_sha256'] if traffic else source_hash()}`", "",
             "## By kernel class", "", "| class | calls | total ms | avg us | % of GPU time | HBM MB/dispatch |",
             "|---|---|---|---|---|---|"]
    for cls, (n, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        hb = famb.get(cls)
        hbs = f"{hb[1] / hb[0] / 1e6:.2f}" if hb and hb[0] else "-"
        lines.append(f"| {cls} | {n} | {t / 1e6:.2f} | {t / n / 1e3:.2f} | {100 * t / tot:.1f} | {hbs} |")
    lines += ["", "## By kernel (top 16 by time)", "", "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:16]:
        lines.append(f"| `{_kname(r['Name'])[:100]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    if traffic:
        lines += ["", f"## HBM traffic (FETCH_SIZE, WRITE_SIZE)", "",
                  f"Copy calibration (1 GiB read + 1 GiB written per launch, `{traffic['copy_kernel']}`): FETCH_SIZE "
                  f"{traffic['copy_fetch_kib']:.0f} KiB, WRITE_SIZE {traffic['copy_write_kib']:.0f} KiB per dispatch -> "
                  f"scale {traffic['scale_fetch']:.4f} (fetch), {traffic['scale_write']:.4f} (write).", "",
                  "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB/dispatch |", "|---|---|---|---|---|"]
        for nm, v in sorted(kernels.items(), key=lambda kv: -kv[1]["hbm_bytes_per_dispatch"] * kv[1]["dispatches"])[:12]:
            lines.append(f"| `{_kname(nm)[:100]}` | {v['dispatches']} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | "
                         f"{v['hbm_bytes_per_dispatch'] / 1e6:.2f} |")
    with open(os.path.join(PROFILES, f"{workload}_kernels.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"wrote": [f"profiles/{workload}_kernels.md"] + ([f"profiles/{workload}_traffic.json"] if traffic else [])}))


def measured_traffic(workload, cls):
    """HBM bytes per launch of kernel class cls from the committed counter summary,
    or None when there is none or the kernels changed since it was taken."""
    path = os.path.join(PROFILES, f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != source_hash():
        return None
    hits = [v for nm, v in t["kernels"].items() if kernel_class(nm) == cls]
    if not hits:
        return None
    n = sum(v["dispatches"] for v in hits)
    return sum(v["hbm_bytes_per_dispatch"] * v["dispatches"] for v in hits) / max(n, 1)


def roofline(prof, workload):
    if not prof:
        return None, None
    # per-iteration classes are timed on a sample of their launches: rank classes by the
    # estimated total (average timed launch x launches issued)
    est = {k: v["ms"] / v["launches"] * v.get("issued", v["launches"]) for k, v in prof.items()}
    name = max(est, key=est.get)
    v = prof[name]

    def entry(nm, e):
        avg_s = e["ms"] / e["launches"] / 1e3
        per_launch = e["bytes"] / e["launches"]
        gbs = per_launch / avg_s / 1e9
        tr = measured_traffic(workload, nm)
        return {"kernel": nm, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": tr,
                "bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": e["launches"], "launches_issued": e.get("issued", e["launches"]),
                "share_of_gpu_time": round(est[nm] / sum(est.values()), 4)}

    apply_name = "apply_bj_fused" if "apply_bj_fused" in prof else ("apply" if "apply" in prof else None)
    apply = entry(apply_name, prof[apply_name]) if apply_name else None
    return entry(name, v), apply


def _oracle_sample_step(args):
    """One full oracle implicit step of the CPU sample (module-level: runs in worker
    processes for the all-core measurement).  Returns (seconds, converged, newton, krylov)."""
    workload, threads = args
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import m1_oracle as O

    q = WORKLOADS[workload]["cpu_sample"](W)
    solver = WORKLOADS[workload]["solver"]
    with threadpool_limits(limits=threads):
        sch = O.Scheme.from_problem(q)
        Un = O.state_from_problem(q)
        t0 = time.perf_counter()
        r = O.implicit_step(sch, q["sigma"], q.get("rho_cv"), Un, q["dt"], rtol=solver["rtol"],
                            newton_rtol=solver["newton_rtol"], newton_max=solver["newton_max"],
                            max_iters=solver["max_iters"], line_search=solver.get("line_search", False))
        t = time.perf_counter() - t0
    return t, bool(r.converged), int(r.newton_iters), int(r.krylov_iters)


def cpu_baseline(p, U0, results, workload):
    """The oracle beside the GPU: (1) full implicit steps (Newton to 1e-8, block-Jacobi
    GMRES(30) to 1e-8) of a reduced instance of the same generator, one process with one
    thread, then one process per core running the same step at once (aggregate rate);
    (2) the oracle's residual ||R(U)|| / ||R(U^n)|| of every variant's GPU result at full
    size (the error statement of each result)."""
    import concurrent.futures as cf

    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import m1_oracle as O

    out = {"kind": "oracle", "unit": "cell-updates/s"}
    make = WORKLOADS[workload]["cpu_sample"]
    if make is not None:
        q = make(W)
        Nq = int(np.prod(q["n"][:q["ndim"]]))
        t1, conv, nn, nk = _oracle_sample_step((workload, 1))
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = max(1, min(avail, 16))
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=cores) as ex:
            res = list(ex.map(_oracle_sample_step, [(workload, 1)] * cores))
        tall = time.perf_counter() - t0
        out.update({
            "value": Nq / t1, "cores": 1,
            "value_all_cores": cores * Nq / tall, "cores_all": cores, "cpus_available": avail,
            "nproc": os.cpu_count(),
            "sample": (f"one full oracle implicit step of {workload}'s generator at {'x'.join(map(str, q['n']))} "
                       f"(converged={conv}, {nn} Newton, {nk} Krylov iterations, {t1:.1f} s on one thread); "
                       f"all cores: {cores} processes running the same step at once, {tall:.1f} s"),
        })
    else:
        out.update({"value": None, "cores": 1, "sample": "no reduced instance converges (see the design notes)"})
    checks = {}
    rho_cv = p.get("rho_cv")
    with threadpool_limits(limits=1):
        sch = O.Scheme.from_problem(p)
        r0 = float(np.linalg.norm(O.residual(O.linearize(sch, p["sigma"], rho_cv, U0, U0, p["dt"]))))
        for name, v in results.items():
            lin = O.linearize(sch, p["sigma"], rho_cv, v["U"], U0, p["dt"])
            checks[name] = float(np.linalg.norm(O.residual(lin))) / r0
    out["oracle_residual_of_gpu_result"] = checks
    return out


TIME_STEP_METRIC = {
    "semi_implicit": "semi-implicit M1 cell-updates/s at the CFL time step (sources implicit)",
    "explicit": "explicit M1 cell-updates/s at the CFL time step",
}


def time_step_cpu_baseline(p, U0, scheme, dt):
    """The oracle's explicit / semi-implicit step on the whole grid, one step, 1 thread."""
    from threadpoolctl import threadpool_limits

    import numpy as np
    from oracle import m1_oracle as O

    N = int(np.prod(p["n"][:p["ndim"]]))
    what = "the whole grid"
    if N > (1 << 21):
        # a slab of whole planes along the slowest axis, outflow on its cut faces
        nz = p["n"][-1]
        k = max(1, (1 << 21) // (N // nz))
        q = dict(p, n=tuple(p["n"][:-1]) + (k,), bc=list(p["bc"]))
        q["bc"][2 * (p["ndim"] - 1)] = q["bc"][2 * (p["ndim"] - 1) + 1] = "outflow"
        q["ghost"] = {f: v for f, v in p["ghost"].items() if f < 2 * (p["ndim"] - 1)}
        q["ghost_mask"] = {f: v for f, v in p["ghost_mask"].items() if f < 2 * (p["ndim"] - 1)}
        for key in ("sigma", "rho_cv", "E", "T"):
            if q.get(key) is not None:
                q[key] = p[key][:k]
        q["F"] = p["F"][:, :k]
        p, U0 = q, U0[:, :k]
        what = f"a slab of {k} of the {nz} planes (outflow on the cut)"
    with threadpool_limits(limits=1):
        sch = O.Scheme.from_problem(p)
        f = O.semi_implicit_step if scheme == "semi_implicit" else O.explicit_step
        t0 = time.perf_counter()
        f(sch, p["sigma"], p.get("rho_cv"), U0, dt)
        t = time.perf_counter() - t0
    n_sample = int(np.prod(p["n"][:p["ndim"]]))
    return {"value": n_sample / t, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one oracle {scheme} step of {what}, {n_sample} cells ({t:.2f}s); BLAS limited to 1 thread"}


def time_step_bench(args):
    """Explicit or semi-implicit steps at the CFL time step c dt = dx / ndim; one
    timed step advances the workload's own dt (the interval one implicit step
    covers) in ceil(dt / dt_CFL) sub-steps, from the same initial state each time."""
    import math

    import numpy as np
    import torch

    import paper_2011_13926_amd as P
    import workloads as W

    workload = args.workload
    p = WORKLOADS[workload]["make"](W)
    if args.scheme == "semi_implicit":
        p["flux_source"] = "centered"
    U0 = state0(p)
    dt_cfl = p["dx"] / (p["c"] * p["ndim"])
    nsub = int(math.ceil(p["dt"] / dt_cfl - 1e-12))
    s = P.Solver(p, restart=1)
    f = s.semi_implicit_step if args.scheme == "semi_implicit" else s.explicit_step
    try:
        U0d = s.to_device(U0)
        U = U0d.clone()
        for _ in range(args.warmup):
            U.copy_(U0d)
            f(U, dt=dt_cfl, nsteps=nsub, raise_on_fail=False)
        torch.cuda.synchronize()
        s.profile_enable(not args.no_events)
        wall, statuses = 0.0, []
        for k in range(args.steps):
            U.copy_(U0d)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, sd = f(U, dt=dt_cfl, nsteps=nsub, raise_on_fail=False)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            statuses.append(st)
            print(f"[bench] {args.scheme} step {k}: {nsub} sub-steps status={st} {sd['seconds'] * 1e3:.2f} ms "
                  f"min E {float(U[0].min()):.3e}", file=sys.stderr, flush=True)
        prof = s.profile() if not args.no_events else {}
        s.profile_enable(False)
    finally:
        s.close()
    N = int(np.prod(p["n"][:p["ndim"]]))
    roof, _ = roofline(prof, workload + "_" + args.scheme)
    out = {
        "metric": TIME_STEP_METRIC[args.scheme],
        "value": N * nsub * args.steps / wall,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "grid": list(p["n"][:p["ndim"]]), "scheme": args.scheme,
                   "dt_cfl": dt_cfl, "substeps_per_step": nsub, "advanced_per_step": nsub * dt_cfl,
                   "flux_source": p["flux_source"], "lambda_floor": p["lambda_floor"]},
        "status": statuses,
        "roofline": roof,
        "kernels": prof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = time_step_cpu_baseline(p, U0, args.scheme, dt_cfl)
    print(json.dumps(out), flush=True)


BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA


def nn_flops(cin, cout, channels, H, W):
    """Multiply-add work (2 flops each) of one forward pass of the U-Net: per level two
    3x3 convolutions on the way down, two on the way up (after concatenating the
    upsampled coarser level with the skip), a 1x1 head."""
    f = 0.0
    prev = cin
    for l, c in enumerate(channels):
        hw = (H >> l) * (W >> l)
        f += 2.0 * 9 * prev * c * hw + 2.0 * 9 * c * c * hw
        prev = c
    for l in range(len(channels) - 2, -1, -1):
        hw = (H >> l) * (W >> l)
        c = channels[l]
        f += 2.0 * 9 * (channels[l + 1] + c) * c * hw + 2.0 * 9 * c * c * hw
    f += 2.0 * channels[0] * cout * H * W
    return f


def nn_bench(args):
    """Forward pass and training step of the 4-level U-Net (32/48/64/64 channels) at 512^2
    on random inputs; TFLOP/s from the layer specification (the backward pass counted as
    twice the forward: input and weight gradients)."""
    import numpy as np
    import torch

    import paper_2011_13926_amd as P
    H = W = 512
    ch = (32, 48, 64, 64)
    net = P.Net(9, 3, ch, Hmax=H, Wmax=W)
    net.init_params(seed=0, head_scale=0.1)
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.standard_normal((H, W, 9)), dtype=torch.float32, device="cuda")
    t = torch.as_tensor(rng.standard_normal((H, W, 3)), dtype=torch.float32, device="cuda")
    for _ in range(max(args.warmup, 1)):
        net.forward(x)
        net.train_step(x, t, 1e-6)
    torch.cuda.synchronize()
    reps = max(args.steps, 1) * 10
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, t, 1e-6)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    net.close()
    f = nn_flops(9, 3, ch, H, W)
    tf = f / t_fwd / 1e12
    out = {
        "metric": "learned-preconditioner U-Net forward TFLOP/s (BF16 MFMA, FP32 accumulate)",
        "value": tf, "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": 1e3 * t_fwd, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "unet_512", "grid": [H, W], "channels": list(ch), "cin": 9, "cout": 3,
                   "forward_gflop": f / 1e9},
        "forward_ms": 1e3 * t_fwd, "train_step_ms": 1e3 * t_train,
        "train_step_tflops": 3.0 * f / t_train / 1e12,
        "roofline": {"kernel": "forward pass", "bound": "mfma", "achieved": round(tf, 2), "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(tf / BF16_PEAK_TFLOPS, 4), "traffic": None},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.profile_name or args.workload, args.profile_commands)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.nn:
        nn_bench(args)
        return
    if args.scheme != "implicit":
        time_step_bench(args)
        return
    import numpy as np
    import torch

    import paper_2011_13926_amd as P
    import workloads as W

    workload = args.workload
    p = WORKLOADS[workload]["make"](W)
    U0 = state0(p)
    results = {}
    for name in [v for v in args.variants.split(",") if v]:
        results[name] = run_variant(P, torch, p, U0, name, args)
    # error of every result against the plain FP64 block-Jacobi result
    ref = results.get("fp64_bj")
    for name, v in results.items():
        if ref is None:
            v["error_vs_fp64_bj"] = None
            continue
        a, b = v["U"], ref["U"]
        v["error_vs_fp64_bj"] = {
            "rel_l2": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
            "max_abs_by_component": [float(np.max(np.abs(a[c] - b[c])) / max(np.max(np.abs(b[c])), 1e-300))
                                     for c in range(b.shape[0])],
        }
    # the headline: mixed precision with an FP64 Krylov basis (the FP32-stored basis is a
    # separate variant, reported but not picked)
    mixed = {k: v for k, v in results.items()
             if k.startswith("mixed") and not VARIANTS[k].get("basis_fp32") and v["converged_all"]}
    pick = max(mixed, key=lambda k: mixed[k]["cell_updates_per_s"]) if mixed else None
    head = results[pick] if pick else None
    base = results.get("fp64_bj")
    # kernel rooflines: of the headline variant, else (no variant converged) of the first one run
    rname = pick or next(iter(results), None)
    rsrc = results[rname] if rname else None
    roof, roof_apply = roofline(rsrc["kernels"] if rsrc else {}, workload)
    out = {
        "metric": METRIC,
        "value": head["cell_updates_per_s"] if head else None,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"] if head else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[pick] if pick else None,
        "data": "synthetic",
        "config": {"workload": workload, "grid": list(p["n"][:p["ndim"]]), "dt_over_cfl": p["dt"],
                   "flux_source": p["flux_source"], "lambda_floor": p["lambda_floor"], "variant": pick,
                   "restart": 30, **WORKLOADS[workload]["solver"],
                   "preconditioner": VARIANTS[pick].get("pc") if pick else None},
        "converged": bool(head and head["converged_all"]),
        "admissible": bool(head and head["admissible"]),
        "speedup_vs_plain_fp64_bj": (head["cell_updates_per_s"] / base["cell_updates_per_s"]
                                     if head and base and base["converged_all"] else None),
        "variants": {k: {kk: vv for kk, vv in v.items() if kk not in ("kernels", "U")} for k, v in results.items()},
        "roofline": roof,
        "roofline_apply": roof_apply,
        "roofline_variant": rname,
        "kernels": rsrc["kernels"] if rsrc else None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, U0, results, workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
