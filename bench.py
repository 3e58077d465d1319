"""Benchmark: EXX pair Poisson solves/s and EXX evaluation time on one MI355X.

A step is one full exx_eval (pair list, pair densities, moments, boundary
values, CG solves, E_xx, D_xx and sigma_xx) over every pair of a water-like
workload, with the orbitals already resident in HBM.  The default workload is
the 64-molecule set (cubic 23.5 bohr cell, 120^3 grid, 256 orbitals, R_pair
10, R_PE 6, R_ME 9 bohr, l_max 6, 19-point stencil, CG tol 1e-10), timed in
FP64 and in mixed precision; the mixed figure is the headline value.  Prints
one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision both|fp64|mixed]
                  [--workload water64|water128|water256|water512|hex64|tri64]

water256 runs as the MD-like repeated-call case: per-orbital sphere radii (9
classes), a fixed pair capacity, one eager warm-up call (which runs the CG
autotuner), the call recorded into a HIP graph, then K replays; before each
replay every centre moves 0.02 bohr and the orbitals are regenerated on the
device in the same buffers (not timed).  Each replay is timed with HIP events.
By default each replay's CG starts from the pair's solution of the previous
replay (--no-warm-start: from zero).

The roofline entry is for the dominant kernel, the persistent CG solve:
algorithmic bytes (8 N_PE b per pair per iteration) over the summed device
time of its launches in the timed region, from HIP events that the library
records on its stream (eager calls only).  moments_roofline gives the moment
contraction's matrix-core rate.  The CPU baseline is the FP64 oracle on a
deterministic pair subset of the same workload, on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 2500.0}   # dense FP64 and BF16 matrix peaks
METRIC = "EXX pair Poisson solves/s + EXX eval time, mixed vs FP64 at 1e-6 tol"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve_traffic.json")
# sources of the CG kernel, its launch shape and its data layout: the stored
# counter traffic is used only while these are unchanged
KERNEL_SOURCES = ["paper_2011_07209_amd/csrc/solve_impl.h", "paper_2011_07209_amd/csrc/solve.hip",
                  "paper_2011_07209_amd/csrc/solve_n1.hip", "paper_2011_07209_amd/csrc/solve_n2.hip",
                  "paper_2011_07209_amd/csrc/solve_n3.hip", "paper_2011_07209_amd/csrc/exx_internal.h",
                  "paper_2011_07209_amd/csrc/plan_geometry.cpp"]
MOLECULES = {"water64": 64, "water128": 128, "water256": 256, "water512": 512, "hex64": 64, "tri64": 64}
D_CHECK_ROWS = 16   # orbitals whose D the mixed/FP64 comparison uses


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, precision: str, threads: int, depth: int, layout: int):
    """HBM bytes per solve launch from the committed counter runs, or None when
    the kernels changed since they were taken or the run used another CG
    variant (workgroup size, load depth, column or quad layout) than the one
    measured."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/{precision}")
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    args = [a.strip() for a in e.get("kernel", "").split("<", 1)[-1].rstrip(">").split(",")]
    if len(args) < 7 or args[2] != str(threads) or args[3] != str(depth):
        return None
    if (args[6] == "true") != (layout == 2):
        return None
    return e.get("hbm_bytes_per_launch")


def describe(cfg) -> str:
    grid = "x".join(str(n) for n in cfg.grid)
    cell = "x".join(f"{x:g}" for x in cfg.cell)
    if cfg.general:
        import numpy as np
        h = cfg.h
        ang = [math.degrees(math.acos(np.dot(h[:, i], h[:, j]) / np.linalg.norm(h[:, i]) / np.linalg.norm(h[:, j])))
               for i, j in ((1, 2), (0, 2), (0, 1))]
        cell += " (angles " + "/".join(f"{x:.0f}" for x in ang) + " deg, NK Laplacian)"
    radii = (f"R_PE {cfg.R_orb_range[0]:g}-{cfg.R_orb_range[1]:g} per orbital ({cfg.R_PE_classes[2]} classes)"
             if cfg.R_PE_classes else f"R_PE {cfg.R_PE:g}")
    return (f"{cfg.key}: water-like {MOLECULES[cfg.key]}-molecule set, {cfg.lattice} lattice, cell {cell} bohr, "
            f"{grid} grid, {cfg.n_orb} orbitals ({cfg.orb_dtype}), R_pair {cfg.R_pair:g}, {radii}, "
            f"R_ME {cfg.R_ME:g}, l_max {cfg.l_max}, n {cfg.stencil_n}, CG tol {cfg.cg_tol:g}")


def cpu_baseline(cfg, orbs, phi, n_pairs_total, sample_pairs: int):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    frac = min(1.0, sample_pairs / max(1, n_pairs_total))
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol,
                           sample_seed=2011072092, sample_frac=frac, n_threads=threads)
    t0 = time.perf_counter()
    r = oracle.evaluate(P, phi, orbs.centres, want_D=True)
    dt = time.perf_counter() - t0
    n = len(r["pairs"])
    return {"value": n / dt, "unit": "pair solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {n_pairs_total} pairs (SplitMix64 subset, seed 2011072092), full E/D/sigma per pair, "
                      f"{dt:.1f} s"}


def _plan(exx, cfg, precision, **kw):
    opt = dict(stencil_n=cfg.stencil_n, cg_tol=cfg.cg_tol,
               precision=exx.EXX_PREC_MIXED if precision == "mixed" else exx.EXX_PREC_FP64,
               workspace_gb=24.0 if cfg.key == "water512" else 48.0)
    if cfg.R_PE_classes is not None:
        opt.update(R_PE_min=cfg.R_PE_classes[0], R_PE_step=cfg.R_PE_classes[1], R_PE_nclass=cfg.R_PE_classes[2])
    opt.update(kw)
    return exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **opt)


def run_precision(exx, torch, synth, cfg, orbs, bufs, precision, steps, warmup, graph, warm=False):
    """Times `steps` evaluations (after `warmup`) in one precision; returns the
    measurement and the outputs of the last evaluation."""
    orb_t, cen_t, R_t, D = bufs
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    kw = {"autotune": 1 if warmup > 0 else 0}
    if graph:
        probe = _plan(exx, cfg, precision)
        n0 = probe.count_pairs(cen_t, R_t)
        probe.close()
        kw["max_pairs"] = int(math.ceil(1.05 * n0)) + 64   # displacements change the pair list a little
        kw["warm_start"] = 1 if warm else 0
    plan = _plan(exx, cfg, precision, **kw)
    geo = plan.geometry()
    n_warm = max(warmup, 1 if graph else 0)
    for w in range(n_warm):
        plan.eval(orb_t, cen_t, E, D, S, R_t)
        torch.cuda.synchronize()
        print(f"[bench] {cfg.key} {precision} warmup {w + 1}/{n_warm} E={E.item():.10f}", file=sys.stderr, flush=True)
    zero = {"solve_launches": 0, "solve_ms_total": 0.0, "cg_alg_bytes_total": 0.0}
    s0 = plan.stats() if n_warm > 0 else zero
    step_ms, step_pairs, step_iters, step_warm = [], [], [], []
    s_last = None
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            plan.set_stream(side)
            with torch.cuda.graph(g, stream=side):
                plan.eval(orb_t, cen_t, E, D, S, R_t)
        torch.cuda.current_stream().wait_stream(side)
        plan.set_stream(torch.cuda.current_stream())
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        traj = orbs
        for k in range(steps):
            traj = synth.displace(cfg, traj, k + 1)
            synth.fill_orbitals_device(cfg, traj, dev, out=orb_t)
            cen_t.copy_(torch.from_numpy(traj.centres).to(dev))
            torch.cuda.synchronize()
            ev0.record()
            g.replay()
            ev1.record()
            torch.cuda.synchronize()
            st = plan.stats()
            step_ms.append(ev0.elapsed_time(ev1))
            step_pairs.append(st["n_pairs"])
            step_iters.append(st["cg_iter_sum"] / max(1, st["n_pairs"]))
            step_warm.append(st["warm_pairs"])
            s_last = st
            print(f"[bench] {cfg.key} {precision} replay {k + 1}/{steps}: {step_ms[-1]:.1f} ms, {st['n_pairs']} pairs "
                  f"({st['warm_pairs']} warm-started), mean iterations {step_iters[-1]:.1f}, E={E.item():.10f}",
                  file=sys.stderr, flush=True)
        del g
        ms = sum(step_ms) / len(step_ms)
        value = sum(step_pairs) / (sum(step_ms) / 1000.0)
        cg = None   # replays record no per-kernel events
    else:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.eval(orb_t, cen_t, E, D, S, R_t)
            st = plan.stats()            # waits for the evaluation; device times of this one
            step_ms.append(st["eval_ms"])
            step_pairs.append(st["n_pairs"])
            s_last = st
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1000.0 / steps
        value = s_last["n_pairs"] / (ms / 1000.0)
        launches = s_last["solve_launches"] - s0["solve_launches"]
        solve_ms = s_last["solve_ms_total"] - s0["solve_ms_total"]
        alg = s_last["cg_alg_bytes_total"] - s0["cg_alg_bytes_total"]
        achieved = (alg / max(launches, 1)) / (solve_ms / max(launches, 1) / 1000.0) / 1e9 if solve_ms > 0 else 0.0
        cg = {"bound": "hbm", "kernel": "k_solve_mixed" if precision == "mixed" else "k_solve",
              "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
              "traffic": stored_traffic(cfg.key, precision, s_last["solve_threads"], s_last["solve_depth"],
                                        s_last["cg_layout"]),
              "alg_bytes_per_launch": alg / max(launches, 1),
              "launch_ms": solve_ms / max(launches, 1)}
    print(f"[bench] {cfg.key} {precision} timed {steps} steps: {ms:.1f} ms/step E={E.item():.10f}", file=sys.stderr,
          flush=True)
    moments = None
    if s_last["moment_ms"] > 0:
        # moment contraction of the last evaluation: executed MFMA flops (padded
        # rows and points, three products in the mixed path) and the algorithmic
        # 2 N_lm N_PE per pair, over the device time of its launches
        mom_s = s_last["moment_ms"] / 1000.0
        mfma = s_last["moment_mfma_flops"] / mom_s / 1e12
        alg_tf = s_last["moment_flops"] / mom_s / 1e12
        peak = MFMA_PEAK_TFLOPS[precision]
        moments = {"bound": "mfma", "kernel": "k_moments_bf16" if precision == "mixed" else "k_moments_f64",
                   "achieved": mfma, "peak": peak, "unit": "TFLOP/s", "frac": mfma / peak,
                   "algorithmic_tflops": alg_tf, "algorithmic_frac": alg_tf / peak,
                   "density_read_gbs": 8.0 * s_last["moment_flops"] / (2.0 * (cfg.l_max + 1) ** 2) / mom_s / 1e9,
                   "launch_ms": s_last["moment_ms"]}
    plan.close()
    n_pairs = s_last["n_pairs"]
    return {
        "value": value, "ms_per_step": ms, "n_pairs": n_pairs, "n_pe": geo["n_pe"],
        "eval_ms_median": statistics.median(step_ms), "eval_ms_steps": step_ms,
        "cg_iters_mean_steps": step_iters, "warm_pairs_steps": step_warm,
        "cg_iters_mean": s_last["cg_iter_sum"] / max(1, n_pairs), "cg_iters_max": s_last["cg_iter_max"],
        "updates_max": s_last["refine_passes_max"], "max_rel_residual": s_last["max_rel_residual"],
        "solve_variant": {"threads": s_last["solve_threads"], "depth": s_last["solve_depth"],
                          "layout": "quads" if s_last["cg_layout"] == 2 else "columns", "tune_ms": s_last["tune_ms"]},
        "roofline": cg, "moments_roofline": moments,
        "E": E.item(), "sigma": S.cpu().numpy().reshape(3, 3, order="F"),
        "D_rows": D[:D_CHECK_ROWS].double().cpu(),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 5; 10 replays for water256)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(MOLECULES), default="water64")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both",
                    help="both: time the FP64 and the mixed path, report the mixed one as the value")
    ap.add_argument("--cpu-sample-pairs", type=int, default=640)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="water256: start every replay's CG from zero instead of the previous solution")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="after the timed steps, copy this many GiB device-to-device (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU pair sharding is "
              f"a design, not part of this build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2011_07209_amd import exx, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    cfg = synth.CONFIGS[args.workload]
    graph = cfg.key == "water256"
    steps = args.steps if args.steps is not None else (10 if graph else 5)
    orbs = synth.make_orbitals(cfg)
    t0 = time.perf_counter()
    orb_t = synth.fill_orbitals_device(cfg, orbs, dev)
    cen_t = torch.from_numpy(orbs.centres).to(dev)
    R_t = torch.from_numpy(orbs.R_orb).to(dev) if cfg.R_PE_classes is not None else None
    D = torch.empty_like(orb_t)
    torch.cuda.synchronize()
    print(f"[bench] {cfg.key}: {orb_t.numel() * orb_t.element_size() / 1e9:.1f} GB of orbitals generated on the "
          f"device in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precs:
        if graph:   # every precision replays the same trajectory from the same start
            synth.fill_orbitals_device(cfg, orbs, dev, out=orb_t)
            cen_t.copy_(torch.from_numpy(orbs.centres).to(dev))
        res[p] = run_precision(exx, torch, synth, cfg, orbs, (orb_t, cen_t, R_t, D), p, steps, args.warmup, graph,
                               warm=graph and not args.no_warm_start)
    main_p = "mixed" if "mixed" in res else "fp64"
    r = res[main_p]

    accuracy = None
    if "fp64" in res and "mixed" in res:
        a, b = res["mixed"], res["fp64"]
        n_mol = MOLECULES[cfg.key]
        accuracy = {
            "vs": "FP64 GPU path (itself parity-tested against the FP64 oracle)",
            "dE_Ha_per_molecule": abs(a["E"] - b["E"]) / n_mol,
            "sigma_rel_1norm": float(np.abs(a["sigma"] - b["sigma"]).sum() / np.abs(b["sigma"]).sum()),
            "D_rel_1norm": float((a["D_rows"] - b["D_rows"]).abs().sum().item() / b["D_rows"].abs().sum().item()),
            "D_rows_compared": D_CHECK_ROWS,
            "targets": {"dE_Ha_per_molecule": 1e-6, "sigma_rel_1norm": 1e-6},
        }

    if args.copy_probe_gib > 0:
        nbytes = int(args.copy_probe_gib * (1 << 30))
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline and cfg.key == "water64":
        phi = orb_t.cpu().numpy()   # exactly the inputs the GPU path read
        cpu = cpu_baseline(cfg, orbs, phi, r["n_pairs"], args.cpu_sample_pairs)
        del phi

    def summary(x):
        return {k: x[k] for k in ("value", "ms_per_step", "eval_ms_median", "eval_ms_steps", "cg_iters_mean_steps",
                                  "warm_pairs_steps", "cg_iters_mean",
                                  "cg_iters_max", "updates_max", "max_rel_residual", "solve_variant", "roofline",
                                  "moments_roofline")}

    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "pair solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": describe(cfg),
            "precision": main_p,
            "n_pairs": r["n_pairs"],
            "n_pe": r["n_pe"],
            "exx_eval_s": r["ms_per_step"] / 1000.0,
            "timing": ("mean of event-timed graph replays over displaced centres (orbital regeneration not timed)"
                       if graph else "host clock around the timed exx_eval calls"),
            "warm_start": bool(graph and not args.no_warm_start),
            "E_xx": r["E"],
        },
        "roofline": r["roofline"],
        "moments_roofline": r["moments_roofline"],
        "cpu_baseline": cpu,
        "by_precision": {p: summary(x) for p, x in res.items()},
        "mixed_accuracy": accuracy,
    }
    if "fp64" in res and "mixed" in res:
        out["mixed_speedup_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
