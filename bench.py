"""Benchmark of the SPH hot path on one MI355X.

One step = build_cells -> sort_cells -> mark_active(m) -> density_pass ->
force_pass -> kick_drift on the clustered workload (2,097,152 particles: 90 %
uniform background, 10 % in 20 Plummer spheres, u log-uniform, 14 model
time-bins), at the deep bin m whose active set {bin <= m} is closest to 1 %
of the particles.  Steps run at integer times t with ctz(t) = m, so the active
set keeps its size from step to step; each step advances time by the step of
bin m, 2^m t_min.

Prints one JSON line: interactions/s (density + force, in-support pairs only,
counted by the kernels) over the whole step, the fraction of FP32 vector peak,
the roofline of the dominant kernel, and the FP64 oracle's rate on a bounded
sample of the same step on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK = 157.3e12      # MI355X FP32 vector, FLOP/s
FP32_UNPACKED = 78.6e12   # one FMA per lane per clock (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
HBM_PEAK = 8.0e12         # bytes/s
# algorithmic FLOP per interaction of the two loops (mul/add = 1, fma = 2,
# rsqrt/rcp = 1, compare/select = 0), counted from the pair formulas
FLOP_DENSITY = 60
FLOP_FORCE = 72


def kernel_model(name, n, n_active, n_leaves, n_dens, n_force, launches):
    """Algorithmic bytes (hbm) or flops (alu) of ONE launch of a kernel group,
    for the roofline of the dominant kernel."""
    if name == "density_loop":
        return "alu", FLOP_DENSITY * n_dens / launches
    if name == "force_loop":
        return "alu", FLOP_FORCE * n_force / launches
    if name == "radix_scatter":
        return "hbm", 24.0 * n             # read key+value, write key+value
    if name == "radix_hist":
        return "hbm", 8.0 * n
    if name == "permute":
        return "hbm", None
    if name == "axis_sort":
        return "hbm", (16.0 + 13 * 2.0) * n  # read offsets, write 13 uint16 orders
    if name == "kick_drift":
        return "hbm", n * (2 * 9 * 8 + 2 * 2 * 4 + 6 * 4 + 1)
    if name == "morton_keys":
        return "hbm", n * (3 * 8 * 2 + 4 + 8 + 4)
    if name == "offsets":
        return "hbm", n * (3 * 8 + 4 + 4 + 16)
    return "hbm", None


def run_cpu_baseline(ic, active_orig, n_sample, seed=5):
    """The FP64 oracle, unchanged, on a sample of the step's active particles:
    density solve for the sample and every particle within reach of it, force
    loop for the sample.  Rate = the sample's in-support interactions / time."""
    import torch

    from oracle import sph
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(active_orig, size=min(n_sample, active_orig.size), replace=False))
    t0 = time.perf_counter()
    from scipy.spatial import cKDTree
    tree = cKDTree(ic["x"], boxsize=1.0)
    reach = 2.0 * sph.GAMMA_K * float(ic["h"].max()) * 1.5
    near = np.unique(np.concatenate(tree.query_ball_point(ic["x"][sample], reach)))
    dens = sph.density_and_ghost(ic["x"], ic["v"], ic["m"], ic["h"], 1.0, u=ic["u"], centres=near)
    N = ic["x"].shape[0]
    full = {}
    for k in ("h", "rho", "f", "P", "c", "B"):
        a = torch.full((N,), float("nan"), dtype=torch.float64)
        a[torch.as_tensor(near)] = dens[k]
        full[k] = a
    fo = sph.force(ic["x"], ic["v"], ic["m"], full["h"], full["rho"], full["f"], full["P"], full["c"], full["B"],
                   1.0, centres=sample)
    t = time.perf_counter() - t0
    pos = np.searchsorted(near, sample)
    inter = int(dens["count"].numpy()[pos].sum() + fo["count"].numpy().sum())
    return dict(value=inter / t, unit="interactions/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{sample.size} active particles of the step (density solve for the {near.size} particles "
                       f"within reach, force for the sample), {inter} interactions in {t:.1f} s",
                seconds=t)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--active-fraction", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=24)
    ap.add_argument("--split", type=int, default=None)
    ap.add_argument("--cand-cap", type=int, default=None)
    ap.add_argument("--list-cap", type=int, default=None)
    ap.add_argument("--profile-steps", type=int, default=None)
    ap.add_argument("--h-tol", type=float, default=None)
    ap.add_argument("--nw", type=int, default=None)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "gpurun_out", "tuning_clustered.txt"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU decomposition "
                                   "is design-only)"}))
        sys.exit(2)

    import torch

    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()

    ic = ics.clustered()
    N = ic["x"].shape[0]
    m = ics.deep_bin_for_fraction(ic["bin"], args.active_fraction)
    t_min = ic["t_min_model"]
    kw = {}
    if args.split:
        kw["split_count"] = args.split
    if args.cand_cap:
        kw["cand_cap"] = args.cand_cap
    if args.list_cap:
        kw["list_cap"] = args.list_cap
    if args.h_tol:
        kw["h_tol"] = args.h_tol
    if args.nw:
        kw["waves_per_chunk"] = args.nw
    ctx = sg.Context(**kw)
    p = sg.Particles.from_initial(ic)

    # setup (untimed): every particle gets its density-loop state once
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, ics.N_BINS - 1)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    ctx.sync()

    def step(s):
        ti = (2 * s + 1) << m
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, m, want_count=False)
        ctx.density_pass(p, entropy_from_u=False)
        ctx.force_pass(p)
        ctx.kick_drift(p, ti, t_min, 1 << m, False)

    tuned = None
    if not args.no_tune:
        # one step whose loops are tuned on the step's own active chunks
        ti = 1 << m
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, m, want_count=False)
        ctx.density_pass(p, entropy_from_u=False)
        ctx.force_pass(p)
        os.makedirs(os.path.dirname(args.tune_file), exist_ok=True)
        if os.path.exists(args.tune_file):
            os.remove(args.tune_file)
        ctx.autotune(p, args.tune_file)
        tuned = [l.split() for l in open(args.tune_file) if l.startswith("best")]
        ctx.kick_drift(p, ti, t_min, 1 << m, False)

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    inf0 = ctx.info()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        step(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inf1 = ctx.info()
    wall = t1 - t0
    I_d = inf1["interactions_density"] - inf0["interactions_density"]
    I_f = inf1["interactions_force"] - inf0["interactions_force"]
    inter = I_d + I_f
    value = inter / wall

    # the same steps again with HIP events around every launch of the library
    ksteps = args.profile_steps or args.steps
    ctx.profile(True)
    t2 = time.perf_counter()
    for s in range(args.warmup + args.steps, args.warmup + args.steps + ksteps):
        step(s)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = ctx.profile_read()
    last = ctx.info()
    ctx.profile(False)
    inf2 = ctx.info()
    I_d2 = inf2["interactions_density"] - inf1["interactions_density"]
    I_f2 = inf2["interactions_force"] - inf1["interactions_force"]
    kernels = {k: {"launches": c, "ms_total": round(ms, 4), "ms_per_step": round(ms / ksteps, 4)}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    cnt, ms = prof[dom]
    bound, per_launch = kernel_model(dom, N, inf2["n_active"], inf2["n_leaves"], I_d2, I_f2, cnt)
    roof = None
    if per_launch is not None:
        dur = ms / 1e3 / cnt
        achieved = per_launch / dur
        if bound == "alu":
            roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
                    "frac": achieved / FP32_PEAK, "traffic": None, "kernel": dom}
        else:
            roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": None, "kernel": dom}
    loop_ms = sum(prof.get(k, (0, 0.0))[1] for k in ("density_loop", "force_loop")) / ksteps
    flops_step = (FLOP_DENSITY * I_d + FLOP_FORCE * I_f) / args.steps
    out = {
        "metric": "active particle-neighbour interactions/s (density+force), % FP32 peak, vs plain",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 positions/integration",
        "data": "synthetic",
        "config": {"workload": f"clustered {N} particles (90% uniform + 10% in 20 Plummer spheres, "
                               f"a in [0.002,0.02], u log-uniform 1e-2..1e2, 14 bins), deep-bin step m={m}",
                   "n_particles": N, "max_active_bin": m, "n_active": inf1["n_active"],
                   "active_fraction": inf1["n_active"] / N, "n_leaves": inf1["n_leaves"],
                   "split_count": ctx.params.split_count},
        "interactions_per_step": inter / args.steps,
        "fp32_peak_frac_step": flops_step / (wall / args.steps) / FP32_PEAK,
        "fp32_peak_frac_loops": (flops_step / (loop_ms / 1e3) / FP32_PEAK) if loop_ms > 0 else None,
        "loops_rate_interactions_per_s": ((I_d2 + I_f2) / ksteps) / (loop_ms / 1e3) if loop_ms > 0 else None,
        "profiled_ms_per_step": (t3 - t2) / ksteps * 1e3,
        "last_step_newton": {"unconverged_after_pass": last["unconverged_after_pass"],
                             "pair_rebuilds": last["pair_rebuilds"]},
        "kernels": kernels,
        "tuned_loops": [{"loop": ("density", "force")[int(t[1])], "chunk_class": int(t[2]), "waves_per_chunk": int(t[3]),
                         "tile": int(t[4]), "cost_ordered": int(t[5]), "persistent": int(t[6]), "ms": float(t[7])}
                        for t in (tuned or [])],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        act = ic["bin"] <= m
        out["cpu_baseline"] = run_cpu_baseline(ic, np.nonzero(act)[0], args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
