"""Benchmark of the SPH hot path on one MI355X.

One step = build_cells -> sort_cells -> mark_active(m) -> density_pass ->
force_pass -> kick_drift on the clustered workload (2,097,152 particles: 90 %
uniform background, 10 % in 20 Plummer spheres, u log-uniform, 14 model
time-bins), at the deep bin m whose active set {bin <= m} is closest to 1 %
of the particles.  The step's input is the state one deep-bin drift after an
all-active density + force pass (positions moved, h predicted); every timed
step starts from that input (a fused device copy of the arrays a step
changes, inside the timed region) and runs the whole path on it, so all
steps do the same work.

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
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK = 157.3e12      # MI355X FP32 vector, FLOP/s
FP32_UNPACKED = 78.6e12   # one FMA per lane per clock (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
HBM_PEAK = 8.0e12         # bytes/s
# HBM traffic of the loop kernels per launch, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a plain 512 MiB
# copy (profiles/force_sweep_deepbin_pmc.md, profiles/density_sweep_deepbin_pmc.md),
# valid while the kernels' sources are the ones that were measured (else
# reported as null)
MEASURED_TRAFFIC = {
    "force_loop": {"bytes": 15783444.0,
                   "sources": ["paper_1807_01341_amd/csrc/loops.hip", "paper_1807_01341_amd/csrc/loops_common.h",
                               "paper_1807_01341_amd/csrc/sph_internal.h"],
                   "sha256": "ed72f7189f6ec3482c3075fe0b2d365e4dba243ddbb5eb553b5bebed380fb013"},
    "density_loop": {"bytes": 10457098.0,
                     "sources": ["paper_1807_01341_amd/csrc/loops.hip", "paper_1807_01341_amd/csrc/loops_common.h",
                                 "paper_1807_01341_amd/csrc/sph_internal.h"],
                     "sha256": "ed72f7189f6ec3482c3075fe0b2d365e4dba243ddbb5eb553b5bebed380fb013"},
}


def measured_traffic(kernel):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return m["bytes"] if h.hexdigest() == m["sha256"] else None


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


def _loops_ms(prof):
    return sum(prof.get(k, (0, 0.0))[1] for k in ("density_loop", "force_loop"))


def measure_all_active(sg, ic, reps=3, **kw):
    """All-active density + force on the same clustered particles (a fresh
    context with the step's parameters): the loops at full occupancy, for the
    ALU roofline."""
    import torch
    ctx = sg.Context(**kw)
    p = sg.Particles.from_initial(ic)
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    ctx.autotune(p, None)
    ctx.sync()
    i0 = ctx.info()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.density_pass(p, entropy_from_u=False)
        ctx.force_pass(p)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    prof = ctx.profile_read()
    ctx.profile(False)
    i1 = ctx.info()
    I_d = (i1["interactions_density"] - i0["interactions_density"]) / reps
    I_f = (i1["interactions_force"] - i0["interactions_force"]) / reps
    d_cnt, d_ms = prof["density_loop"]
    f_cnt, f_ms = prof["force_loop"]
    dens_rate = FLOP_DENSITY * I_d * reps / (d_ms / 1e3)
    force_rate = FLOP_FORCE * I_f * reps / (f_ms / 1e3)
    return {
        "workload": "the same 2,097,152 clustered particles, all active (density from A at converged h, then force)",
        "interactions_per_pass": I_d + I_f,
        "ms_density_plus_force": wall * 1e3,
        "interactions_per_s": (I_d + I_f) / wall,
        "newton_passes": i1["density_iterations"],
        "density_loop": {"launches_per_pass": d_cnt / reps, "ms_per_launch": d_ms / d_cnt,
                         "tflops": dens_rate / 1e12, "fp32_peak_frac": dens_rate / FP32_PEAK},
        "force_loop": {"launches_per_pass": f_cnt / reps, "ms_per_launch": f_ms / f_cnt,
                       "tflops": force_rate / 1e12, "fp32_peak_frac": force_rate / FP32_PEAK},
    }


def measure_batch(sg, reps=5):
    """64 boxes (N log-uniform in [1e3, 2e5], one clump each, per-box active
    fraction): density + force of every box as 64 separate passes, then as
    batched passes (one launch per loop pass over all boxes) with the batch
    autotuner's tiling.  Same contexts, converged h, timed alternately."""
    import torch

    import ics
    boxes = ics.batch_of_boxes()
    cs, ps = [], []
    n_act = 0
    for b in boxes:
        p = sg.Particles.from_initial(b)
        c = sg.Context()
        c.build_cells(p)
        c.sort_cells()
        c.mark_active(p, c.params.n_bins - 1)
        c.density_pass(p, True)
        n_act += c.mark_active(p, ics.deep_bin_for_fraction(b["bin"], b["target_active_fraction"]))
        cs.append(c)
        ps.append(p)
    batch = sg.Batch(cs, ps)
    batch.density_pass(False)
    batch.force_pass()
    batch.autotune(None)

    def separate():
        for c, p in zip(cs, ps):
            c.density_pass(p, False)
            c.force_pass(p)

    def batched():
        batch.density_pass(False)
        batch.force_pass()

    def counts():
        return sum(c.info()["interactions_density"] + c.info()["interactions_force"] for c in cs)

    t_sep, t_bat = [], []
    inter = None
    for _ in range(reps):
        for fn, acc in ((separate, t_sep), (batched, t_bat)):
            torch.cuda.synchronize()
            k0 = counts()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            acc.append(time.perf_counter() - t0)
            inter = counts() - k0
    ts, tb = float(np.median(t_sep)), float(np.median(t_bat))
    return {
        "workload": f"64 boxes, {sum(b['x'].shape[0] for b in boxes)} particles, {n_act} active",
        "interactions_per_pass": inter,
        "ms_separate_64_passes": ts * 1e3,
        "ms_batched": tb * 1e3,
        "speedup": ts / tb,
        "interactions_per_s_batched": inter / tb,
        "interactions_per_s_separate": inter / ts,
    }


def measure_adjoint(sg, reps=5):
    """Differentiation workload (32,768 particles, all active): forward
    (build, density, force) and backward (sph_adjoint) of SPHForce."""
    import torch

    import ics
    ic = ics.differentiation()
    dev = torch.device("cuda")
    x = torch.tensor(ic["x"], dtype=torch.float64, device=dev, requires_grad=True)
    u = torch.tensor(ic["u"], dtype=torch.float32, device=dev, requires_grad=True)
    v = torch.tensor(ic["v"], dtype=torch.float64, device=dev)
    m = torch.tensor(ic["m"], dtype=torch.float32, device=dev)
    h = torch.tensor(ic["h"], dtype=torch.float32, device=dev)
    w = torch.tensor(ic["w"], dtype=torch.float32, device=dev)
    ctx = sg.Context()
    tf, tb = [], []
    for r in range(reps + 1):
        x.grad = None
        u.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = sg.SPHForce.apply(x, u, v, m, h, ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (a * w).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r > 0:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
    return {"workload": "32,768 particles (31^3 jittered lattice + 2,977-particle clump), all active, "
                        "L = sum w.a with seeded Gaussian w",
            "ms_forward": float(np.median(tf)) * 1e3, "ms_backward": float(np.median(tb)) * 1e3,
            "backward_over_forward": float(np.median(tb) / np.median(tf))}



def run_large(args):
    """Large single-GPU share: 256^3 lattice displaced by a Zel'dovich
    Gaussian random field (P(k) ~ k^-2.5), u log-uniform, 14 model bins.
    (i) all-active steps; (ii) one top-level step of `substeps` sub-steps
    t = 1.. with max active bin min(ctz(t), 13), each a full step (build,
    sort, mark, density, force, kick_drift by t_min)."""
    import torch

    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()
    t_gen = time.perf_counter()
    ic = ics.grf_zeldovich(amplitude=args.grf_amplitude)
    print(f"generated {ic['x'].shape[0]} particles in {time.perf_counter() - t_gen:.0f} s", file=sys.stderr,
          flush=True)
    N = ic["x"].shape[0]
    ctx = sg.Context(lazy_drift=int(args.lazy_drift))
    p = sg.Particles.from_initial(ic)
    del ic
    top = ctx.params.n_bins - 1
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, top)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    ctx.autotune(p, None)
    # t_min = the smallest Eq. 1 time-step of the converged state, so that
    # every particle's bin satisfies its own Courant condition
    vs = p["vsig"].double()
    dt = torch.where(vs > 0, ctx.params.cfl * p["h"].double() / vs, torch.full_like(vs, float("inf")))
    t_min = float(dt.min())
    ctx.kick_drift(p, 0, t_min, 0, True)
    ctx.sync()
    # (i) all-active steps (no time advance: the kick_drift of the sweep does that)
    reps = 3
    i0 = ctx.info()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, top, want_count=False)
        ctx.density_pass(p, entropy_from_u=False)
        ctx.force_pass(p)
    torch.cuda.synchronize()
    wall_all = (time.perf_counter() - t0) / reps
    prof = ctx.profile_read()
    ctx.profile(False)
    i1 = ctx.info()
    I_d = (i1["interactions_density"] - i0["interactions_density"]) / reps
    I_f = (i1["interactions_force"] - i0["interactions_force"]) / reps
    d_cnt, d_ms = prof["density_loop"]
    f_cnt, f_ms = prof["force_loop"]
    all_active = {
        "interactions_per_step": I_d + I_f, "ms_per_step": wall_all * 1e3,
        "interactions_per_s": (I_d + I_f) / wall_all,
        "fp32_peak_frac_step": (FLOP_DENSITY * I_d + FLOP_FORCE * I_f) / wall_all / FP32_PEAK,
        "density_loop_tflops": FLOP_DENSITY * I_d * reps / (d_ms / 1e3) / 1e12,
        "force_loop_tflops": FLOP_FORCE * I_f * reps / (f_ms / 1e3) / 1e12,
        "newton_passes": i1["density_iterations"],
        "kernels_ms_per_step": {k: round(ms / reps, 3) for k, (cnt, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])},
    }
    print(f"all-active: {wall_all * 1e3:.1f} ms/step, {(I_d + I_f) / wall_all:.3g} interactions/s", file=sys.stderr,
          flush=True)
    # (ii) the sub-step sweep
    S = args.substeps
    per_m = {}
    k0 = ctx.info()
    t_sweep = time.perf_counter()
    for t in range(1, S + 1):
        m = min((t & -t).bit_length() - 1, top)
        ts = time.perf_counter()
        na = ctx.step(p, m, t, t_min, 1, False, want_count=True)
        ctx.sync()
        dt = time.perf_counter() - ts
        e = per_m.setdefault(m, [0, 0.0, 0])
        e[0] += 1
        e[1] += dt
        e[2] += na
        if t % 256 == 0:
            print(f"sub-step {t}/{S}: {(time.perf_counter() - t_sweep):.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t_sweep
    k1 = ctx.info()
    I_sd = k1["interactions_density"] - k0["interactions_density"]
    I_sf = k1["interactions_force"] - k0["interactions_force"]
    inter = I_sd + I_sf
    out = {
        "metric": "active particle-neighbour interactions/s (density+force), % FP32 peak, vs plain",
        "value": inter / wall,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": S,
        "warmup": 0,
        "ms_per_step": wall / S * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 positions/integration",
        "data": "synthetic",
        "t_min": t_min,
        "config": {"workload": f"grf {N} particles (256^3 lattice + Zel'dovich displacement of a P(k)~k^-2.5 "
                               f"field, rms {args.grf_amplitude} spacings; u log-uniform; 14 bins), "
                               f"{S} sub-steps t=1..{S} with max active bin min(ctz(t),13)",
                   "n_particles": N, "drift": "lazy (needed leaves)" if args.lazy_drift else "all particles"},
        "interactions": inter,
        "full_builds_in_sweep": k1["full_builds"] - k0["full_builds"],
        "cell_updates_in_sweep": k1["cell_updates"] - k0["cell_updates"],
        "fp32_peak_frac_sweep": (FLOP_DENSITY * I_sd + FLOP_FORCE * I_sf) / wall / FP32_PEAK,
        "all_active": all_active,
        "per_bin": [{"max_active_bin": m, "sub_steps": e[0], "mean_active": e[2] / e[0],
                     "mean_ms": e[1] / e[0] * 1e3} for m, e in sorted(per_m.items())],
    }
    print(json.dumps(out))


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
    ap.add_argument("--sweep-below", type=int, default=None)
    ap.add_argument("--sweep-waves", type=int, default=None)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--load-tune", default=None, help="load a tuning file instead of tuning")
    ap.add_argument("--tune-file", default=os.path.join(tempfile.gettempdir(), "sph_tuning_clustered.txt"))
    ap.add_argument("--workload", choices=("deepbin", "large"), default="deepbin")
    ap.add_argument("--substeps", type=int, default=8192, help="large workload: sub-steps of the sweep")
    ap.add_argument("--grf-amplitude", type=float, default=12.0)
    ap.add_argument("--lazy-drift", action="store_true",
                    help="large workload: drift only the particles each sub-step needs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (for scaling HBM counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the all-active, 64-box batch and adjoint companion measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU decomposition "
                                   "is design-only)"}))
        sys.exit(2)
    if args.workload == "large":
        run_large(args)
        return
    if args.copy_calibration:
        import torch
        n = 512 << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))
        return

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
    if args.sweep_below is not None:
        kw["sweep_below"] = args.sweep_below
    if args.sweep_waves is not None:
        kw["sweep_waves"] = args.sweep_waves
    ctx = sg.Context(**kw)
    p = sg.Particles.from_initial(ic)

    # setup (untimed): every particle gets its density-loop state once, then
    # one deep-bin step moves the particles off the converged state and
    # predicts h.  That state is the step's input: every step starts from it.
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, ics.N_BINS - 1)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, m)
    ctx.density_pass(p, entropy_from_u=False)
    ctx.force_pass(p)
    ctx.kick_drift(p, 1 << m, t_min, 1 << m, False)
    ctx.sync()
    # the arrays a step changes that a later step reads: positions,
    # velocities, entropies, h and bins (every other per-particle input of an
    # active particle is recomputed before it is read, and the step does not
    # write those of inactive particles)
    names = ["x", "y", "z", "vx", "vy", "vz", "vfx", "vfy", "vfz", "A", "Af", "h", "time_bin"]
    # they are moved into one device buffer (256-byte aligned slices), so
    # that the restore is a single copy
    sizes = [p[k].numel() * p[k].element_size() for k in names]
    offs, tot = [], 0
    for sz in sizes:
        offs.append(tot)
        tot += (sz + 255) // 256 * 256
    state = torch.empty(tot, dtype=torch.uint8, device="cuda")
    for k, o, sz in zip(names, offs, sizes):
        t = state[o:o + sz].view(p[k].dtype)
        t.copy_(p[k])
        p[k] = t
    snapshot = state.clone()

    def restore():
        state.copy_(snapshot)

    def step(s):
        restore()
        # build, sort, mark, density, force, kick_drift: one library call
        ctx.step(p, m, 3 << m, t_min, 1 << m, False)

    tuned = None
    if args.load_tune:
        ctx.load_tuning(args.load_tune)
        tuned = [l.split() for l in open(args.load_tune) if l.startswith("best")]
    elif not args.no_tune:
        # one step whose loops are tuned on the step's own active chunks
        restore()
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

    # cost of the input restore alone (it is inside every timed step)
    torch.cuda.synchronize()
    tr = time.perf_counter()
    for _ in range(10):
        restore()
    torch.cuda.synchronize()
    restore_ms = (time.perf_counter() - tr) / 10 * 1e3

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
                    "frac": achieved / FP32_PEAK, "traffic": measured_traffic(dom), "kernel": dom}
        else:
            roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": measured_traffic(dom), "kernel": dom}
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
        "input_restore_ms_per_step": restore_ms,
        "fp32_peak_frac_step": flops_step / (wall / args.steps) / FP32_PEAK,
        "fp32_peak_frac_loops": (flops_step / (loop_ms / 1e3) / FP32_PEAK) if loop_ms > 0 else None,
        "loops_rate_interactions_per_s": ((I_d2 + I_f2) / ksteps) / (loop_ms / 1e3) if loop_ms > 0 else None,
        "profiled_ms_per_step": (t3 - t2) / ksteps * 1e3,
        "last_step_newton": {"unconverged_after_pass": last["unconverged_after_pass"],
                             "pair_rebuilds": last["pair_rebuilds"]},
        "kernels": kernels,
        "tuned_loops": [{"loop": ("density", "force")[int(t[1])], "chunk_class": int(t[2]), "waves_per_chunk": int(t[3]),
                         "tile": int(t[4]), "cost_ordered": int(t[5]), "persistent": int(t[6]), "chunk_split": int(t[7]),
                         "ms": float(t[8])}
                        for t in (tuned or [])],
        "roofline": roof,
    }
    if not args.no_extras:
        del p, ctx, state, snapshot
        torch.cuda.empty_cache()
        out["all_active"] = measure_all_active(sg, ic, **kw)
        out["batch"] = measure_batch(sg)
        out["adjoint"] = measure_adjoint(sg)
    if not args.no_cpu_baseline:
        act = ic["bin"] <= m
        out["cpu_baseline"] = run_cpu_baseline(ic, np.nonzero(act)[0], args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
