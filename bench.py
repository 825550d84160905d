"""Benchmark of the SPH hot path on one MI355X.

Default workload: the large single-GPU share, 16,777,216 particles (a 256^3
lattice displaced by the Zel'dovich field of a Gaussian random field with
P(k) ~ k^-2.5, u log-uniform in [1e-2, 1e2], 14 power-of-two time-bins of
Eq. 2).  One benchmark step is one top-level step of the bin hierarchy: the
2^13 sub-steps t, each running the whole path -- build_cells (cell update,
or a full build when particles moved too far), sort_cells, mark_active(m)
with m = min(ctz(t), 13), density_pass, force_pass, kick_drift -- with only
the particles a sub-step needs drifted (Sec. II-A, Sec. III-D).  The
simulation continues from step to step.

Prints one JSON line: active particle-neighbour interactions/s (density +
force, in-support pairs only, counted by the kernels) over the timed
top-level steps, the roofline of the dominant kernel group (HIP events on
the library's stream in a profiled top-level step after the timed ones),
the per-bin time against the number of active particles (the single-GPU
analogue of the paper's Fig. 7), and the FP64 oracle's rate on a bounded
sample of the same particles on the host cores.  `--workload clustered`
runs the 2,097,152-particle deep-bin step instead (also reported as an
extra key of the default line).
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
# copy (FETCH x 2.000, WRITE x 1.000), each on the workload whose roofline
# kernel it is: the density chunk loop over one 2^13 period of the large
# share's time line (profiles/c5_density_loop_traffic_pmc.md), the force sweep
# of the clustered deep-bin step (profiles/clustered_deepbin_sweeps_pmc.md);
# valid while the kernels' sources are the ones that were measured (else
# reported as null)
_LOOP_SOURCES = ["paper_1807_01341_amd/csrc/loops.hip", "paper_1807_01341_amd/csrc/loops_common.h",
                 "paper_1807_01341_amd/csrc/sph_internal.h"]
_LOOP_SHA = "440a7d9d03be16db30f53c9311e036a21897bd5bd362fb06b84d85593ca5827f"
MEASURED_TRAFFIC = {
    "density_loop": {"bytes": 7.08897e8, "sources": _LOOP_SOURCES, "sha256": _LOOP_SHA},
    "force_loop": {"bytes": 2.01347e9, "sources": _LOOP_SOURCES, "sha256": _LOOP_SHA},
    "force_sweep": {"bytes": 1.78494e7, "sources": _LOOP_SOURCES, "sha256": _LOOP_SHA},
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


# algorithmic FLOP per in-support interaction of the two loops, from the
# operation list of the pair formulas (mul/add = 1, fma = 2, rsqrt/rcp = 1,
# compare/select = 0): density 54, force 67
FLOP_DENSITY = 54
FLOP_FORCE = 67


def kernel_model(name, n, n_active, n_leaves, n_dens, n_force, launches):
    """Algorithmic bytes (hbm) or flops (alu) of ONE launch of a kernel group,
    for the roofline of the dominant kernel."""
    if name in ("density_loop", "density_sweep"):
        return "alu", FLOP_DENSITY * n_dens / launches
    if name in ("force_loop", "force_sweep"):
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


def cpu_info():
    """The host's CPU model and core counts (for the baseline's record)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "usable_cpus": usable}


def oracle_on_cube(ic, centre, half, label):
    """The FP64 oracle, unchanged, on the particles of a cube of half-side
    `half` around `centre` (periodic): the density loop with the h solve for
    every particle at least 1.6 max(H) inside the cube (their neighbours all
    lie in the cube), the ghost, and the force loop for every particle at
    least 2.7 max(H) inside (its neighbours are all solved).  Credits every
    in-support interaction it evaluated at the converged h."""
    import torch

    from oracle import sph
    x = ic["x"]
    d = x - centre
    d -= np.round(d)
    cheb = np.max(np.abs(d), 1)
    sub = np.nonzero(cheb < half)[0]
    Hmax = sph.GAMMA_K * float(ic["h"][sub].max())
    dens = np.searchsorted(sub, sub[cheb[sub] < half - 1.6 * Hmax])
    forc = np.searchsorted(sub, sub[cheb[sub] < half - 2.7 * Hmax])
    if dens.size == 0 or forc.size == 0:
        return None
    xs, vs, ms, us, hs = ic["x"][sub], ic["v"][sub], ic["m"][sub], ic["u"][sub], ic["h"][sub]
    t0 = time.perf_counter()
    out = sph.density_and_ghost(xs, vs, ms, hs, 1.0, u=us, centres=dens)
    full = {}
    for k in ("h", "rho", "f", "P", "c", "B"):
        a = torch.full((sub.size,), float("nan"), dtype=torch.float64)
        a[torch.as_tensor(dens)] = out[k]
        full[k] = a
    fo = sph.force(xs, vs, ms, full["h"], full["rho"], full["f"], full["P"], full["c"], full["B"], 1.0,
                   centres=forc)
    t = time.perf_counter() - t0
    inter = int(out["count"].sum() + fo["count"].sum())
    return dict(value=inter / t, unit="interactions/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{label}: the {sub.size} particles of a cube of half-side {half:.3f} around a seeded "
                       f"particle; density loop with the h solve for the {dens.size} at least 1.6 max H inside, "
                       f"force loop for the {forc.size} at least 2.7 max H inside; every in-support interaction "
                       f"evaluated at the converged h credited: {inter} in {t:.1f} s",
                seconds=t, interactions=inter, **cpu_info())


def run_cpu_baseline(ic, label, seed=5, target_centres=90000, max_half=0.3):
    """The oracle on a bounded sample: a cube around a seeded particle, grown
    until its density region holds about `target_centres` particles."""
    from oracle import sph
    rng = np.random.default_rng(seed)
    centre = ic["x"][int(rng.integers(ic["x"].shape[0]))]
    d = ic["x"] - centre
    d -= np.round(d)
    cheb = np.max(np.abs(d), 1)
    half = 0.02
    while half < max_half:
        sub = cheb < half
        Hmax = sph.GAMMA_K * float(ic["h"][sub].max()) if sub.any() else 0.0
        if np.count_nonzero(cheb < half - 1.6 * Hmax) >= target_centres and np.any(cheb < half - 2.7 * Hmax):
            break
        half *= 1.15
    return oracle_on_cube(ic, centre, min(half, max_half), label)


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



def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ctz(t):
    return (t & -t).bit_length() - 1


def loop_kwargs(args):
    kw = {}
    for a, k in (("split", "split_count"), ("cand_cap", "cand_cap"), ("list_cap", "list_cap"), ("h_tol", "h_tol"),
                 ("nw", "waves_per_chunk"), ("sweep_below", "sweep_below"), ("sweep_waves", "sweep_waves"),
                 ("rebuild_frac", "rebuild_frac")):
        v = getattr(args, a, None)
        if v is not None and v is not False:
            kw[k] = v
    return kw


def fixed_tiling_file(tiling):
    """A tuning table that gives every pass of both loops the tiling
    "NW,TILE" (waves per chunk, tile class), Morton order, grid launch."""
    nw, tile = (int(v) for v in tiling.split(","))
    path = os.path.join(tempfile.gettempdir(), f"sph_tiling_{nw}_{tile}.txt")
    with open(path, "w") as f:
        for loop in (0, 1):
            for cls in range(32):
                f.write(f"best {loop} {cls} {nw} {tile} 0 0 0 0 0\n")
    return path


def grf_setup(sg, ic, lazy, kw, tune_file=None, n_bins=None, tiling=None):
    """Context and particles of the large share, after an all-active density
    + force pass (u the thermal input), the loop tuning on those chunks, the
    t_min of Eq. 1 (the smallest time-step of the converged state, so every
    particle's bin satisfies its own Courant condition) and the first kick
    with the drift to t = 1."""
    import torch
    kw = dict(kw)
    if n_bins is not None:
        kw["n_bins"] = n_bins
    ctx = sg.Context(lazy_drift=int(lazy), **kw)
    p = sg.Particles.from_initial(ic)
    if n_bins is not None:
        p["time_bin"].clamp_(max=n_bins - 1)   # every particle in a bin the context has
    top = ctx.params.n_bins - 1
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, top)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    if tiling:
        ctx.load_tuning(fixed_tiling_file(tiling))
    elif tune_file is not False:
        if tune_file and os.path.exists(tune_file):
            os.remove(tune_file)
        ctx.autotune(p, tune_file or None)
    vs = p["vsig"].double()
    dt = torch.where(vs > 0, ctx.params.cfl * p["h"].double() / vs, torch.full_like(vs, float("inf")))
    t_min = float(dt.min())
    ctx.kick_drift(p, 0, t_min, 1, True)
    ctx.sync()
    return ctx, p, t_min


class TimeLine:
    """The individual-time-step time line of one context after grf_setup
    (whose kick_drift at t = 0 moved the line to 1): advance(n) moves the line
    on by n units of t_min, taking a step at each time some particle is
    active (Sec. II-A) and none at the times in between -- the step at tn runs
    with no drift, then sph_drift moves the line on to the next active time."""

    def __init__(self, ctx, p, t_min):
        self.ctx, self.p, self.t_min = ctx, p, t_min
        self.top = ctx.params.n_bins - 1
        self.t, self.line, self.end, self.stepped = 0, 1, 0, 0

    def advance(self, n, per_sub=None):
        self.end += n
        while True:
            tn = self.ctx.next_active_time(self.p, self.t)
            if tn > self.end:
                return
            if tn > self.line:
                self.ctx.drift(self.p, self.t_min, tn - self.line)
            m = min(ctz(tn), self.top)
            self.t = self.line = tn
            self.stepped += 1
            if per_sub is None:
                self.ctx.step(self.p, m, tn, self.t_min, 0, False)
            else:
                ts = time.perf_counter()
                na = self.ctx.step(self.p, m, tn, self.t_min, 0, False, want_count=True)
                self.ctx.sync()
                per_sub(m, na, time.perf_counter() - ts)


def all_active_steps(ctx, p, reps=3):
    """Whole steps with every particle active (no time advance): build, sort,
    mark, density (all Newton passes), force; the loops at full occupancy."""
    import torch
    top = ctx.params.n_bins - 1
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
    wall = (time.perf_counter() - t0) / reps
    prof = ctx.profile_read()
    ctx.profile(False)
    i1 = ctx.info()
    I_d = (i1["interactions_density"] - i0["interactions_density"]) / reps
    I_f = (i1["interactions_force"] - i0["interactions_force"]) / reps
    out = {"interactions_per_step": I_d + I_f, "ms_per_step": wall * 1e3, "interactions_per_s": (I_d + I_f) / wall,
           "fp32_peak_frac_step": (FLOP_DENSITY * I_d + FLOP_FORCE * I_f) / wall / FP32_PEAK,
           "newton_passes": i1["density_iterations"],
           "kernels_ms_per_step": {k: round(ms / reps, 3)
                                   for k, (cnt, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}}
    for name, flop, I in (("density_loop", FLOP_DENSITY, I_d), ("force_loop", FLOP_FORCE, I_f)):
        if name in prof:
            cnt, ms = prof[name]
            out[name + "_tflops"] = flop * I * reps / (ms / 1e3) / 1e12
    return out


def run_grf(args):
    """The default line: the 2^13-sub-step hierarchy on the 16,777,216-particle
    share, one benchmark step = `--substeps` consecutive sub-steps (2048: 20
    timed steps are exactly five top-level periods), then one whole period
    with a synchronisation after every sub-step for the per-bin table."""
    import torch

    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()
    tg = time.perf_counter()
    ic = ics.grf_zeldovich(amplitude=args.grf_amplitude)
    N = ic["x"].shape[0]
    log(f"generated {N} particles in {time.perf_counter() - tg:.0f} s")
    lazy = not args.drift_all
    ctx, p, t_min = grf_setup(sg, ic, lazy, loop_kwargs(args),
                              tune_file=False if args.no_tune else args.tune_file, tiling=args.tiling)
    top = ctx.params.n_bins - 1
    S = args.substeps
    sweep_below = ctx.params.sweep_below
    log(f"setup done: t_min {t_min:.4e}")
    line = TimeLine(ctx, p, t_min)

    def top_step(per_sub=None, n_sub=S):
        line.advance(n_sub, per_sub)

    for w in range(args.warmup):
        tw = time.perf_counter()
        top_step()
        torch.cuda.synchronize()
        log(f"warm-up step {w + 1}/{args.warmup}: {time.perf_counter() - tw:.2f} s")
    torch.cuda.synchronize()
    i0 = ctx.info()
    stepped0 = line.stepped
    t0 = time.perf_counter()
    for k in range(args.steps):
        top_step()
        torch.cuda.synchronize()
        log(f"timed step {k + 1}/{args.steps}: {time.perf_counter() - t0:.2f} s so far")
    t1 = time.perf_counter()
    i1 = ctx.info()
    stepped_timed = line.stepped - stepped0
    wall = t1 - t0
    I_d = i1["interactions_density"] - i0["interactions_density"]
    I_f = i1["interactions_force"] - i0["interactions_force"]
    value = (I_d + I_f) / wall

    # one more top-level period with HIP events around every launch group and
    # a synchronisation after each sub-step (per-bin times, interactions per
    # loop form)
    per_m = {}
    I_grp = {"density_loop": 0, "density_sweep": 0, "force_loop": 0, "force_sweep": 0}
    last = {"i": ctx.info()}

    newton = []

    def per_sub(m, na, dt):
        inf = ctx.info()
        dd = inf["interactions_density"] - last["i"]["interactions_density"]
        df = inf["interactions_force"] - last["i"]["interactions_force"]
        last["i"] = inf
        form = "loop" if na >= sweep_below else "sweep"
        if form == "loop":
            newton.append({"max_active_bin": m, "active": na, "ms": round(dt * 1e3, 3),
                           "unconverged_after_pass": inf["unconverged_after_pass"],
                           "full_build": inf["full_builds"] != last.setdefault("fb", inf["full_builds"])})
        last["fb"] = inf["full_builds"]
        I_grp["density_" + form] += dd
        I_grp["force_" + form] += df
        e = per_m.setdefault(m, [0, 0.0, 0, 0])
        e[0] += 1
        e[1] += dt
        e[2] += na
        e[3] += dd + df

    # one whole period (bins 0..13 each at its own rate), from a period boundary
    period = 1 << top
    top_step(None, (-line.end) % period)
    stepped_p = line.stepped
    torch.cuda.synchronize()
    last["i"] = ctx.info()
    last["fb"] = last["i"]["full_builds"]
    # a one-element int16 fill on each side of the profiled period: the only
    # launches of that kernel in the run, so a kernel trace can cut out the
    # period's dispatches
    torch.ones(1, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    ctx.profile(True)
    tp = time.perf_counter()
    top_step(per_sub, period)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    prof = ctx.profile_read()
    ctx.profile(False)
    torch.ones(1, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    log(f"profiled period: {prof_wall:.2f} s")
    kernels = {k: {"launches": c, "ms_per_period": round(ms, 3)}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    groups = {}
    for name, flop in (("density_loop", FLOP_DENSITY), ("density_sweep", FLOP_DENSITY),
                       ("force_loop", FLOP_FORCE), ("force_sweep", FLOP_FORCE)):
        if name in prof:
            c, ms = prof[name]
            groups[name] = {"launches": c, "ms": ms, "interactions": I_grp[name],
                            "tflops": flop * I_grp[name] / (ms / 1e3) / 1e12 if ms > 0 else None}
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    cnt, ms = prof[dom]
    roof = None
    if dom in groups:
        flop = FLOP_DENSITY if dom.startswith("density") else FLOP_FORCE
        per_launch = flop * I_grp[dom] / cnt
        dur = ms / 1e3 / cnt
        achieved = per_launch / dur
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK, "traffic": measured_traffic(dom), "kernel": dom,
                "launches": cnt, "avg_launch_ms": ms / cnt, "flop_per_launch": per_launch}
    else:
        bound, per_launch = kernel_model(dom, N, 0, 0, 0, 0, cnt)
        if per_launch is not None:
            achieved = per_launch / (ms / 1e3 / cnt)
            roof = {"bound": bound, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": None, "kernel": dom}
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
        "dtype": "f32",
        "dtype_note": "FP32 pair arithmetic on cell-relative offsets with compensated per-particle sums; FP64 "
                      "positions, velocities and time integration",
        "data": "synthetic",
        "config": {"workload": f"large single-GPU share: {N} particles (256^3 lattice displaced by the Zel'dovich "
                               f"field of a Gaussian random field, P(k)~k^-2.5, rms {args.grf_amplitude} spacings; "
                               f"u adiabatic with log-normal scatter, 2% of the particles in 16 Plummer clumps; 14 time-bins); one step "
                               f"= {S} units t_min of the time line (a quarter of the 2^13 period), stepped at "
                               f"each time t some bin is active (max active bin min(ctz(t),13))",
                   "n_particles": N, "substeps_per_step": S,
                   "drift": "lazy (only the particles a sub-step needs)" if lazy else "every particle each sub-step"},
        "interactions": I_d + I_f,
        "interactions_density": I_d,
        "interactions_force": I_f,
        "fp32_peak_frac_step": (FLOP_DENSITY * I_d + FLOP_FORCE * I_f) / wall / FP32_PEAK,
        "times_stepped_timed": stepped_timed,
        "times_on_line_timed": args.steps * S,
        "full_builds_timed": i1["full_builds"] - i0["full_builds"],
        "cell_updates_timed": i1["cell_updates"] - i0["cell_updates"],
        "t_min": t_min,
        "roofline": roof,
        "loop_groups": groups,
        "profiled_period_s": prof_wall,
        "profiled_period_times_stepped": line.stepped - stepped_p,
        "kernels": kernels,
        "per_bin": [{"max_active_bin": m, "steps_taken": e[0], "mean_active": e[2] / e[0], "mean_ms": e[1] / e[0] * 1e3,
                     "interactions_per_s": e[3] / e[1] if e[1] > 0 else None}
                    for m, e in sorted(per_m.items())],
        "dense_substeps": newton[:24],
    }
    out["all_active"] = all_active_steps(ctx, p)
    log("all-active steps done")
    del ctx, p
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["clustered_deepbin"] = run_clustered(args, with_baseline=False)
        log("clustered deep-bin line done")
        out["batch"] = measure_batch(sg)
        out["adjoint"] = measure_adjoint(sg)
        log("batch and adjoint done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(ic, "all-active state of the large share (u the thermal input)")
        log("cpu baseline done")
    print(json.dumps(out))


def run_all_active(args):
    """The large share's all-active step alone (the loops at full occupancy):
    setup as in the default line, then `--steps` whole steps with every
    particle active; the command the loop kernels are profiled with."""
    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()
    ic = ics.grf_zeldovich(amplitude=args.grf_amplitude)
    log(f"generated {ic['x'].shape[0]} particles")
    ctx, p, t_min = grf_setup(sg, ic, not args.drift_all, loop_kwargs(args),
                              tune_file=False if args.no_tune else args.tune_file, tiling=args.tiling)
    out = all_active_steps(ctx, p, reps=max(1, args.steps))
    out["workload"] = f"large share {ic['x'].shape[0]} particles, all active"
    print(json.dumps(out))


def run_strategies(args):
    """The strategy comparison of the paper's Fig. 2 on the large share: one
    2^13 period of the time line with every particle drifted at each step,
    one with only the needed particles drifted (both stepping only at times
    some bin is active), and the global step (every particle active at every
    time t_min: n_bins = 1), the last extrapolated from a few steps to the
    same 2^13."""
    import torch

    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()
    ic = ics.grf_zeldovich(amplitude=args.grf_amplitude)
    N = ic["x"].shape[0]
    res = {}
    S = None
    for name, lazy in (("relevant_only_drift", True), ("drift_all_kick_active", False)):
        ctx, p, t_min = grf_setup(sg, ic, lazy, loop_kwargs(args), tune_file=None)
        S = 1 << (ctx.params.n_bins - 1)
        line = TimeLine(ctx, p, t_min)
        i0 = ctx.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        line.advance(S)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        i1 = ctx.info()
        I = i1["interactions_density"] + i1["interactions_force"] - i0["interactions_density"] - i0["interactions_force"]
        res[name] = {"seconds": wall, "interactions": I, "interactions_per_s": I / wall, "t_min": t_min,
                     "times_stepped": line.stepped}
        log(f"{name}: {wall:.2f} s")
        del ctx, p
        torch.cuda.empty_cache()
    G = args.global_substeps
    ctx, p, t_min = grf_setup(sg, ic, False, loop_kwargs(args), tune_file=None, n_bins=1)
    i0 = ctx.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, G + 1):
        ctx.step(p, 0, t, t_min, 1, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    i1 = ctx.info()
    I = i1["interactions_density"] + i1["interactions_force"] - i0["interactions_density"] - i0["interactions_force"]
    res["global_step"] = {"seconds_measured": wall, "substeps_measured": G, "seconds": wall * S / G,
                          "extrapolated": True, "interactions_per_s": I / wall, "t_min": t_min,
                          "note": f"every particle active at every sub-step of t_min; {G} sub-steps timed, "
                                  f"scaled to {S}"}
    base = res["global_step"]["seconds"]
    for k in res:
        res[k]["speedup_vs_global_step"] = base / res[k]["seconds"]
    print(json.dumps({"workload": f"large share {N} particles, {S} sub-steps", "strategies": res}))


def run_clustered(args, with_baseline=True, steps=20, warmup=3):
    """The 2,097,152-particle clustered box at the deep bin with about 1 % of
    the particles active: every timed step starts from the same input state
    (a fused device copy of the arrays a step changes, inside the timed
    region) and runs the whole path on it."""
    import torch

    import ics
    import paper_1807_01341_amd as sg
    sg.require_device()

    ic = ics.clustered()
    N = ic["x"].shape[0]
    m = ics.deep_bin_for_fraction(ic["bin"], args.active_fraction)
    t_min = ic["t_min_model"]
    kw = loop_kwargs(args)
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
        os.makedirs(os.path.dirname(args.tune_file_clustered), exist_ok=True)
        if os.path.exists(args.tune_file_clustered):
            os.remove(args.tune_file_clustered)
        ctx.autotune(p, args.tune_file_clustered)
        tuned = [l.split() for l in open(args.tune_file_clustered) if l.startswith("best")]

    # cost of the input restore alone (it is inside every timed step)
    torch.cuda.synchronize()
    tr = time.perf_counter()
    for _ in range(10):
        restore()
    torch.cuda.synchronize()
    restore_ms = (time.perf_counter() - tr) / 10 * 1e3

    for s in range(warmup):
        step(s)
    torch.cuda.synchronize()
    inf0 = ctx.info()
    t0 = time.perf_counter()
    for s in range(warmup, warmup + steps):
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
    ksteps = args.profile_steps or steps
    ctx.profile(True)
    t2 = time.perf_counter()
    for s in range(warmup + steps, warmup + steps + ksteps):
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
    loop_ms = sum(prof.get(k, (0, 0.0))[1]
                  for k in ("density_loop", "force_loop", "density_sweep", "force_sweep")) / ksteps
    flops_step = (FLOP_DENSITY * I_d + FLOP_FORCE * I_f) / steps
    out = {
        "metric": "active particle-neighbour interactions/s (density+force), % FP32 peak, vs plain",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"clustered {N} particles (90% uniform + 10% in 20 Plummer spheres, "
                               f"a in [0.002,0.02], u log-uniform 1e-2..1e2, 14 bins), deep-bin step m={m}",
                   "n_particles": N, "max_active_bin": m, "n_active": inf1["n_active"],
                   "active_fraction": inf1["n_active"] / N, "n_leaves": inf1["n_leaves"],
                   "split_count": ctx.params.split_count},
        "interactions_per_step": inter / steps,
        "input_restore_ms_per_step": restore_ms,
        "fp32_peak_frac_step": flops_step / (wall / steps) / FP32_PEAK,
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
    del p, ctx, state, snapshot
    torch.cuda.empty_cache()
    out["all_active"] = measure_all_active(sg, ic, **kw)
    if with_baseline and not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(ic, "clustered workload, initial state (u the thermal input)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed steps (large share: top-level steps)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("grf", "clustered", "strategies", "allactive"), default="grf")
    ap.add_argument("--substeps", type=int, default=2048,
                    help="sub-steps per benchmark step (a divisor of the 2^13-sub-step period: K steps with K a "
                         "multiple of 8192/substeps cover whole periods, every bin in its exact proportion)")
    ap.add_argument("--global-substeps", type=int, default=16,
                    help="strategies: sub-steps timed for the global-step arm")
    ap.add_argument("--grf-amplitude", type=float, default=12.0)
    ap.add_argument("--drift-all", action="store_true", help="large share: drift every particle each sub-step")
    ap.add_argument("--active-fraction", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--split", type=int, default=None)
    ap.add_argument("--cand-cap", type=int, default=None)
    ap.add_argument("--list-cap", type=int, default=None)
    ap.add_argument("--profile-steps", type=int, default=None)
    ap.add_argument("--h-tol", type=float, default=None)
    ap.add_argument("--rebuild-frac", type=float, default=0.25,
                    help="cells kept while every particle moved less than this fraction of its leaf "
                         "(the library's default is 1/8; 1/4 halves the large share's full builds)")
    ap.add_argument("--nw", type=int, default=None)
    ap.add_argument("--sweep-below", type=int, default=None)
    ap.add_argument("--sweep-waves", type=int, default=None)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tiling", default=None,
                    help="large share: 'NW,TILE' for every loop pass instead of the autotuner's choice")
    ap.add_argument("--load-tune", default=None, help="clustered: load a tuning file instead of tuning")
    ap.add_argument("--tune-file", default=os.path.join(tempfile.gettempdir(), "sph_tuning_grf.txt"))
    ap.add_argument("--tune-file-clustered", default=os.path.join(tempfile.gettempdir(), "sph_tuning_clustered.txt"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (for scaling HBM counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the clustered deep-bin, 64-box batch and adjoint companion measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU decomposition "
                                   "is design-only)"}))
        sys.exit(2)
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
    if args.workload == "grf":
        run_grf(args)
    elif args.workload == "strategies":
        run_strategies(args)
    elif args.workload == "allactive":
        run_all_active(args)
    else:
        out = run_clustered(args, steps=max(args.steps, 20), warmup=max(args.warmup, 3))
        if not args.no_extras:
            import paper_1807_01341_amd as sg
            out["batch"] = measure_batch(sg)
            out["adjoint"] = measure_adjoint(sg)
        print(json.dumps(out))


if __name__ == "__main__":
    main()
