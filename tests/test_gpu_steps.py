"""GPU parity of the path as a running simulation uses it, against the FP64
oracle: steps after the first, on cells and axis orders kept by cell
updates, with the H orders re-keyed as smoothing lengths change, with every
particle drifted each sub-step and with only the particles a step needs
drifted (Sec. II-A, Sec. III-D):

* the benchmark's deep-bin step on the 2,097,152-particle clustered box in
  the benchmark's own call sequence: counts of every active particle exact,
  the physics of about a thousand active particles spread over all clumps
  and the background against the oracle;
* the first 64 sub-steps (bins 0-6) of the 16,777,216-particle share, with
  both drift policies (and the benchmark's cell-keeping fraction 1/4 with
  lazy drift), checked at five sub-steps;
* all 64 boxes of the batching workload at their active fractions, batched;
* the individual-time-step kick-drift-kick of 16 sub-steps, both drift
  policies, against the oracle's kick_drift driven with the same
  accelerations, signal speeds and smoothing lengths.

Each check takes the step's inputs from the state the path reached (the
oracle at the GPU's positions); see tests/gpu_cases.check_step_vs_oracle."""
import numpy as np
import pytest
import torch

import ics
from oracle import sph
from tests.gpu_cases import CellTracker, check_step_vs_oracle, host, spread_sample, step_state

pytestmark = pytest.mark.gpu


def _build(ctx, p, perm, tr):
    f0 = ctx.info()["full_builds"]
    ctx.build_cells(p, perm)
    return tr.after_build(ctx, p, perm, f0)


def _active(ctx):
    return ctx.copy_active()[0].cpu().numpy().astype(bool)


def test_clustered_bench_sequence_full_size(gpu_lib):
    sg = gpu_lib
    ic = ics.clustered()
    N = ic["x"].shape[0]
    m = ics.deep_bin_for_fraction(ic["bin"], 0.01)
    t_min = ic["t_min_model"]
    print(f"case clustered full N={N} m={m}: bench sequence", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    tr = CellTracker()
    perm = torch.empty(N, dtype=torch.int64, device="cuda")
    # the benchmark's setup: all-active density + force, one deep-bin step and its kick-drift
    assert _build(ctx, p, perm, tr)
    ctx.sort_cells()
    ctx.mark_active(p, ics.N_BINS - 1)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    assert not _build(ctx, p, perm, tr)
    ctx.sort_cells()
    ctx.mark_active(p, m)
    ctx.density_pass(p, entropy_from_u=False)
    ctx.force_pass(p)
    ctx.kick_drift(p, 1 << m, t_min, 1 << m, False)
    # the timed step: cell update on the moved particles, kept sorts, marking,
    # density with the h solve, force
    assert not _build(ctx, p, perm, tr), "the benchmark's step is a cell update"
    ctx.sort_cells()
    ctx.mark_active(p, m)
    ctx.density_pass(p, entropy_from_u=False)
    ctx.force_pass(p)
    ctx.sync()
    inf = ctx.info()
    assert inf["cell_updates"] == 2 and inf["full_builds"] == 1 and inf["n_unconverged"] == 0
    st = step_state(p)
    act = _active(ctx)
    assert 0.005 < act.sum() / N < 0.02
    xs = np.stack([st["x"], st["y"], st["z"]], 1)
    samples = spread_sample(act, st["h"], 560, np.random.default_rng(3), centres=ic["clump_centres"], x=xs,
                            per_centre=25)
    assert samples.size >= 1000
    check_step_vs_oracle(st, act, m, samples, tr.now(st), label="clustered 2,097,152, bench step")


@pytest.fixture(scope="module")
def grf_share():
    return ics.grf_zeldovich()


@pytest.mark.parametrize("lazy,rebuild_frac", [(0, 0.125), (1, 0.125), (1, 0.25)])
def test_large_share_first_64_substeps(gpu_lib, grf_share, lazy, rebuild_frac):
    sg = gpu_lib
    ic = grf_share
    N = ic["x"].shape[0]
    print(f"case large share N={N} lazy_drift={lazy} rebuild_frac={rebuild_frac}: sub-steps 1..64", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context(lazy_drift=lazy, rebuild_frac=rebuild_frac)
    tr = CellTracker()
    perm = torch.empty(N, dtype=torch.int64, device="cuda")
    top = ctx.params.n_bins - 1
    assert _build(ctx, p, perm, tr)
    ctx.sort_cells()
    ctx.mark_active(p, top)
    ctx.density_pass(p, entropy_from_u=True)
    ctx.force_pass(p)
    vs = p["vsig"].double()
    t_min = float(torch.where(vs > 0, ctx.params.cfl * p["h"].double() / vs, torch.full_like(vs, np.inf)).min())
    ctx.kick_drift(p, 0, t_min, 1, True)
    rng = np.random.default_rng(7 + lazy)
    checks = {1, 8, 24, 32, 64}
    for t in range(1, 65):
        mb = min((t & -t).bit_length() - 1, top)
        full = _build(ctx, p, perm, tr)
        ctx.sort_cells()
        na = ctx.mark_active(p, mb)
        ctx.density_pass(p, entropy_from_u=False)
        ctx.force_pass(p)
        if t in checks:
            ctx.sync()
            st = step_state(p)
            act = _active(ctx)
            assert act.sum() == na
            idx = np.nonzero(act)[0]
            cs = idx if idx.size <= 40000 else np.sort(rng.choice(idx, 40000, replace=False))
            samples = spread_sample(act, st["h"], 48, rng)
            check_step_vs_oracle(st, act, mb, samples, tr.now(st), count_samples=cs,
                                 label=f"large share lazy={lazy} t={t} m={mb} active={na} full_build={full}")
        ctx.kick_drift(p, t, t_min, 1, False)
    ctx.sync()


def test_batch_64_boxes_at_their_fractions(gpu_lib):
    sg = gpu_lib
    boxes = ics.batch_of_boxes()
    ms = [ics.deep_bin_for_fraction(b["bin"], b["target_active_fraction"]) for b in boxes]
    print(f"case batch64 N={sum(b['x'].shape[0] for b in boxes)}, default parameters, batched", flush=True)
    cs, ps, trs = [], [], []
    for b, m in zip(boxes, ms):
        p = sg.Particles.from_initial(b)
        c = sg.Context()
        tr = CellTracker()
        perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
        assert _build(c, p, perm, tr)
        c.sort_cells()
        c.mark_active(p, c.params.n_bins - 1)
        c.density_pass(p, True)
        c.mark_active(p, m)
        cs.append(c)
        ps.append(p)
        trs.append(tr)
    batch = sg.Batch(cs, ps)
    batch.density_pass(False)
    batch.force_pass()
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for b in range(len(boxes)):
        st = step_state(ps[b])
        act = _active(cs[b])
        samples = spread_sample(act, st["h"], 8, rng)
        check_step_vs_oracle(st, act, ms[b], samples, trs[b].now(st),
                             label=f"box {b} N={ps[b].n} m={ms[b]} active={int(act.sum())}")


@pytest.mark.parametrize("lazy", [0, 1])
def test_individual_steps_kick_drift_vs_oracle(gpu_lib, lazy):
    """Sixteen sub-steps of the bin hierarchy on a moving clustered box: the
    GPU's kicks, bins, drifts and h predictions against the oracle's
    kick_drift driven, sub-step by sub-step, with the accelerations, dA/dt,
    signal speeds, div v and (for active particles) smoothing lengths of the
    GPU's loops.  With lazy drift the GPU brings every particle to the
    current time only at the end (sph_drift_all); the oracle drifts every
    particle every sub-step."""
    sg = gpu_lib
    ic = dict(ics.clustered(n_total=20000, n_clumps=3))
    rng = np.random.default_rng(5)
    ic["v"] = rng.normal(0.0, 0.3, size=ic["x"].shape)
    print(f"case kick-drift clustered20k lazy={lazy} 16 sub-steps", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context(lazy_drift=lazy)
    top = ctx.params.n_bins - 1
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, top)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    vs = p["vsig"].double()
    t_min = float((ctx.params.cfl * p["h"].double() / vs).min())

    def inputs():
        return {k: host(p, k).astype(np.float64) if k != "time_bin" else host(p, k).astype(np.int64)
                for k in ("ax", "ay", "az", "dA_dt", "h", "vsig", "divv", "time_bin")}

    # oracle state (the step's order never changes: every build here is a cell update)
    o = dict(x=np.stack([host(p, k) for k in "xyz"], 1), vf=np.stack([host(p, k) for k in ("vfx", "vfy", "vfz")], 1),
             vp=np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1), Af=host(p, "Af").astype(np.float64),
             Ap=host(p, "A").astype(np.float64), bins=host(p, "time_bin").astype(np.int64),
             h=host(p, "h").astype(np.float64))
    full0 = ctx.info()["full_builds"]
    for t in range(0, 17):
        if t > 0:
            mb = min((t & -t).bit_length() - 1, top)
            ctx.build_cells(p)
            ctx.sort_cells()
            ctx.mark_active(p, mb)
            ctx.density_pass(p, False)
            ctx.force_pass(p)
        ctx.sync()
        act = _active(ctx)
        g = inputs()
        assert np.array_equal(act, o["bins"] <= (top if t == 0 else mb)), t
        a = np.stack([g["ax"], g["ay"], g["az"]], 1)
        h_in = np.where(act, g["h"], o["h"])
        r = sph.kick_drift(o["x"], o["vf"], o["vp"], o["Af"], o["Ap"], a, g["dA_dt"], h_in, g["vsig"], o["bins"],
                           act, t, t_min, 1, 1.0, first_step=(t == 0), divv=g["divv"])
        o.update(x=r["x"], vf=r["vf"], vp=r["vp"], Af=r["Af"], Ap=r["Ap"], bins=r["bins"], h=r["h"])
        ctx.kick_drift(p, t, t_min, 1, t == 0)
    ctx.drift_all(p)
    ctx.sync()
    assert ctx.info()["full_builds"] == full0
    gx = np.stack([host(p, k) for k in "xyz"], 1)
    d = gx - o["x"]
    d -= np.round(d)
    dv = np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1) - o["vp"]
    dvf = np.stack([host(p, k) for k in ("vfx", "vfy", "vfz")], 1) - o["vf"]
    vscale = np.max(np.abs(o["vf"]))
    err = {"x": float(np.max(np.abs(d))), "v": float(np.max(np.abs(dv)) / vscale),
           "vf": float(np.max(np.abs(dvf)) / vscale),
           "A": float(np.max(np.abs(host(p, "A") / o["Ap"] - 1))),
           "Af": float(np.max(np.abs(host(p, "Af") / o["Af"] - 1))),
           "h": float(np.max(np.abs(host(p, "h") / o["h"] - 1)))}
    print(f"lazy={lazy} t_min {t_min:.3e}: " + " ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    assert np.array_equal(host(p, "time_bin").astype(np.int64), o["bins"])
    assert len(set(o["bins"].tolist())) > 1
    # positions and velocities: FP64 on both sides, the lazy drift adding a
    # lag of several sub-steps at once; entropies and h: stored in FP32 by the
    # path, one rounding (at most 2^-24 relative) per sub-step that updates
    # them, against the oracle's FP64: 17 sub-steps x 2^-23
    assert err["x"] < 1e-12 and err["v"] < 1e-12 and err["vf"] < 1e-12
    tol32 = 17 * 2.0 ** -23
    assert err["A"] < tol32 and err["Af"] < tol32 and err["h"] < tol32


@pytest.mark.parametrize("lazy", [0, 1])
def test_drift_over_inactive_times_equals_drift_in_the_step(gpu_lib, lazy):
    """Steps taken only at the times some particle is active (Sec. II-A):
    each step's kick_drift moving the time line on to the next active time
    equals, bit for bit, the step with no drift followed by sph_drift over
    the times in between (nothing but the drift happens there).  The first
    run takes the times from sph_next_active_time; the second replays them."""
    sg = gpu_lib
    ic = dict(ics.clustered(n_total=20000, n_clumps=3))
    rng = np.random.default_rng(8)
    ic["v"] = rng.normal(0.0, 0.3, size=ic["x"].shape)
    print(f"case drift over inactive times clustered20k lazy={lazy}", flush=True)
    runs, times = [], []
    for split in (True, False):
        p = sg.Particles.from_initial(ic)
        ctx = sg.Context(lazy_drift=lazy)
        top = ctx.params.n_bins - 1
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, top)
        ctx.density_pass(p, True)
        ctx.force_pass(p)
        ctx.sync()
        t_min = float((ctx.params.cfl * p["h"].double() / p["vsig"].double()).min()) / 4
        if split:
            ctx.kick_drift(p, 0, t_min, 0, True)
            t = 0
            for _ in range(4):
                tn = ctx.next_active_time(p, t)
                assert tn > t
                times.append(tn)
                ctx.drift(p, t_min, tn - t)
                ctx.step(p, min((tn & -tn).bit_length() - 1, top), tn, t_min, 0, False)
                t = tn
        else:
            ctx.kick_drift(p, 0, t_min, times[0], True)
            for q, tn in enumerate(times):
                nxt = times[q + 1] - tn if q + 1 < len(times) else 0
                ctx.step(p, min((tn & -tn).bit_length() - 1, top), tn, t_min, nxt, False)
        ctx.drift_all(p)
        ctx.sync()
        runs.append({k: host(p, k).copy() for k in ("x", "y", "z", "vx", "vy", "vz", "vfx", "vfy", "vfz", "A", "Af",
                                                    "h", "time_bin", "ax", "rho")})
    print("active times", times, flush=True)
    # t_min a quarter of the smallest step: every particle sits in bin >= 2,
    # so the line passes over times with nothing active
    assert times[0] > 1
    if lazy:
        for k in runs[0]:
            assert np.array_equal(runs[0][k].view(np.uint8), runs[1][k].view(np.uint8)), k
        return
    # drifting every particle, the step with no drift stores the entropy it
    # kicked in FP32 before the drift adds dA/dt dt (one more rounding, at
    # most 2^-24 relative): the same times and bins, the state within that
    assert np.array_equal(runs[0]["time_bin"], runs[1]["time_bin"])
    rel = {k: float(np.max(np.abs(runs[0][k].astype(np.float64) - runs[1][k]) /
                           np.abs(runs[1][k].astype(np.float64))))
           for k in ("A", "Af", "h", "rho")}
    rel.update({k: float(np.max(np.abs(runs[0][k].astype(np.float64) - runs[1][k])) /
                         np.max(np.abs(runs[1][k].astype(np.float64))))
                for k in ("vx", "vy", "vz", "ax")})
    dx = max(float(np.max(np.abs(runs[0][k] - runs[1][k]))) for k in "xyz")
    print("drift-all differences", dx, rel, flush=True)
    assert dx < 1e-9
    assert max(rel.values()) < 1e-4
