"""GPU parity of the cell update (cells kept between builds while particles
stay near them): structures bit-exact against the C definitions of the
update, and the physics against the FP64 oracle at the moved positions."""
import numpy as np
import pytest
import torch

import ics
from oracle import cells as emu
from oracle import sph
from tests.gpu_cases import A_TOL, RHO_TOL, host, pair_set, with_slack

pytestmark = pytest.mark.gpu


def test_cell_update_matches_definitions_and_oracle(gpu_lib):
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.3)
    print("case update tiny16 sigma=0.3", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context(split_count=64)
    perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    perm = perm.cpu().numpy()
    cl = emu.build_cells(ic["x"], ic["h"], split=64, D=16)
    assert np.array_equal(perm, cl["perm"])
    x_build = np.stack([host(p, k) for k in "xyz"], 1)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    # move every particle by a few per cent of a leaf (drift of the given step)
    ctx.kick_drift(p, 0, 2e-3, 1, True)
    ctx.sync()
    x_moved = np.stack([host(p, k) for k in "xyz"], 1)
    h_now = host(p, "h").copy()
    assert np.max(np.abs(x_moved - x_build)) > 0
    perm2 = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm2)
    inf = ctx.info()
    assert inf["full_builds"] == 1 and inf["cell_updates"] == 1 and inf["dx_max"] > 0
    assert np.array_equal(perm2.cpu().numpy(), np.arange(p.n))
    up, flag = emu.update(cl, x_moved, h_now, x_build)
    assert not flag
    # positions wrapped in place, offsets, leaf max H and drift margins bit for bit
    assert np.array_equal(np.stack([host(p, k) for k in "xyz"], 1), np.stack([up["xw"], up["yw"], up["zw"]], 1))
    keys, o = ctx.copy_particles()
    for d, k in enumerate(("ox", "oy", "oz")):
        assert np.array_equal(o[d].cpu().numpy().view(np.uint32), up[k].view(np.uint32)), k
    lv = {k: v.cpu().numpy() for k, v in ctx.copy_leaves().items()}
    assert np.array_equal(lv["begin"], cl["leaf_begin"]) and np.array_equal(lv["count"], cl["leaf_count"])
    assert np.array_equal(lv["hmax"].view(np.uint32), up["leaf_hmax"].view(np.uint32))
    assert np.array_equal(lv["drift"].view(np.uint32), up["leaf_dx"].view(np.uint32))
    # the step on the kept cells: pair sets with the margins, counts, physics
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    act = emu.mark_active(up, host(p, "time_bin"), ctx.params.n_bins - 1, H=up["H"])
    a, b, s = ctx.copy_pairs(0)
    ea, eb, es = emu.pairs(up, with_slack(act, ctx.params.pair_slack), "density", leaf_dx=up["leaf_dx"])
    assert pair_set(a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy()) == pair_set(ea, eb, es)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    H = (np.float32(1.825742) * host(p, "h")).astype(np.float32)
    idx = np.arange(0, p.n, 7)
    assert np.array_equal(host(p, "nngb_density")[idx], emu.counts(up, "density", idx, H=H))
    assert np.array_equal(host(p, "nngb_force")[idx], emu.counts(up, "force", idx, H=H))
    lh = emu.leaf_hmax(up, H)
    a, b, s = ctx.copy_pairs(1)
    ea, eb, es = emu.pairs(up, act, "force", leaf_hmax_arr=lh, leaf_dx=up["leaf_dx"])
    assert pair_set(a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy()) == pair_set(ea, eb, es)
    # the axis orders are those of the full build's offsets
    order_ref, _ = emu.axis_sort(cl)
    assert np.array_equal(ctx.copy_axis_order().cpu().numpy().view(np.uint16), order_ref)
    # physics at the moved positions, in cell order
    xs = np.stack([up["xw"], up["yw"], up["zw"]], 1)
    v = np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1)
    u = host(p, "u").astype(np.float64)
    out = sph.density_and_ghost(xs, v, host(p, "m"), h_now, 1.0, u=u)
    fo = sph.force(xs, v, host(p, "m"), out["h"], out["rho"], out["f"], out["P"], out["c"], out["B"], 1.0)
    rho_err = np.max(np.abs(host(p, "rho") / out["rho"].numpy() - 1))
    a_g = np.stack([host(p, k) for k in ("ax", "ay", "az")], 1).astype(np.float64)
    a_r = fo["a"].numpy()
    den = np.maximum(np.linalg.norm(a_r, axis=1), 1e-2 * fo["scale"].numpy())
    a_err = np.max(np.linalg.norm(a_g - a_r, axis=1) / den)
    print(f"rho {rho_err:.2e} a {a_err:.2e}", flush=True)
    assert rho_err < RHO_TOL and a_err < A_TOL


def test_large_move_rebuilds(gpu_lib):
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    ctx.build_cells(p)
    shift = torch.full_like(p["x"], 0.05)
    p["x"].add_(shift)
    ctx.build_cells(p)
    inf = ctx.info()
    assert inf["full_builds"] == 2 and inf["cell_updates"] == 0
    ctx0 = sg.Context(rebuild_frac=0.0)
    p0 = sg.Particles.from_initial(ic)
    ctx0.build_cells(p0)
    ctx0.build_cells(p0)
    assert ctx0.info()["full_builds"] == 2


def test_kept_axis_orders_on_clustered_update(gpu_lib):
    """Cells and axis orders kept across an update on a clustered box with
    leaves past two tiles (their partners are swept in the kept order, with
    the stop widened by the drift margins): physics against the oracle."""
    sg = gpu_lib
    ic = dict(ics.clustered(n_total=20000, n_clumps=3))
    rng = np.random.default_rng(11)
    ic["v"] = rng.normal(0.0, 0.3, size=ic["x"].shape)
    print("case update clustered20k", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    lv = {k: v.cpu().numpy() for k, v in ctx.copy_leaves().items()}
    assert lv["count"].max() > 128
    # every particle moves by up to 5% of its leaf's width
    width = np.repeat(np.ldexp(1.0, -lv["level"]), lv["count"])
    xs = np.stack([host(p, k) for k in "xyz"], 1)
    xs = np.mod(xs + rng.uniform(-0.03, 0.03, size=xs.shape) * width[:, None], 1.0)
    for d, k in enumerate("xyz"):
        p[k].copy_(torch.from_numpy(np.ascontiguousarray(xs[:, d])))
    h_now = host(p, "h").copy()
    ctx.build_cells(p)
    inf = ctx.info()
    assert inf["full_builds"] == 1 and inf["cell_updates"] == 1 and inf["dx_max"] > 0
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    cl = emu.build_cells(ic["x"], ic["h"], split=400, D=16)
    assert np.array_equal(perm.cpu().numpy(), cl["perm"])
    order_ref, _ = emu.axis_sort(cl)
    assert np.array_equal(ctx.copy_axis_order().cpu().numpy().view(np.uint16), order_ref)
    xs = np.stack([host(p, k) for k in "xyz"], 1)
    v = np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1)
    u = host(p, "u").astype(np.float64)
    out = sph.density_and_ghost(xs, v, host(p, "m"), h_now, 1.0, u=u)
    fo = sph.force(xs, v, host(p, "m"), out["h"], out["rho"], out["f"], out["P"], out["c"], out["B"], 1.0)
    H = (np.float32(1.825742) * host(p, "h")).astype(np.float32)
    up, flag = emu.update(cl, xs, host(p, "h"), np.stack([ic["x"][cl["perm"], d] for d in range(3)], 1))
    assert not flag
    idx = np.arange(0, p.n, 5)
    assert np.array_equal(host(p, "nngb_density")[idx], emu.counts(up, "density", idx, H=H))
    assert np.array_equal(host(p, "nngb_force")[idx], emu.counts(up, "force", idx, H=H))
    rho_err = np.max(np.abs(host(p, "rho") / out["rho"].numpy() - 1))
    a_g = np.stack([host(p, k) for k in ("ax", "ay", "az")], 1).astype(np.float64)
    a_r = fo["a"].numpy()
    den = np.maximum(np.linalg.norm(a_r, axis=1), 1e-2 * fo["scale"].numpy())
    a_err = np.max(np.linalg.norm(a_g - a_r, axis=1) / den)
    print(f"rho {rho_err:.2e} a {a_err:.2e}", flush=True)
    assert rho_err < RHO_TOL and a_err < A_TOL


def test_lazy_drift_matches_drift_all(gpu_lib):
    """Sixteen sub-steps of the bin hierarchy with lazy drift (only the leaves
    a step needs are drifted) and with every particle drifted each step: the
    same active sets, and after drifting everything the same state to
    rounding."""
    sg = gpu_lib
    ic = dict(ics.clustered(n_total=20000, n_clumps=3))
    rng = np.random.default_rng(5)
    ic["v"] = rng.normal(0.0, 0.3, size=ic["x"].shape)
    print("case lazy drift clustered20k 16 sub-steps", flush=True)
    keys = ("x", "y", "z", "vx", "vfx", "A", "h", "rho", "ax", "ay", "az", "vsig", "time_bin")
    runs = []
    for lazy in (0, 1):
        p = sg.Particles.from_initial(ic)
        ctx = sg.Context(lazy_drift=lazy)
        top = ctx.params.n_bins - 1
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, top)
        ctx.density_pass(p, True)
        ctx.force_pass(p)
        vs = p["vsig"].double()
        t_min = float((ctx.params.cfl * p["h"].double() / vs).min())
        ctx.kick_drift(p, 0, t_min, 0, True)
        counts = []
        for t in range(1, 17):
            m = min((t & -t).bit_length() - 1, top)
            counts.append(ctx.step(p, m, t, t_min, 1, False, want_count=True))
        ctx.drift_all(p)
        ctx.sync()
        inf = ctx.info()
        runs.append((counts, {k: host(p, k).copy() for k in keys}, inf))
    (c0, s0, i0), (c1, s1, i1) = runs
    print("active per sub-step", c0, "builds", i0["full_builds"], i1["full_builds"], flush=True)
    # the two runs differ by rounding only: the lazy drift adds each
    # particle's motion over several sub-steps at once, so its h prediction
    # and positions round differently, and the accelerations (FP32) that
    # feed the kicks follow; a missed or repeated drift would move a particle
    # by |vf| t_min (about 1e-6 here)
    dx = max(np.max(np.minimum(np.abs(s0[k] - s1[k]), 1.0 - np.abs(s0[k] - s1[k]))) for k in ("x", "y", "z"))
    dv = np.max(np.abs(s0["vx"] - s1["vx"])) / np.max(np.abs(s0["vx"]))
    dvf = np.max(np.abs(s0["vfx"] - s1["vfx"])) / np.max(np.abs(s0["vfx"]))
    rel = {k: float(np.max(np.abs(s1[k] / s0[k] - 1))) for k in ("A", "h", "rho", "vsig")}
    print(f"t_min {t_min:.3e} max |dx| {dx:.2e} dv {dv:.2e} dvf {dvf:.2e} {rel}", flush=True)
    assert c0 == c1 and sum(c0) > 0
    assert np.array_equal(s0["time_bin"], s1["time_bin"])
    assert dx < 1e-9 and dv < 1e-6 and dvf < 1e-6
    for k in ("A", "h", "rho", "vsig"):
        assert rel[k] < 1e-5, k
    a0 = np.stack([s0[k] for k in ("ax", "ay", "az")], 1).astype(np.float64)
    a1 = np.stack([s1[k] for k in ("ax", "ay", "az")], 1).astype(np.float64)
    assert np.linalg.norm(a1 - a0) < 1e-5 * np.linalg.norm(a0)


@pytest.mark.parametrize("growth", [1.015, 1.3])
def test_force_counts_after_h_growth_on_kept_cells(gpu_lib, growth):
    """The force loop reads a partner leaf beyond H_i only up to the rank of
    its H order past which no particle's H can reach the gap.  After the
    smoothing lengths on kept cells grow by up to `growth` (below the re-key
    margin the growth bound scales the keys, above it the orders are keyed
    again from the current H), the counts of a deep time-bin are still those
    of the all-pairs definition."""
    sg = gpu_lib
    ic = ics.clustered(n_total=20000, n_clumps=3)
    m = ics.deep_bin_for_fraction(ic["bin"], 0.05)
    print(f"case clustered20k h growth {growth} m={m}", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    rng = np.random.default_rng(11)
    fac = torch.as_tensor(rng.uniform(1.0, growth, p.n).astype(np.float32), device="cuda")
    p["h"].mul_(fac)
    ctx.build_cells(p)
    assert ctx.info()["cell_updates"] == 1
    ctx.sort_cells()
    ctx.mark_active(p, m)
    ctx.density_pass(p, False)
    ctx.force_pass(p)
    ctx.sync()
    cl = emu.build_cells(ic["x"], ic["h"], split=400, D=16)
    assert np.array_equal(perm.cpu().numpy(), cl["perm"])
    H = (np.float32(1.825742) * host(p, "h")).astype(np.float32)
    act = emu.mark_active(cl, ic["bin"][cl["perm"]], m, H=H)
    idx = np.nonzero(act["active"])[0]
    assert 0 < idx.size < p.n
    assert np.array_equal(host(p, "nngb_density")[idx], emu.counts(cl, "density", idx, H=H))
    assert np.array_equal(host(p, "nngb_force")[idx], emu.counts(cl, "force", idx, H=H))
