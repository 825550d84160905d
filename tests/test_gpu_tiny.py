"""GPU parity on the tiny workload (16^3 jittered lattice, all active) and
its variants, through the C-ABI."""
import math

import numpy as np
import pytest
import torch

import ics
from oracle import sph
from tests.gpu_cases import (A_TOL, RHO_TOL, check_counts, check_structures, float_errors, host, oracle_all,
                             run_gpu_step)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_tiny_lattice_step(gpu_lib, sigma):
    ic = ics.tiny_lattice(16, velocity_sigma=sigma)
    print(f"case tiny16 sigma={sigma}", flush=True)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, 0)
    cl, act = check_structures(ic, perm, snap)
    check_counts(cl, p, snap, perm, ic, 0)
    out, fo = oracle_all(ic)
    e = float_errors(p, perm, out, fo)
    print({k: f"{v:.2e}" for k, v in e.items()})
    assert e["rho"] < RHO_TOL
    assert e["h"] < 1e-5
    assert e["a"] < A_TOL
    assert e["f"] < 1e-5 and e["P"] < 1e-5 and e["c"] < 1e-5
    assert e["vsig"] < 1e-5
    if sigma > 0:
        assert e["divv"] < 1e-3 and e["curlv"] < 1e-3 and e["B"] < 1e-3 and e["dA_dt"] < 1e-3
    assert snap["info"]["n_unconverged"] == 0


def test_perfect_lattice_counts_and_density(gpu_lib):
    ic = ics.perfect_lattice(16)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, 0)
    # 56 neighbours besides itself for every particle, the lattice root density
    assert np.all(host(p, "nngb_density") == 56)
    rho = host(p, "rho").astype(np.float64)
    assert np.max(np.abs(rho / 1.004021830777798 - 1)) < RHO_TOL
    assert np.max(np.abs(host(p, "h") * 16 / 1.2331490390680415 - 1)) < 1e-5
    a = np.stack([host(p, k) for k in ("ax", "ay", "az")], 1)
    out, fo = oracle_all(ic)
    S = fo["scale"].numpy()[perm]
    assert np.max(np.linalg.norm(a, axis=1) / S) < 1e-6


def test_deterministic(gpu_lib):
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    r = []
    for _ in range(2):
        _, p, perm, _ = run_gpu_step(gpu_lib, ic, 0)
        r.append({k: host(p, k).copy() for k in ("h", "rho", "ax", "ay", "az", "dA_dt", "vsig", "nngb_force")})
    for k in r[0]:
        assert np.array_equal(r[0][k].view(np.uint8), r[1][k].view(np.uint8)), k


def _step_with_tiling(sg, ic, path, nw, ordered, persistent):
    """build -> sort -> mark (all active) -> density -> force with the chunk
    loops only, every pass at the tiling (nw, tile 0, ordered, persistent)."""
    with open(path, "w") as f:
        for loop in (0, 1):
            for cls in range(32):
                f.write(f"best {loop} {cls} {nw} 0 {ordered} {persistent} 0 0 0\n")
    ctx = sg.Context(sweep_below=0)
    ctx.load_tuning(str(path))
    p = sg.Particles.from_initial(ic)
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, 0)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    return {k: host(p, k).copy() for k in ("h", "rho", "f_gradh", "ax", "ay", "az", "dA_dt", "vsig",
                                           "nngb_density", "nngb_force")}


@pytest.mark.parametrize("nw", [1, 4])
def test_work_order_does_not_change_bits(gpu_lib, tmp_path, nw):
    """The chunk loops' work items in other orders: the natural chunk order,
    the cost-ordered list, and a persistent grid pulling items from one
    counter (an order that changes from run to run, run twice here).  Each
    chunk forms its particles' sums within itself in a fixed order, so every
    result is the same to the bit."""
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    ref = _step_with_tiling(gpu_lib, ic, tmp_path / "t00.txt", nw, 0, 0)
    for ordered, persistent in ((1, 0), (0, 1), (1, 1), (1, 1)):
        out = _step_with_tiling(gpu_lib, ic, tmp_path / f"t{ordered}{persistent}.txt", nw, ordered, persistent)
        for k in ref:
            assert np.array_equal(ref[k].view(np.uint8), out[k].view(np.uint8)), (k, ordered, persistent)


def test_kick_drift_matches_oracle(gpu_lib):
    """kick_drift alone, on synthetic accelerations, smoothing lengths and
    signal speeds (seeded), bit for bit against the FP64 definition."""
    ic = ics.tiny_lattice(16, velocity_sigma=0.2)
    rng = np.random.default_rng(11)
    N = ic["x"].shape[0]
    ic["bin"] = rng.integers(0, 6, size=N).astype(np.int8)
    m_bin = 3
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, m_bin)
    a = rng.normal(size=(N, 3)).astype(np.float32)
    dA = rng.normal(size=N).astype(np.float32)
    h = rng.uniform(0.05, 0.1, size=N).astype(np.float32)
    vs = rng.uniform(0.5, 5.0, size=N).astype(np.float32)
    vs[::17] = 0.0
    Af = rng.uniform(0.5, 1.5, size=N).astype(np.float32)
    dv = rng.normal(scale=300.0, size=N).astype(np.float32)
    p["divv"].copy_(torch.from_numpy(dv))
    for d, k in enumerate(("ax", "ay", "az")):
        p[k].copy_(torch.from_numpy(a[:, d]))
    p["dA_dt"].copy_(torch.from_numpy(dA))
    p["h"].copy_(torch.from_numpy(h))
    p["vsig"].copy_(torch.from_numpy(vs))
    p["Af"].copy_(torch.from_numpy(Af))
    p["A"].copy_(torch.from_numpy(Af))
    x0 = np.stack([host(p, k) for k in "xyz"], 1)
    vf0 = np.stack([host(p, k) for k in ("vfx", "vfy", "vfz")], 1)
    vp0 = np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1)
    bins0 = host(p, "time_bin").astype(np.int64)
    act = snap["active"]
    t_min, ti, drift = 1e-4, 24, 8
    ctx.kick_drift(p, ti, t_min, drift, False)
    ctx.sync()
    ref = sph.kick_drift(x0, vf0, vp0, Af.astype(np.float64), Af.astype(np.float64), a, dA, h, vs, bins0, act, ti,
                         t_min, drift, 1.0, divv=dv)
    assert np.array_equal(host(p, "time_bin").astype(np.int64), ref["bins"])
    assert np.array_equal(np.stack([host(p, k) for k in "xyz"], 1), ref["x"])
    assert np.array_equal(np.stack([host(p, k) for k in ("vfx", "vfy", "vfz")], 1), ref["vf"])
    assert np.array_equal(np.stack([host(p, k) for k in ("vx", "vy", "vz")], 1), ref["vp"])
    assert np.array_equal(host(p, "Af"), ref["Af"].astype(np.float32))
    assert np.array_equal(host(p, "A"), ref["Ap"].astype(np.float32))
    # h after the predicted drift: exp in double on both sides, rounded to float
    hg = host(p, "h").view(np.int32).astype(np.int64)
    hr = ref["h"].astype(np.float32).view(np.int32).astype(np.int64)
    assert np.max(np.abs(hg - hr)) <= 1


def test_call_order_and_argument_errors(gpu_lib):
    sg = gpu_lib
    ic = ics.tiny_lattice(16)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    with pytest.raises(sg.SPHError) as e:
        ctx.density_pass(p, True)
    assert e.value.code == -6
    ctx.build_cells(p)
    ctx.sort_cells()
    with pytest.raises(sg.SPHError) as e:
        ctx.mark_active(p, 14)
    assert e.value.code == -1
    with pytest.raises(sg.SPHError) as e:
        ctx.force_pass(p)
    assert e.value.code == -6
    # a box too small for the smoothing lengths
    big = dict(ic)
    big["h"] = np.full_like(ic["h"], 0.2)
    pb = sg.Particles.from_initial(big)
    with pytest.raises(sg.SPHError) as e:
        ctx.build_cells(pb)
    assert e.value.code == -1
    # non-convergence reported with a tiny iteration budget
    ctx2 = sg.Context(h_max_iter=1)
    ic2 = dict(ic)
    ic2["h"] = (ic["h"] * 1.3).astype(np.float32)
    p2 = sg.Particles.from_initial(ic2)
    ctx2.build_cells(p2)
    ctx2.sort_cells()
    ctx2.mark_active(p2, 0)
    with pytest.raises(sg.SPHError) as e:
        ctx2.density_pass(p2, True)
    assert e.value.code == -4
    assert ctx2.info()["n_unconverged"] > 0


@pytest.mark.parametrize("nw,split,sweep", [(1, 0, 0), (2, 0, 0), (4, 0, 0), (8, 0, 0), (1, 1, 0), (2, 2, 0),
                                             (4, 1, 0), (8, 1, 0), (4, 0, 1 << 30)])
def test_waves_per_chunk_variants_agree(gpu_lib, nw, split, sweep):
    """Every loop tiling (waves per chunk, candidate/list capacities, chunks
    split into parts of their cell-pair lists, one wave per particle) gives
    the same neighbour counts and the same sums to rounding."""
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    _, p0, perm0, _ = run_gpu_step(gpu_lib, ic, 0, ctx_kw=dict(waves_per_chunk=1, cand_cap=2048, list_cap=192,
                                                               sweep_below=0))
    _, p1, perm1, _ = run_gpu_step(gpu_lib, ic, 0, ctx_kw=dict(waves_per_chunk=nw, cand_cap=256, list_cap=64,
                                                               chunk_split=split, sweep_below=sweep))
    assert np.array_equal(perm0, perm1)
    for k in ("nngb_density", "nngb_force"):
        assert np.array_equal(host(p0, k), host(p1, k)), k
    for k in ("h", "rho", "vsig"):
        assert np.max(np.abs(host(p0, k) / host(p1, k) - 1)) < 2e-6, k
    a0 = np.stack([host(p0, k) for k in ("ax", "ay", "az")], 1)
    a1 = np.stack([host(p1, k) for k in ("ax", "ay", "az")], 1)
    assert np.max(np.linalg.norm(a0 - a1, axis=1)) < 1e-5 * np.max(np.linalg.norm(a0, axis=1))


@pytest.mark.parametrize("eta,h_scale", [(None, 1.0), (None, 1.25), (None, 0.8), (1.9, 1.0)])
def test_sweep_solver_steps_match_chunk_loop(gpu_lib, eta, h_scale):
    """The density sweep (one wave per particle) takes the h solve's Newton
    steps on the neighbours it keeps within 1.1 H and leaves the last one to
    the ghost.  Starting h off the root (x1.25, x0.8), and with eta 1.9
    (about 200 neighbours: more within 1.1 H than the sweep keeps, and a
    first step that leaves the reach of the cell-pair lists, which are then
    widened), it gives the converged h, the neighbour counts and the sums of
    the chunk loop (one step per pass) and of the sweep with two waves per
    particle (no steps of its own), in no more passes.  With sweep_below 2000
    the chunk loop takes the first passes and, once fewer particles are left
    (a count known only on the device), the sweep over the particles whose
    flag says they are not done takes the rest: the same results again."""
    ic = ics.tiny_lattice(24, velocity_sigma=0.1)
    ic["h"] = (ic["h"] * h_scale).astype(np.float32)
    kw = {} if eta is None else {"eta": eta}
    print(f"case tiny24 eta={eta} h_scale={h_scale}", flush=True)
    runs = []
    for extra in (dict(sweep_below=0), dict(), dict(sweep_waves=2), dict(sweep_below=2000)):
        _, p, perm, snap = run_gpu_step(gpu_lib, ic, 0, ctx_kw={**kw, **extra})
        runs.append((p, perm, snap["info"]))
    (p0, perm0, i0), (p1, perm1, i1), (p2, perm2, i2), (p3, perm3, i3) = runs
    assert np.array_equal(perm0, perm1) and np.array_equal(perm0, perm2) and np.array_equal(perm0, perm3)
    print("passes", [r[2]["density_iterations"] for r in runs], "rebuilds", [r[2]["pair_rebuilds"] for r in runs],
          "unconverged after pass", i3["unconverged_after_pass"])
    for info in (i0, i1, i2, i3):
        assert info["n_unconverged"] == 0
    assert i1["density_iterations"] <= i0["density_iterations"]
    if eta is not None:
        # at least 150 within H, so above 192 within 1.1 H
        assert min(host(p0, "nngb_density")) > 150
    for pq in (p1, p2, p3):
        for k in ("nngb_density", "nngb_force"):
            assert np.array_equal(host(p0, k), host(pq, k)), k
        for k in ("h", "rho", "vsig"):
            assert np.max(np.abs(host(p0, k) / host(pq, k) - 1)) < 2e-6, k
        a0 = np.stack([host(p0, k) for k in ("ax", "ay", "az")], 1)
        a1 = np.stack([host(pq, k) for k in ("ax", "ay", "az")], 1)
        assert np.max(np.linalg.norm(a0 - a1, axis=1)) < 1e-5 * np.max(np.linalg.norm(a0, axis=1))


def test_autotune_keeps_results(gpu_lib, tmp_path):
    """Tuning picks a loop configuration per pass; passes run with it give
    the same counts and the same sums to rounding."""
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, 0)
    ref = {k: host(p, k).copy() for k in ("rho", "ax", "nngb_density", "nngb_force")}
    path = str(tmp_path / "tune.txt")
    ctx.autotune(p, path)
    lines = open(path).read().splitlines()
    assert sum(l.startswith("best") for l in lines) == 2
    assert sum(l.startswith("candidate") for l in lines) >= 2 * 24
    # a fresh context with the loaded table reproduces the step
    ctx2, p2, perm2, _ = run_gpu_step(gpu_lib, ic, 0)
    ctx3 = gpu_lib.Context()
    ctx3.load_tuning(path)
    p3 = gpu_lib.Particles.from_initial(ic)
    ctx3.build_cells(p3)
    ctx3.sort_cells()
    ctx3.mark_active(p3, 0)
    ctx3.density_pass(p3, True)
    ctx3.force_pass(p3)
    ctx3.sync()
    assert np.array_equal(host(p3, "nngb_density"), ref["nngb_density"])
    assert np.array_equal(host(p3, "nngb_force"), ref["nngb_force"])
    assert np.max(np.abs(host(p3, "rho") / ref["rho"] - 1)) < 2e-6


def test_unsorted_small_leaves_match_full_sorts(gpu_lib):
    """A deep-bin step on the sorts of the full build (leaves of at most two
    tiles are not sorted: the loops read them whole) gives the same bits as
    the step after a sort of every leaf."""
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    ic["bin"] = np.random.default_rng(7).integers(0, 6, size=ic["x"].shape[0]).astype(np.int8)
    out = []
    for full in (False, True):
        p = sg.Particles.from_initial(ic)
        ctx = sg.Context(split_count=64)
        ctx.build_cells(p)
        ctx.sort_cells()
        ctx.mark_active(p, ctx.params.n_bins - 1)
        ctx.density_pass(p, True)
        ctx.force_pass(p)
        ctx.build_cells(p)
        ctx.sort_cells()
        if full:
            ctx.copy_axis_order()
        ctx.mark_active(p, 0)
        ctx.density_pass(p, False)
        ctx.force_pass(p)
        ctx.sync()
        out.append({k: host(p, k).copy() for k in ("h", "rho", "ax", "ay", "az", "vsig", "nngb_density", "nngb_force")})
    for k in out[0]:
        assert np.array_equal(out[0][k].view(np.uint8), out[1][k].view(np.uint8)), k


def test_step_call_equals_separate_calls(gpu_lib):
    """sph_step gives the same bits as its six calls made one by one, over two
    steps (the second on kept cells)."""
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    ic["bin"] = np.random.default_rng(3).integers(0, 4, size=ic["x"].shape[0]).astype(np.int8)
    out = []
    for fused in (False, True):
        p = sg.Particles.from_initial(ic)
        ctx = sg.Context(split_count=64)
        for t, (m, first) in enumerate(((ctx.params.n_bins - 1, True), (0, False))):
            if fused:
                ctx.step(p, m, t, 1e-4, 1, first, entropy_from_u=first)
            else:
                ctx.build_cells(p)
                ctx.sort_cells()
                ctx.mark_active(p, m)
                ctx.density_pass(p, first)
                ctx.force_pass(p)
                ctx.kick_drift(p, t, 1e-4, 1, first)
        ctx.sync()
        out.append({k: host(p, k).copy() for k in ("x", "vx", "h", "rho", "ax", "vsig", "time_bin", "nngb_force")})
    for k in out[0]:
        assert np.array_equal(out[0][k].view(np.uint8), out[1][k].view(np.uint8)), k


def test_next_active_time_matches_oracle(gpu_lib):
    """sph_next_active_time against the oracle's scan of Sec. II-A's
    activity rule, on one context and on a batch context of three boxes
    (the earliest over the boxes)."""
    sg = gpu_lib
    ic = ics.tiny_lattice(12)
    n = ic["x"].shape[0]
    print("case next_active_time tiny12 and a batch of 3", flush=True)
    rng = np.random.default_rng(4)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    ctx.build_cells(p)
    for trial in range(12):
        lo = int(rng.integers(0, 14))
        bins = rng.integers(lo, 14, size=n)
        p["time_bin"].copy_(torch.from_numpy(bins.astype(np.int8)))
        for t0 in (0, int(rng.integers(1, 1 << 13)), (1 << 13) - 1):
            assert ctx.next_active_time(p, t0) == sph.next_active_time(bins, t0), (trial, t0)
    boxes = [ics.tiny_lattice(10), ics.tiny_lattice(12), ics.tiny_lattice(11)]
    sizes = [b["x"].shape[0] for b in boxes]
    cat = {k: np.concatenate([b[k] for b in boxes]) for k in ("x", "v", "m", "u", "h", "bin")}
    P = sg.Particles.from_initial(cat)
    bctx = sg.Context().batch_create(sizes)
    bctx.build_cells(P)
    for trial in range(6):
        bins = rng.integers(int(rng.integers(0, 14)), 14, size=sum(sizes))
        P["time_bin"].copy_(torch.from_numpy(bins.astype(np.int8)))
        t0 = int(rng.integers(0, 1 << 13))
        assert bctx.next_active_time(P, t0) == sph.next_active_time(bins, t0), trial
    with pytest.raises(sg.SPHError):
        ctx.next_active_time(p, -1)
