"""GPU parity of the batched passes: one launch per loop pass over many
boxes equals each box's own passes run with the same loop tiling (bitwise),
and small all-active boxes match the FP64 oracle."""
import numpy as np
import pytest
import torch

import ics
from tests.gpu_cases import A_TOL, RHO_TOL, float_errors, host, oracle_all

pytestmark = pytest.mark.gpu

TILING = dict(waves_per_chunk=4, cand_cap=256, list_cap=64, sweep_below=0)
OUTPUTS = ("h", "rho", "drho_dh", "f_gradh", "divv", "curlx", "curly", "curlz", "P", "c", "balsara", "A",
           "ax", "ay", "az", "dA_dt", "du_dt", "vsig", "nngb_density", "nngb_force")


def prepare(sg, boxes, bins_m, kw):
    """Per box: build, sort, an all-active density pass (state for every
    particle), then mark the box's bin.  Returns contexts, particles, perms."""
    cs, ps, perms = [], [], []
    for b, m in zip(boxes, bins_m):
        p = sg.Particles.from_initial(b)
        c = sg.Context(**kw)
        perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
        c.build_cells(p, perm)
        c.sort_cells()
        c.mark_active(p, c.params.n_bins - 1)
        c.density_pass(p, True)
        c.mark_active(p, m)
        cs.append(c)
        ps.append(p)
        perms.append(perm)
    return cs, ps, perms


def snapshot(ps):
    return [{k: host(p, k).copy() for k in OUTPUTS} for p in ps]


@pytest.mark.parametrize("split", [0, 1])
def test_batch_equals_separate_passes_64_boxes(gpu_lib, split):
    sg = gpu_lib
    boxes = ics.batch_of_boxes()
    ms = [ics.deep_bin_for_fraction(b["bin"], b["target_active_fraction"]) for b in boxes]
    print(f"case batch64 N={sum(b['x'].shape[0] for b in boxes)} split={split}", flush=True)
    tiling = dict(TILING, chunk_split=split)
    cs, ps, _ = prepare(sg, boxes, ms, tiling)
    for c, p in zip(cs, ps):
        c.density_pass(p, False)
        c.force_pass(p)
    torch.cuda.synchronize()
    ref = snapshot(ps)
    ref_info = [c.info() for c in cs]
    del cs, ps
    cs, ps, _ = prepare(sg, boxes, ms, tiling)
    batch = sg.Batch(cs, ps)
    batch.density_pass(False)
    batch.force_pass()
    torch.cuda.synchronize()
    got = snapshot(ps)
    for b in range(len(boxes)):
        inf = cs[b].info()
        assert inf["n_active"] == ref_info[b]["n_active"]
        assert inf["density_iterations"] == ref_info[b]["density_iterations"], b
        assert inf["n_force_pairs"] == ref_info[b]["n_force_pairs"], b
        for k in OUTPUTS:
            assert np.array_equal(got[b][k].view(np.uint8), ref[b][k].view(np.uint8)), (b, k)


def small_boxes(n=4):
    boxes = ics.batch_of_boxes(n_boxes=n, n_range=(1_000, 4_000), frac_range=(1.0, 1.0))
    for b in boxes:
        b["bin"] = np.zeros_like(b["bin"])
        b["u"] = np.ones_like(b["u"])
    return boxes


def test_batch_small_boxes_match_oracle(gpu_lib):
    sg = gpu_lib
    boxes = small_boxes(4)
    # a fifth box with nothing active: bins all 3, marked at bin 0
    empty = dict(boxes[0])
    empty["bin"] = np.full_like(boxes[0]["bin"], 3)
    boxes.append(empty)
    ms = [0, 0, 0, 0, 0]
    print("case batch small 4+1", flush=True)
    cs, ps, perms = [], [], []
    for b, m in zip(boxes, ms):
        p = sg.Particles.from_initial(b)
        c = sg.Context()
        perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
        c.build_cells(p, perm)
        c.sort_cells()
        c.mark_active(p, m)
        cs.append(c)
        ps.append(p)
        perms.append(perm.cpu().numpy())
    batch = sg.Batch(cs, ps)
    batch.density_pass(True)
    batch.force_pass()
    torch.cuda.synchronize()
    assert cs[4].info()["n_active"] == 0
    assert cs[4].info()["n_force_pairs"] == 0
    for b in range(4):
        out, fo = oracle_all(boxes[b])
        e = float_errors(ps[b], perms[b], out, fo)
        print(b, {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        assert e["rho"] < RHO_TOL and e["a"] < A_TOL and e["h"] < 1e-5


def test_batch_autotune_and_reload(gpu_lib, tmp_path):
    sg = gpu_lib
    boxes = small_boxes(6)
    ms = [0] * len(boxes)
    cs, ps, _ = prepare(sg, boxes, ms, {})
    batch = sg.Batch(cs, ps)
    batch.density_pass(False)
    batch.force_pass()
    ref = snapshot(ps)
    path = str(tmp_path / "batch_tune.txt")
    batch.autotune(path)
    lines = open(path).read().splitlines()
    assert sum(l.startswith("batch_best") for l in lines) == 2
    # 2 loops x 3 split classes x 2 launch styles x 11 (waves, tile) pairs that fit the LDS
    assert sum(l.startswith("batch_candidate") for l in lines) == 2 * 3 * 2 * 11
    # the tuned tiling gives the same counts, and the same densities within
    # the solve's tolerance (another summation order can end the Newton
    # iteration one step apart)
    cs2, ps2, _ = prepare(sg, boxes, ms, {})
    cs2[0].load_tuning(path)
    b2 = sg.Batch(cs2, ps2)
    b2.density_pass(False)
    b2.force_pass()
    got = snapshot(ps2)
    for b in range(len(boxes)):
        assert np.array_equal(got[b]["nngb_density"], ref[b]["nngb_density"])
        assert np.array_equal(got[b]["nngb_force"], ref[b]["nngb_force"])
        assert np.max(np.abs(got[b]["rho"] / ref[b]["rho"] - 1)) < RHO_TOL


def test_batch_argument_errors(gpu_lib):
    sg = gpu_lib
    boxes = small_boxes(2)
    cs, ps, _ = prepare(sg, boxes, [0, 0], {})
    with pytest.raises(sg.SPHError) as e:
        sg.Batch([cs[0], cs[0]], [ps[0], ps[0]]).density_pass(False)
    assert e.value.code == -1
    with pytest.raises(sg.SPHError) as e:
        sg.Batch(cs, ps).force_pass()   # marked, but no density pass since
    assert e.value.code == -6
    p = sg.Particles.from_initial(boxes[0])   # built and sorted, never marked
    c = sg.Context()
    c.build_cells(p)
    c.sort_cells()
    with pytest.raises(sg.SPHError) as e:
        sg.Batch([cs[0], c], [ps[0], p]).density_pass(False)
    assert e.value.code == -6


def test_h_solve_converges_where_a_clamped_step_cycled(gpu_lib):
    """Box 10 of the 64-box workload (1,158 particles): one particle's
    clamped Newton step used to jump between two earlier iterates (x2, then
    x0.5) for the whole iteration budget.  Regression test of the strict
    bracket."""
    sg = gpu_lib
    box = ics.batch_of_boxes()[10]
    p = sg.Particles.from_initial(box)
    c = sg.Context()
    c.build_cells(p)
    c.sort_cells()
    c.mark_active(p, c.params.n_bins - 1)
    c.density_pass(p, True)
    inf = c.info()
    assert inf["n_unconverged"] == 0 and inf["density_iterations"] <= 12


def test_batch_of_more_boxes_than_host_slots(gpu_lib):
    """70 small all-active boxes: the batched force pass reads the boxes' cell
    pair totals in groups of 64; results equal the boxes' own passes bitwise."""
    sg = gpu_lib
    boxes = ics.batch_of_boxes(n_boxes=70, n_range=(2_000, 4_000), frac_range=(1.0, 1.0))
    for b in boxes:
        b["bin"] = np.zeros_like(b["bin"])
    ms = [0] * len(boxes)
    print(f"case batch70 N={sum(b['x'].shape[0] for b in boxes)}", flush=True)
    cs, ps, _ = prepare(sg, boxes, ms, TILING)
    for c, p in zip(cs, ps):
        c.density_pass(p, False)
        c.force_pass(p)
    torch.cuda.synchronize()
    ref = snapshot(ps)
    del cs, ps
    cs, ps, _ = prepare(sg, boxes, ms, TILING)
    batch = sg.Batch(cs, ps)
    batch.density_pass(False)
    batch.force_pass()
    torch.cuda.synchronize()
    got = snapshot(ps)
    for b in range(len(boxes)):
        for k in OUTPUTS:
            assert np.array_equal(got[b][k].view(np.uint8), ref[b][k].view(np.uint8)), (b, k)
