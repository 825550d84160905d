"""GPU parity on the large single-GPU share at full size (16,777,216
particles of the Zel'dovich-displaced 256^3 lattice), in the launch
configuration of its benchmark: the cell build bit-exact against the C
definitions, and an all-active density and force step checked on a sample
in the densest region (exact neighbour counts, physics against the FP64
oracle)."""
import numpy as np
import pytest
import torch

import ics
from oracle import cells as emu
from oracle import sph
from tests.gpu_cases import A_TOL, RHO_TOL, float_errors, host

pytestmark = pytest.mark.gpu


def test_large_share_full_size_all_active(gpu_lib):
    sg = gpu_lib
    ic = ics.grf_zeldovich()
    N = ic["x"].shape[0]
    print(f"case large share N={N}", flush=True)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    perm = torch.empty(N, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ctx.sync()
    perm = perm.cpu().numpy()
    cl = emu.build_cells(ic["x"], ic["h"], split=400, D=16)
    assert np.array_equal(perm, cl["perm"])
    keys, o = ctx.copy_particles()
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), cl["key"])
    for d, k in enumerate(("ox", "oy", "oz")):
        assert np.array_equal(o[d].cpu().numpy().view(np.uint32), cl[k].view(np.uint32)), k
    lv = {k: v.cpu().numpy() for k, v in ctx.copy_leaves().items()}
    assert np.array_equal(lv["begin"], cl["leaf_begin"]) and np.array_equal(lv["count"], cl["leaf_count"])
    assert np.array_equal(lv["level"], cl["leaf_level"])
    # the sample: the particle of smallest h (densest region) and its 47
    # nearest neighbours, in cell order
    from scipy.spatial import cKDTree
    xs = np.stack([host(p, k) for k in "xyz"], 1)
    h_ic_sorted = ic["h"][perm]
    _, nn = cKDTree(xs, boxsize=1.0).query(xs[int(np.argmin(h_ic_sorted))], k=48)
    idx = np.sort(nn)
    H = (np.float32(1.825742) * host(p, "h")).astype(np.float32)
    assert np.array_equal(host(p, "nngb_density")[idx], emu.counts(cl, "density", idx, H=H))
    assert np.array_equal(host(p, "nngb_force")[idx], emu.counts(cl, "force", idx, H=H))
    orig = perm[idx]
    tree = cKDTree(ic["x"], boxsize=1.0)
    reach = 1.5 * sph.GAMMA_K * float(ic["h"].max())
    near = np.unique(np.concatenate(list(tree.query_ball_point(ic["x"][orig], reach)) + [orig]))
    print(f"oracle set {near.size}", flush=True)
    out = sph.density_and_ghost(ic["x"], ic["v"], ic["m"], ic["h"], 1.0, u=ic["u"], centres=near)
    full = {}
    for k in ("h", "rho", "drho_dh", "f", "P", "c", "B", "divv"):
        a = torch.full((N,), float("nan"), dtype=torch.float64)
        a[torch.as_tensor(near)] = out[k]
        full[k] = a
    cv = torch.full((N, 3), float("nan"), dtype=torch.float64)
    cv[torch.as_tensor(near)] = out["curlv"]
    full["curlv"] = cv
    fo = sph.force(ic["x"], ic["v"], ic["m"], full["h"], full["rho"], full["f"], full["P"], full["c"], full["B"],
                   1.0, centres=orig)
    e = float_errors(p, perm, full, fo, idx_sorted=idx, fo_aligned=True)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    assert e["rho"] < RHO_TOL and e["h"] < 1e-5 and e["a"] < A_TOL
    assert ctx.info()["n_unconverged"] == 0
