"""GPU parity on a small clustered workload: several radix tiles, leaves of
every size class, a deep time-bin with few active particles."""
import numpy as np
import pytest

import ics
from oracle import sph
from tests.gpu_cases import (A_TOL, RHO_TOL, check_counts, check_structures, float_errors, host, run_gpu_step)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clustered20k():
    return ics.clustered(n_total=20000, n_clumps=3)


@pytest.mark.parametrize("frac", [1.0, 0.05])
def test_clustered_step(gpu_lib, clustered20k, frac):
    ic = clustered20k
    m = ics.N_BINS - 1 if frac >= 1.0 else ics.deep_bin_for_fraction(ic["bin"], frac)
    print(f"case clustered20k frac={frac} m={m}", flush=True)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, m, setup_all=frac < 1.0)
    cl, act = check_structures(ic, perm, snap, m_bin=m)
    assert cl["leaf_count"].max() > 64          # the multi-element sort widths ran
    check_counts(cl, p, snap, perm, ic, m)
    # oracle: every active particle and every particle within reach of one
    active = snap["active"]
    idx = np.nonzero(active)[0]
    orig = perm[idx]
    from scipy.spatial import cKDTree
    tree = cKDTree(ic["x"], boxsize=1.0)
    reach = 1.5 * sph.GAMMA_K * float(ic["h"].max())
    near = np.unique(np.concatenate(list(tree.query_ball_point(ic["x"][orig], reach)) + [orig]))
    out = sph.density_and_ghost(ic["x"], ic["v"], ic["m"], ic["h"], 1.0, u=ic["u"], centres=near)
    import torch
    N = ic["x"].shape[0]
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
    print({k: f"{v:.2e}" for k, v in e.items()})
    assert e["rho"] < RHO_TOL and e["h"] < 1e-5 and e["a"] < A_TOL
    assert snap["info"]["n_unconverged"] == 0


def test_clustered_full_size_deep_bin(gpu_lib):
    """The benchmark's workload at its full size and launch configuration
    (default parameters, 2,097,152 particles, the deep bin with about 1 %
    active): every structure bit-exact against the C definitions, neighbour
    counts of a sample exact, and the sample's density and force against
    the FP64 oracle."""
    ic = ics.clustered()
    m = ics.deep_bin_for_fraction(ic["bin"], 0.01)
    print(f"case clustered full N={ic['x'].shape[0]} m={m}", flush=True)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, m, setup_all=True)
    cl, act = check_structures(ic, perm, snap, m_bin=m)
    active = np.nonzero(snap["active"])[0]
    assert 0.005 < active.size / ic["x"].shape[0] < 0.02
    # a sample of 48 active particles around one of them (one clump keeps the
    # oracle's set of particles within reach small)
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(17)
    xa = ic["x"][perm[active]]
    seed = int(rng.integers(active.size))
    _, nn = cKDTree(xa, boxsize=1.0).query(xa[seed], k=48)
    idx = np.sort(active[nn])
    check_counts(cl, p, snap, perm, ic, m, samples=idx)
    orig = perm[idx]
    tree = cKDTree(ic["x"], boxsize=1.0)
    reach = 1.5 * sph.GAMMA_K * float(ic["h"].max())
    near = np.unique(np.concatenate(list(tree.query_ball_point(ic["x"][orig], reach)) + [orig]))
    print(f"oracle set {near.size}", flush=True)
    out = sph.density_and_ghost(ic["x"], ic["v"], ic["m"], ic["h"], 1.0, u=ic["u"], centres=near)
    import torch
    N = ic["x"].shape[0]
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
    assert snap["info"]["n_unconverged"] == 0
