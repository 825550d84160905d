"""Pins of the bit-exact CPU definitions (oracle/cells.c): invariants of the
cell build, axis-sort order, active masks, cell-pair coverage and FP32 counts
against the FP64 oracle's neighbour sets.  CPU only."""
import math

import numpy as np
import pytest
import torch

import ics
from oracle import cells, grad, sph

D = 21


def _deinterleave(key):
    k = [0, 0, 0]
    key = int(key)
    for b in range(D):
        k[0] |= ((key >> (3 * b + 2)) & 1) << b
        k[1] |= ((key >> (3 * b + 1)) & 1) << b
        k[2] |= ((key >> (3 * b)) & 1) << b
    return k


@pytest.fixture(scope="module")
def clustered_small():
    c = ics.clustered(n_total=20000, n_clumps=3)
    cl = cells.build_cells(c["x"], c["h"], split=64)
    return c, cl


def test_build_invariants(clustered_small):
    c, cl = clustered_small
    n = c["x"].shape[0]
    perm, key = cl["perm"], cl["key"].astype(object)
    assert sorted(perm.tolist()) == list(range(n))
    # order by (key, original index)
    order = sorted(range(n), key=lambda s: (int(cl["key"][s]), int(perm[s])))
    assert order == list(range(n))
    # integer coordinates of each particle reproduce its key and are the
    # truncated scaled wrapped position
    xw = np.stack([cl["xw"], cl["yw"], cl["zw"]], 1)
    assert np.array_equal(xw, np.mod(c["x"][perm], 1.0))
    for s in range(0, n, 97):
        k = _deinterleave(cl["key"][s])
        assert k == [min(int(math.floor(xw[s, a] * 2 ** D)), 2 ** D - 1) for a in range(3)]
    # leaves tile [0, n) in order; each leaf box contains its particles;
    # no leaf is splittable; every leaf's parent was full enough to split
    b, cnt, lv = cl["leaf_begin"], cl["leaf_count"], cl["leaf_level"]
    assert b[0] == 0 and np.all(b[1:] == b[:-1] + cnt[:-1]) and b[-1] + cnt[-1] == n
    assert np.all(cnt < 64) or np.all(lv[cnt >= 64] == D)
    assert np.all(lv >= cl["top_level"])
    parent_count = {}
    for l in range(cl["n_leaves"]):
        w = 2 ** (D - lv[l])
        org = np.array([cl["leaf_ix"][l], cl["leaf_iy"][l], cl["leaf_iz"][l]]) * w
        for s in range(b[l], b[l] + cnt[l]):
            k = np.array(_deinterleave(cl["key"][s]))
            assert np.all(k >= org) and np.all(k < org + w)
        if lv[l] > cl["top_level"]:
            pk = (lv[l] - 1, cl["leaf_ix"][l] >> 1, cl["leaf_iy"][l] >> 1, cl["leaf_iz"][l] >> 1)
            parent_count[pk] = parent_count.get(pk, 0) + int(cnt[l])
    # particles in deeper sibling leaves also belong to the parent
    for pk, tot in parent_count.items():
        lvl, ix, iy, iz = pk
        sh = D - lvl
        inside = [(k[0] >> sh, k[1] >> sh, k[2] >> sh) == (ix, iy, iz)
                  for k in (_deinterleave(kk) for kk in cl["key"][::1])]
        assert sum(inside) >= 64
    # offsets: exact FP64 differences rounded once, within the leaf box
    H = cl["H"]
    assert np.array_equal(H, (np.float32(1.825742) * c["h"][perm]).astype(np.float32))
    for l in range(0, cl["n_leaves"], 7):
        half = 0.5 ** (lv[l] + 1)
        s = slice(b[l], b[l] + cnt[l])
        assert np.all(np.abs(cl["ox"][s]) <= half) and np.all(np.abs(cl["oz"][s]) <= half)
    assert 2 <= cl["top_level"] <= 7 and 0.5 ** cl["top_level"] >= H.max()


def test_axis_sort_order(clustered_small):
    _, cl = clustered_small
    order, keys = cells.axis_sort(cl)
    e = cells.axis_vectors()
    # the 13 directions are unit vectors, pairwise non-parallel, first non-zero positive
    assert np.allclose(np.linalg.norm(e.astype(np.float64), axis=1), 1, atol=1e-7)
    g = np.abs(e.astype(np.float64) @ e.astype(np.float64).T)
    assert np.all(g[~np.eye(13, dtype=bool)] < 0.99)
    for l in range(0, cl["n_leaves"], 3):
        b, n = cl["leaf_begin"][l], cl["leaf_count"][l]
        for a in range(13):
            kk = keys[a, b:b + n]
            ref = np.lexsort((np.arange(n), kk))
            assert np.array_equal(order[a, b:b + n], ref)
            # the key is the projection of the offset on the axis
            o = np.stack([cl["ox"][b:b + n], cl["oy"][b:b + n], cl["oz"][b:b + n]], 1).astype(np.float64)
            assert np.allclose(kk, o @ e[a].astype(np.float64), atol=1e-7 * 0.5 ** cl["leaf_level"][l])


def test_active_mask_and_pairs_cover_all_neighbours(clustered_small):
    c, cl = clustered_small
    binsorted = c["bin"][cl["perm"]]
    m = ics.deep_bin_for_fraction(c["bin"], 0.05)
    act = cells.mark_active(cl, binsorted, m)
    assert np.array_equal(act["active"], binsorted <= m)
    leaf_has = np.zeros(cl["n_leaves"], bool)
    leaf_has[cl["leaf_of"][act["active"]]] = True
    assert np.array_equal(np.nonzero(leaf_has)[0], act["active_leaves"])
    for mode in ("density", "force"):
        pa, pb, s = cells.pairs(cl, act, mode)
        got = set(zip(pa.tolist(), pb.tolist()))
        assert len(got) == len(pa)
        # every FP64 neighbour pair of an active particle is covered
        x = np.stack([cl["xw"], cl["yw"], cl["zw"]], 1)
        H = cl["H"].astype(np.float64)
        ia = np.nonzero(act["active"])[0]
        from scipy.spatial import cKDTree
        tree = cKDTree(x, boxsize=1.0)
        rad = H[ia] if mode == "density" else np.full(ia.size, H.max())
        for i, js in zip(ia, tree.query_ball_point(x[ia], rad)):
            for j in js:
                d = x[i] - x[j]
                d -= np.round(d)
                r = math.sqrt(float(d @ d))
                need = r < H[i] if mode == "density" else (r < H[i] or r < H[j])
                if need:
                    assert (cl["leaf_of"][i], cl["leaf_of"][j]) in got
        # shifts are nearest-image centre differences (exact dyadic values)
        for (A, B, sv) in list(zip(pa, pb, s))[::13]:
            ca = (np.array([cl["leaf_ix"][A], cl["leaf_iy"][A], cl["leaf_iz"][A]]) + 0.5) * 0.5 ** cl["leaf_level"][A]
            cb = (np.array([cl["leaf_ix"][B], cl["leaf_iy"][B], cl["leaf_iz"][B]]) + 0.5) * 0.5 ** cl["leaf_level"][B]
            dd = cb - ca
            dd -= np.round(dd)
            assert np.array_equal(sv.astype(np.float64), dd)


def test_cell_update_without_motion_reproduces_the_build(clustered_small):
    c, cl = clustered_small
    xs = np.stack([cl["xw"], cl["yw"], cl["zw"]], 1)
    hs = c["h"][cl["perm"]]
    up, flag = cells.update(cl, xs, hs, xs)
    assert not flag
    for k in ("ox", "oy", "oz", "H", "leaf_hmax"):
        assert np.array_equal(up[k].view(np.uint32), cl[k].view(np.uint32)), k
    assert np.all(up["leaf_dx"] == 0)


def test_cell_update_margins_cover_every_neighbour_pair(clustered_small):
    """Particles moved after the build, cells kept: the drift margins make the
    cell pairs cover every FP64 neighbour pair at the new positions, and a
    large move asks for a rebuild."""
    c, cl = clustered_small
    xs = np.stack([cl["xw"], cl["yw"], cl["zw"]], 1)
    hs = c["h"][cl["perm"]]
    rng = np.random.default_rng(21)
    width = 0.5 ** cl["leaf_level"][cl["leaf_of"]]
    step = (0.1 * width)[:, None] * rng.uniform(-1, 1, size=xs.shape) / math.sqrt(3)
    moved = xs + step
    up, flag = cells.update(cl, moved, hs, xs)
    assert not flag
    assert np.all(up["leaf_dx"] > 0)
    x = np.stack([up["xw"], up["yw"], up["zw"]], 1)
    assert np.all((x >= 0) & (x < 1))
    # offsets are the minimum-image differences to the (unchanged) leaf centres
    lf = cl["leaf_of"]
    cen = (np.stack([cl["leaf_ix"][lf], cl["leaf_iy"][lf], cl["leaf_iz"][lf]], 1) + 0.5) * \
        (0.5 ** cl["leaf_level"][lf])[:, None]
    d = x - cen
    d -= np.round(d)
    assert np.array_equal(up["ox"], d[:, 0].astype(np.float32))
    binsorted = c["bin"][cl["perm"]]
    act = cells.mark_active(up, binsorted, ics.deep_bin_for_fraction(c["bin"], 0.05), H=up["H"])
    H = up["H"].astype(np.float64)
    from scipy.spatial import cKDTree
    tree = cKDTree(x, boxsize=1.0)
    ia = np.nonzero(act["active"])[0]
    for mode in ("density", "force"):
        pa, pb, _ = cells.pairs(up, act, mode, leaf_dx=up["leaf_dx"])
        got = set(zip(pa.tolist(), pb.tolist()))
        p0, _, _ = cells.pairs(up, act, mode)
        assert len(pa) >= len(p0)
        rad = H[ia] if mode == "density" else np.full(ia.size, H.max())
        for i, js in zip(ia, tree.query_ball_point(x[ia], rad)):
            for j in js:
                e = x[i] - x[j]
                e -= np.round(e)
                r = math.sqrt(float(e @ e))
                if (r < H[i]) if mode == "density" else (r < H[i] or r < H[j]):
                    assert (lf[i], lf[j]) in got
    _, flag = cells.update(cl, xs + 3 * step, hs, xs)
    assert flag


def test_fp32_counts_agree_with_fp64_neighbour_sets():
    c = ics.tiny_lattice(16)
    out = sph.solve_density(c["x"], c["v"], c["m"], c["h"], 1.0)
    h = out["h"].numpy()
    cl = cells.build_cells(c["x"], h.astype(np.float32))
    samples = np.arange(0, 4096, 5)
    cnt32 = cells.counts(cl, "density", samples)
    # FP64 counts at the same (float32-rounded) h
    h32 = h.astype(np.float32).astype(np.float64)
    o64 = sph._density_terms(torch.as_tensor(c["x"]), torch.as_tensor(c["v"]),
                             torch.as_tensor(c["m"], dtype=torch.float64),
                             torch.as_tensor(h32 * np.float32(1.825742) / sph.GAMMA_K), 1.0,
                             torch.arange(4096),
                             *map(torch.as_tensor, sph.candidate_pairs(c["x"], 1.0, np.arange(4096),
                                                                        np.float32(1.825742) * h32)))
    cnt64 = o64["count"].numpy()[cl["perm"][samples]]
    assert np.sum(cnt32 != cnt64) <= 2
    assert cnt32.mean() > 40


def test_gradient_matches_finite_differences():
    c = ics.tiny_lattice(6, velocity_sigma=0.3)
    w = np.random.default_rng(7).normal(size=(216, 3))
    gx, gu = grad.gradient(c["x"], c["v"], c["m"], c["u"], c["h"], 1.0, w)
    ps = [0, 17, 100, 201]
    fx, fu = grad.finite_difference(c["x"], c["v"], c["m"], c["u"], c["h"], 1.0, w, ps, 1e-6 / 6)
    assert np.abs(gx[ps] - fx).max() <= 1e-6 * np.abs(fx).max()
    assert np.abs(gu[ps] - fu).max() <= 1e-6 * np.abs(fu).max()


@pytest.mark.parametrize("mode", ["density", "force"])
def test_grid_counts_equal_all_pairs_counts(mode):
    """The grid-pruned counts used on the large workloads equal the
    all-pairs FP32 counts, on a clustered box with grown smoothing lengths
    (leaves of every size class, neighbours across leaf and box faces)."""
    ic = ics.clustered(n_total=12000, n_clumps=3)
    cl = cells.build_cells(ic["x"], ic["h"], split=400, D=16)
    idx = np.arange(0, 12000, 5)
    H = (cl["H"] * np.float32(1.03)).astype(np.float32)
    a = cells.counts(cl, mode, idx, H=H)
    b = cells.counts_grid(cl, mode, idx, H=H)
    assert a.sum() > 0 and np.array_equal(a, b)
