"""Shared drivers of the GPU parity tests: run the HIP path on a workload,
run the oracle on the same inputs, and compare in cell order."""
import numpy as np
import torch

from oracle import cells as emu
from oracle import sph

A_TOL = 1e-4      # accelerations, relative to max(|a_ref|, 1e-2 * S_i)
RHO_TOL = 1e-5    # density, relative


def run_gpu_step(sg, ic, m_bin, ctx_kw=None, entropy_from_u=True, setup_all=False):
    """build -> sort -> mark -> density -> force on the GPU.  Returns the
    context, particles (cell order), perm and a snapshot of the derived
    structures taken right after mark_active.  setup_all first runs an
    all-active density pass, which gives the inactive particles of a deep
    bin their density-loop state (h, rho, f, P, c, B)."""
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context(**(ctx_kw or {}))
    perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    ctx.sort_cells()
    snap = {}
    keys, o = ctx.copy_particles()
    snap["keys"] = keys.cpu().numpy().view(np.uint64)
    snap["o"] = [t.cpu().numpy() for t in o]
    snap["leaves"] = {k: v.cpu().numpy() for k, v in ctx.copy_leaves().items()}
    snap["order"] = ctx.copy_axis_order().cpu().numpy().view(np.uint16)
    snap["info_build"] = ctx.info()
    snap["pair_slack"] = ctx.params.pair_slack
    snap["H_mark"] = None
    if setup_all:
        ctx.mark_active(p, ctx.params.n_bins - 1)
        ctx.density_pass(p, entropy_from_u=entropy_from_u)
        entropy_from_u = False
        snap["H_mark"] = (np.float32(1.825742) * p["h"].cpu().numpy()).astype(np.float32)
    ctx.mark_active(p, m_bin)
    act, al, hm = ctx.copy_active()
    snap["active"] = act.cpu().numpy().astype(bool)
    snap["active_leaves"] = al.cpu().numpy()
    snap["hmax_act"] = hm.cpu().numpy()
    a, b, s = ctx.copy_pairs(0)
    snap["dpairs"] = (a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy())
    ctx.density_pass(p, entropy_from_u=entropy_from_u)
    ctx.force_pass(p)
    a, b, s = ctx.copy_pairs(1)
    snap["fpairs"] = (a.cpu().numpy(), b.cpu().numpy(), s.cpu().numpy())
    snap["info"] = ctx.info()
    ctx.sync()
    return ctx, p, perm.cpu().numpy(), snap


def host(p, k):
    return p[k].detach().cpu().numpy()


def with_slack(act, slack):
    """The active set with the reach of the density cell-pair lists: each
    active leaf's max H times the slack, rounded to FP32 as on the device."""
    out = dict(act)
    out["hmax_act"] = (np.asarray(act["hmax_act"], np.float32) * np.float32(slack)).astype(np.float32)
    return out


def pair_set(a, b, s):
    return sorted(zip(a.tolist(), b.tolist(), [tuple(x) for x in s.astype(np.float32).tolist()]))


def check_structures(ic, perm, snap, split=400, m_bin=0, D=16):
    """Bit-exact: permutation, keys, offsets, leaves, axis orders, active
    set and density cell pairs against the C definitions."""
    cl = emu.build_cells(ic["x"], ic["h"], split=split, D=D)
    assert np.array_equal(perm, cl["perm"])
    assert np.array_equal(snap["keys"], cl["key"])
    for d, k in enumerate(("ox", "oy", "oz")):
        assert np.array_equal(snap["o"][d].view(np.uint32), cl[k].view(np.uint32)), k
    lv = snap["leaves"]
    assert snap["info_build"]["n_leaves"] == cl["n_leaves"]
    assert snap["info_build"]["top_level"] == cl["top_level"]
    assert np.array_equal(lv["level"], cl["leaf_level"])
    assert np.array_equal(lv["ix"], cl["leaf_ix"]) and np.array_equal(lv["iy"], cl["leaf_iy"])
    assert np.array_equal(lv["iz"], cl["leaf_iz"])
    assert np.array_equal(lv["begin"], cl["leaf_begin"]) and np.array_equal(lv["count"], cl["leaf_count"])
    assert np.array_equal(lv["hmax"].view(np.uint32), cl["leaf_hmax"].view(np.uint32))
    order, _ = emu.axis_sort(cl)
    assert np.array_equal(snap["order"], order)
    binsorted = ic["bin"][perm]
    act = emu.mark_active(cl, binsorted, m_bin, H=snap.get("H_mark"))
    assert np.array_equal(snap["active"], act["active"])
    assert np.array_equal(snap["active_leaves"], act["active_leaves"])
    assert np.array_equal(snap["hmax_act"].view(np.uint32), act["hmax_act"].view(np.uint32))
    ea, eb, es = emu.pairs(cl, with_slack(act, snap["pair_slack"]), "density")
    assert pair_set(*snap["dpairs"]) == pair_set(ea, eb, es)
    return cl, act


def check_counts(cl, p, snap, perm, ic, m_bin, samples=None):
    """Neighbour counts bit-exact against the all-pairs FP32 definition at
    the GPU's final h; force cell pairs against the definition with that h."""
    h = host(p, "h")
    H = (np.float32(1.825742) * h).astype(np.float32)
    active = snap["active"]
    idx = np.nonzero(active)[0] if samples is None else samples
    cd = emu.counts(cl, "density", idx, H=H)
    cf = emu.counts(cl, "force", idx, H=H)
    assert np.array_equal(host(p, "nngb_density")[idx], cd)
    assert np.array_equal(host(p, "nngb_force")[idx], cf)
    binsorted = ic["bin"][perm]
    act = emu.mark_active(cl, binsorted, m_bin, H=H)
    lh = emu.leaf_hmax(cl, H)
    ea, eb, es = emu.pairs(cl, act, "force", leaf_hmax_arr=lh)
    assert pair_set(*snap["fpairs"]) == pair_set(ea, eb, es)
    return cd, cf


def oracle_all(ic, entropy_from_u=True):
    out = sph.density_and_ghost(ic["x"], ic["v"], ic["m"], ic["h"], 1.0, u=ic["u"])
    fo = sph.force(ic["x"], ic["v"], ic["m"], out["h"], out["rho"], out["f"], out["P"], out["c"], out["B"], 1.0)
    return out, fo


def float_errors(p, perm, out, fo, idx_sorted=None, fo_aligned=False):
    """Per-quantity errors of the GPU (cell order) against the oracle
    (original order), over the active particles `idx_sorted`.  The force
    arrays are in original order, or aligned with idx_sorted (fo_aligned)."""
    if idx_sorted is None:
        idx_sorted = np.arange(p.n)
    orig = perm[idx_sorted]

    def rel(g, r):
        g = g.astype(np.float64)
        return np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-300))

    e = {}
    e["h"] = rel(host(p, "h")[idx_sorted], out["h"].numpy()[orig])
    e["rho"] = rel(host(p, "rho")[idx_sorted], out["rho"].numpy()[orig])
    e["drho_dh"] = rel(host(p, "drho_dh")[idx_sorted], out["drho_dh"].numpy()[orig])
    e["f"] = rel(host(p, "f_gradh")[idx_sorted], out["f"].numpy()[orig])
    e["P"] = rel(host(p, "P")[idx_sorted], out["P"].numpy()[orig])
    e["c"] = rel(host(p, "c")[idx_sorted], out["c"].numpy()[orig])
    dv_scale = np.maximum(np.abs(out["divv"].numpy()[orig]),
                          1e-2 * np.max(np.abs(out["divv"].numpy()[orig])) + 1e-300)
    e["divv"] = np.max(np.abs(host(p, "divv")[idx_sorted] - out["divv"].numpy()[orig]) / dv_scale)
    curl_g = np.stack([host(p, k)[idx_sorted] for k in ("curlx", "curly", "curlz")], 1).astype(np.float64)
    curl_r = out["curlv"].numpy()[orig]
    cs = np.maximum(np.linalg.norm(curl_r, axis=1), 1e-2 * np.max(np.linalg.norm(curl_r, axis=1)) + 1e-300)
    e["curlv"] = np.max(np.linalg.norm(curl_g - curl_r, axis=1) / cs)
    e["B"] = np.max(np.abs(host(p, "balsara")[idx_sorted] - out["B"].numpy()[orig]))
    a_g = np.stack([host(p, k)[idx_sorted] for k in ("ax", "ay", "az")], 1).astype(np.float64)
    a_r = fo["a"].numpy() if fo_aligned else fo["a"].numpy()[orig]
    S = fo["scale"].numpy() if fo_aligned else fo["scale"].numpy()[orig]
    den = np.maximum(np.linalg.norm(a_r, axis=1), 1e-2 * S)
    e["a"] = np.max(np.linalg.norm(a_g - a_r, axis=1) / den)
    e["a_normwise"] = np.linalg.norm(a_g - a_r) / max(np.linalg.norm(a_r), 1e-300)
    vs_r = fo["vsig"].numpy() if fo_aligned else fo["vsig"].numpy()[orig]
    e["vsig"] = rel(host(p, "vsig")[idx_sorted], vs_r)
    dA_r = fo["dA_dt"].numpy() if fo_aligned else fo["dA_dt"].numpy()[orig]
    e["dA_dt"] = np.max(np.abs(host(p, "dA_dt")[idx_sorted] - dA_r)) / max(np.max(np.abs(dA_r)), 1e-300)
    return e
