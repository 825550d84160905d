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


# ---------------------------------------------------------------- one step of a running simulation

STATE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "A", "h", "time_bin", "rho", "f_gradh", "P", "c", "balsara",
              "divv", "ax", "ay", "az", "dA_dt", "vsig", "nngb_density", "nngb_force")


def step_state(p):
    """Host copy (cell order) of the particle state after a step's force
    pass: the step's inputs (positions, predicted velocities and entropies,
    bins, and the density-loop state inactive particles keep) and outputs."""
    return {k: host(p, k).copy() for k in STATE_KEYS}


class CellTracker:
    """The C definitions' cells for a running GPU context: a full build is
    emulated from the positions the GPU built from (recovered from its
    permutation), a kept build by the update definitions at the positions
    the step's loops read."""

    def __init__(self, D=16, split=400):
        self.D, self.split = D, split
        self.cl_build = None

    def after_build(self, ctx, p, perm_dev, full_before):
        """Call right after ctx.build_cells(p, perm_dev); full_before is
        ctx.info()['full_builds'] before that call.  Returns True if it was a
        full build."""
        inf = ctx.info()
        if inf["full_builds"] == full_before:
            return False
        perm = perm_dev.cpu().numpy()
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        x_in = np.stack([host(p, k) for k in "xyz"], 1)[inv]
        h_in = host(p, "h")[inv]
        cl = emu.build_cells(x_in, h_in, split=self.split, D=self.D)
        assert np.array_equal(perm, cl["perm"]), "full build: permutation differs from the C definitions"
        self.cl_build = cl
        return True

    def now(self, st):
        """The cells at the positions of state st (cell order)."""
        xs = np.stack([st["x"], st["y"], st["z"]], 1)
        xb = np.stack([self.cl_build["xw"], self.cl_build["yw"], self.cl_build["zw"]], 1)
        up, _ = emu.update(self.cl_build, xs, st["h"], xb)
        return up


def reach_set(x, H, samples, L=1.0):
    """Indices j (any order) with r_ij < 1.01 max(H_i, H_j) for some sample
    i (minimum image, FP64): every force neighbour of the samples."""
    from scipy.spatial import cKDTree
    tree = cKDTree(x, boxsize=L)
    Hmax = float(H.max())
    out = [np.asarray(samples)]
    for i in samples:
        c = np.asarray(tree.query_ball_point(x[i], 1.01 * max(float(H[i]), Hmax)), np.int64)
        d = x[c] - x[i]
        d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(1))
        out.append(c[r < 1.01 * np.maximum(H[i], H[c])])
    return np.unique(np.concatenate(out))


def local_subset(cl, x, H, samples, L=1.0):
    """Sorted indices of every particle within 2.6 max(H) of a sample
    (minimum image): a superset of the samples' force neighbours and of
    those neighbours' density neighbours at up to 1.5 times their H, so that
    the oracle's sums over the subset equal its sums over all particles.
    Leaves (bounding boxes of their particles' positions) are tested first."""
    R = 2.6 * float(H.max()) + 1e-9
    b = np.asarray(cl["leaf_begin"], np.int64)
    c = np.asarray(cl["leaf_count"], np.int64)
    lo = np.stack([np.minimum.reduceat(x[:, a], b) for a in range(3)], 1)
    hi = np.stack([np.maximum.reduceat(x[:, a], b) for a in range(3)], 1)
    keep = np.zeros(b.size, bool)
    for i in samples:
        d2 = np.zeros(b.size)
        for a in range(3):
            best = None
            for sh in (-L, 0.0, L):
                p = x[i, a] + sh
                g = np.maximum(np.maximum(lo[:, a] - p, p - hi[:, a]), 0.0)
                best = g if best is None else np.minimum(best, g)
            d2 += best * best
        keep |= d2 < R * R
    idx = [np.arange(bb, bb + cc) for bb, cc in zip(b[keep], c[keep])]
    return np.concatenate(idx) if idx else np.asarray(samples)


def check_step_vs_oracle(st, active, m_bin, samples, cl_now, count_samples=None, entropy_from_u=False,
                         u=None, label=""):
    """One step of the path against the oracle at the step's own inputs.

    st: step_state after the force pass; active: the GPU's active flags
    (cell order).  Checks: the active set is {bin <= m}; neighbour counts of
    every active particle (or count_samples) bit-exact against the FP32
    definitions at the GPU's final h; for `samples`, h, rho, f, P, c within
    1e-5 and a within A_TOL of the FP64 oracle, which solves the density
    loop for every active particle within force reach of a sample and takes
    the stored state of inactive neighbours (their last active step's h,
    rho, f, P, c, B) as the step does.  Returns the error dict."""
    assert np.array_equal(active, st["time_bin"] <= m_bin), f"{label}: active set"
    H = (np.float32(1.825742) * st["h"]).astype(np.float32)
    idx = np.nonzero(active)[0] if count_samples is None else np.asarray(count_samples)
    cd = emu.counts_grid(cl_now, "density", idx, H=H)
    cf = emu.counts_grid(cl_now, "force", idx, H=H)
    nd, nf = st["nngb_density"][idx], st["nngb_force"][idx]
    assert np.array_equal(nd, cd), f"{label}: density counts differ at {int((nd != cd).sum())} of {idx.size}"
    assert np.array_equal(nf, cf), f"{label}: force counts differ at {int((nf != cf).sum())} of {idx.size}"
    samples = np.asarray(samples, np.int64)
    x_all = np.stack([st["x"], st["y"], st["z"]], 1)
    # the oracle runs on a local subset that holds every particle its sums reach
    sub = local_subset(cl_now, x_all, H.astype(np.float64), samples)
    loc = np.searchsorted(sub, samples)
    assert np.array_equal(sub[loc], samples)
    x = x_all[sub]
    v = np.stack([st["vx"], st["vy"], st["vz"]], 1)[sub]
    ms = st["m"][sub]
    act_s = active[sub]
    J = reach_set(x, H[sub].astype(np.float64), loc)
    Ja = J[act_s[J]]
    out = sph.solve_density(x, v, ms, st["h"][sub], 1.0, centres=Ja)
    th = u[sub][Ja].astype(np.float64) if entropy_from_u else None
    tA = None if entropy_from_u else torch.as_tensor(st["A"][sub][Ja].astype(np.float64))
    gh = sph.ghost(out["h"], out["rho"], out["drho_dh"], out["div_raw"], out["curl_raw"],
                   u=None if th is None else torch.as_tensor(th), A=tA)
    full = {}
    for k, gk in (("h", "h"), ("rho", "rho"), ("f", "f_gradh"), ("P", "P"), ("c", "c"), ("B", "balsara")):
        a = torch.as_tensor(st[gk][sub].astype(np.float64))
        a[torch.as_tensor(Ja)] = out[k] if k in out else gh[k]
        full[k] = a
    fo = sph.force(x, v, ms, full["h"], full["rho"], full["f"], full["P"], full["c"], full["B"], 1.0,
                   centres=loc)
    pos = np.searchsorted(Ja, loc)

    def rel(g, r):
        return float(np.max(np.abs(g.astype(np.float64) - r) / np.abs(r)))

    e = {"h": rel(st["h"][samples], out["h"].numpy()[pos]),
         "rho": rel(st["rho"][samples], out["rho"].numpy()[pos]),
         "f": rel(st["f_gradh"][samples], gh["f"].numpy()[pos]),
         "P": rel(st["P"][samples], gh["P"].numpy()[pos]),
         "c": rel(st["c"][samples], gh["c"].numpy()[pos]),
         "vsig": rel(st["vsig"][samples], fo["vsig"].numpy())}
    a_g = np.stack([st[k][samples] for k in ("ax", "ay", "az")], 1).astype(np.float64)
    a_r = fo["a"].numpy()
    den = np.maximum(np.linalg.norm(a_r, axis=1), 1e-2 * fo["scale"].numpy())
    e["a"] = float(np.max(np.linalg.norm(a_g - a_r, axis=1) / den))
    e["a_normwise"] = float(np.linalg.norm(a_g - a_r) / np.linalg.norm(a_r))
    dA_r = fo["dA_dt"].numpy()
    e["dA_dt"] = float(np.max(np.abs(st["dA_dt"][samples] - dA_r)) / max(np.max(np.abs(dA_r)), 1e-300))
    print(f"{label}: {idx.size} counts exact; oracle on {len(samples)} samples ({Ja.size} density solves, "
          f"subset {sub.size}): "
          + " ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    assert e["rho"] < RHO_TOL and e["h"] < 1e-5, label
    assert e["f"] < 1e-5 and e["P"] < 1e-5 and e["c"] < 1e-5 and e["vsig"] < 1e-5, label
    assert e["a"] < A_TOL, label
    return e


def spread_sample(active, h, k, rng, centres=None, x=None, per_centre=0):
    """k active particles spread over the density range (even ranks of h),
    plus `per_centre` nearest active particles to each of `centres`."""
    act = np.nonzero(active)[0]
    order = act[np.argsort(h[act], kind="stable")]
    pick = [order[np.linspace(0, order.size - 1, min(k, order.size)).astype(np.int64)]]
    if centres is not None and per_centre > 0:
        from scipy.spatial import cKDTree
        t = cKDTree(x[act], boxsize=1.0)
        for c in centres:
            _, nn = t.query(c, k=min(per_centre, act.size))
            pick.append(act[np.atleast_1d(nn)])
    return np.unique(np.concatenate(pick))
