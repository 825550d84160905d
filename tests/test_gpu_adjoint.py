"""GPU parity of the adjoint (reverse mode of density + force, with the
implicit smoothing-length derivative) against the FP64 oracle's autograd
gradient and against stored FP64 central finite differences."""
import os

import numpy as np
import pytest
import torch

import ics
from oracle import grad as ograd

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_fd_differentiation.txt")
G_TOL = 1e-5      # normwise relative error of dL/dx and dL/du over all particles
G_TOL_PP = 5e-4   # per particle, relative to max(|g_i|, 0.1 * rms |g|)


def gpu_gradient(sg, ic, w):
    """(dL/dx (N,3), dL/du (N,)) in original order through SPHForce."""
    dev = torch.device("cuda")
    x = torch.tensor(ic["x"], dtype=torch.float64, device=dev, requires_grad=True)
    u = torch.tensor(ic["u"], dtype=torch.float32, device=dev, requires_grad=True)
    v = torch.tensor(ic["v"], dtype=torch.float64, device=dev)
    m = torch.tensor(ic["m"], dtype=torch.float32, device=dev)
    h = torch.tensor(ic["h"], dtype=torch.float32, device=dev)
    a = sg.SPHForce.apply(x, u, v, m, h)
    wt = torch.tensor(w, dtype=torch.float32, device=dev)
    (a * wt).sum().backward()
    torch.cuda.synchronize()
    return x.grad.cpu().numpy(), u.grad.cpu().numpy().astype(np.float64), a.detach().cpu().numpy()


def errors(g, r):
    nw = np.linalg.norm(g - r) / np.linalg.norm(r)
    if r.ndim == 1:
        den = np.maximum(np.abs(r), 0.1 * np.sqrt(np.mean(r * r)))
        pp = np.max(np.abs(g - r) / den)
    else:
        nr = np.linalg.norm(r, axis=1)
        den = np.maximum(nr, 0.1 * np.sqrt(np.mean(nr * nr)))
        pp = np.max(np.linalg.norm(g - r, axis=1) / den)
    return nw, pp


def check_against_oracle(sg, ic, w):
    gx, gu, _ = gpu_gradient(sg, ic, w)
    rx, ru = ograd.gradient(ic["x"], ic["v"], ic["m"], ic["u"], ic["h"], 1.0, w)
    ex, exp = errors(gx, rx)
    eu, eup = errors(gu, ru)
    print(f"dL/dx normwise {ex:.2e} per-particle {exp:.2e}; dL/du normwise {eu:.2e} per-particle {eup:.2e}",
          flush=True)
    assert ex < G_TOL and eu < G_TOL
    assert exp < G_TOL_PP and eup < G_TOL_PP
    return gx, gu


def test_adjoint_tiny_moving_lattice(gpu_lib):
    ic = ics.tiny_lattice(16, velocity_sigma=0.3)
    rng = np.random.default_rng(1807_01341 + 41)
    ic["u"] = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=ic["x"].shape[0])).astype(np.float32)
    w = rng.normal(size=ic["x"].shape)
    print("case adjoint tiny16 sigma=0.3", flush=True)
    check_against_oracle(gpu_lib, ic, w)


def test_adjoint_differentiation_workload(gpu_lib):
    ic = ics.differentiation()
    print("case adjoint differentiation 32768", flush=True)
    gx, gu = check_against_oracle(gpu_lib, ic, ic["w"])
    rows = np.loadtxt(GOLDEN)
    idx = rows[:, 0].astype(np.int64)
    fx, fu = rows[:, 1:4], rows[:, 4]
    ex = np.linalg.norm(gx[idx] - fx) / np.linalg.norm(fx)
    eu = np.linalg.norm(gu[idx] - fu) / np.linalg.norm(fu)
    print(f"vs finite differences on {len(idx)} particles: x {ex:.2e} u {eu:.2e}", flush=True)
    assert ex < G_TOL and eu < G_TOL


def test_adjoint_matches_context_call_and_is_repeatable(gpu_lib):
    """SPHForce's backward and a direct sph_adjoint call on the same state
    agree bit for bit, and two calls give the same bits."""
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.2)
    w = np.random.default_rng(5).normal(size=ic["x"].shape)
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(p, perm)
    ctx.sort_cells()
    ctx.mark_active(p, ctx.params.n_bins - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    ws = torch.tensor(w, dtype=torch.float32, device="cuda")[perm]
    g1, u1 = ctx.adjoint(p, ws)
    g2, u2 = ctx.adjoint(p, ws)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(u1, u2)
    gx, gu, _ = gpu_gradient(sg, ic, w)
    pn = perm.cpu().numpy()
    assert np.array_equal(gx[pn], g1.cpu().numpy())
    assert np.array_equal(gu[pn].astype(np.float32), u1.cpu().numpy())


def test_adjoint_preconditions(gpu_lib):
    sg = gpu_lib
    ic = ics.tiny_lattice(16, velocity_sigma=0.1)
    rng = np.random.default_rng(3)
    ic["bin"] = rng.integers(0, 3, size=ic["x"].shape[0]).astype(np.int8)
    w = torch.zeros(ic["x"].shape[0], 3, dtype=torch.float32, device="cuda")
    p = sg.Particles.from_initial(ic)
    ctx = sg.Context()
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, 2)
    ctx.density_pass(p, True)
    with pytest.raises(sg.SPHError) as e:
        ctx.adjoint(p, w)          # before the force pass
    assert e.value.code == -6
    ctx.force_pass(p)
    ctx.mark_active(p, 1)          # not every particle active
    ctx.density_pass(p, False)
    ctx.force_pass(p)
    with pytest.raises(sg.SPHError) as e:
        ctx.adjoint(p, w)
    assert e.value.code == -1
    ctx.mark_active(p, 2)          # all active, but pressure from A
    ctx.density_pass(p, False)
    ctx.force_pass(p)
    with pytest.raises(sg.SPHError) as e:
        ctx.adjoint(p, w)
    assert e.value.code == -6
