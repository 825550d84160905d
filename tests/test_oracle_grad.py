"""Pins of the oracle's reference gradient (reverse mode through the FP64
density, implicit smoothing length, ghost and force) against FP64 central
finite differences of the loss, which only use the forward oracle."""
import os

import numpy as np
import pytest

import ics
from oracle import grad

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_fd_differentiation.txt")


PARTS = [3, 100, 257, 511]


@pytest.fixture(scope="module")
def small():
    """8^3 moving lattice with log-uniform u: reverse-mode gradient and
    central differences (step 1e-6 of the spacing) at four particles."""
    ic = ics.tiny_lattice(8, velocity_sigma=0.3)
    rng = np.random.default_rng(1807_01341 + 40)
    ic["u"] = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=ic["x"].shape[0]))
    w = rng.normal(size=ic["x"].shape)
    gx, gu = grad.gradient(ic["x"], ic["v"], ic["m"], ic["u"], ic["h"], 1.0, w)
    fx, fu = grad.finite_difference(ic["x"], ic["v"], ic["m"], ic["u"], ic["h"], 1.0, w, PARTS, 1e-6 / 8)
    return ic, w, gx, gu, fx, fu


def test_gradient_matches_finite_differences_small(small):
    ic, w, gx, gu, fx, fu = small
    ex = np.max(np.abs(gx[PARTS] - fx)) / np.max(np.abs(gx))
    eu = np.max(np.abs(gu[PARTS] - fu)) / np.max(np.abs(gu))
    print(f"x {ex:.1e} u {eu:.1e}")
    assert ex < 1e-6 and eu < 1e-6


def test_gradient_without_the_implicit_h_term_fails_the_check(small):
    """A planted mistake: the same reverse mode with h held at its converged
    value (no dh/dx) misses the finite differences by far more than the
    tolerance, so the check above sees the implicit term."""
    import torch
    ic, w, gx, gu, fx, fu = small
    xt = torch.tensor(ic["x"], dtype=torch.float64, requires_grad=True)
    per, _, _ = grad.loss(xt, ic["v"], ic["m"], ic["u"], ic["h"], 1.0, w, differentiable=False)
    per.sum().backward()
    g_wrong = xt.grad.numpy()
    err = np.max(np.abs(g_wrong[PARTS] - fx)) / np.max(np.abs(gx))
    print(f"without dh/dx: {err:.1e}")
    assert err > 1e-3


def test_gradient_matches_stored_finite_differences():
    """Differentiation workload (32,768 particles): the reverse-mode gradient
    at the 64 particles of the stored FP64 central differences."""
    rows = np.loadtxt(GOLDEN)
    idx = rows[:, 0].astype(np.int64)
    assert len(idx) == 64
    ic = ics.differentiation()
    gx, gu = grad.gradient(ic["x"], ic["v"], ic["m"], ic["u"], ic["h"], 1.0, ic["w"])
    fx, fu = rows[:, 1:4], rows[:, 4]
    assert np.linalg.norm(gx[idx] - fx) < 1e-6 * np.linalg.norm(fx)
    assert np.linalg.norm(gu[idx] - fu) < 1e-6 * np.linalg.norm(fu)
