"""Reference gradient of the loss L = sum_i w_i . a_i with respect to the
positions and internal energies (test infrastructure only).

Reverse mode through the FP64 oracle with torch autograd: the density sums,
the smoothing-length root (one differentiable Newton step from the converged
root gives the implicit derivative), the ghost quantities and the force loop,
all active.  A central finite-difference driver checks it from outside.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import sph

F64 = torch.float64


def loss(x, v, m, u, h0, L, w, p: sph.Params = sph.Params(), differentiable=True):
    x = torch.as_tensor(x, dtype=F64)
    u = torch.as_tensor(u, dtype=F64)
    out = sph.density_and_ghost(x, v, m, h0, L, u=u, p=p, differentiable=differentiable)
    fo = sph.force(x, v, m, out["h"], out["rho"], out["f"], out["P"], out["c"], out["B"], L, p=p)
    return (torch.as_tensor(w, dtype=F64) * fo["a"]).sum(1), out, fo


def gradient(x, v, m, u, h0, L, w, p: sph.Params = sph.Params()):
    """dL/dx (N,3) and dL/du (N,) by reverse mode."""
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    ut = torch.tensor(np.asarray(u, np.float64), requires_grad=True)
    per, _, _ = loss(xt, v, m, ut, h0, L, w, p)
    per.sum().backward()
    return xt.grad.numpy(), ut.grad.numpy()


def loss_value(x, v, m, u, h0, L, w, p: sph.Params = sph.Params()):
    """L summed exactly (math.fsum) for finite differences."""
    with torch.no_grad():
        per, _, _ = loss(x, v, m, u, h0, L, w, p, differentiable=False)
    return math.fsum(per.numpy().tolist())


def finite_difference(x, v, m, u, h0, L, w, particles, step, p: sph.Params = sph.Params()):
    """Central differences of L for the listed particles: (k,3) for x and (k,)
    for u.  The x step is absolute; the u step is step/spacing relative."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    gx = np.zeros((len(particles), 3))
    gu = np.zeros(len(particles))
    for t, i in enumerate(particles):
        for a in range(3):
            xp = x.copy(); xp[i, a] += step
            xm = x.copy(); xm[i, a] -= step
            gx[t, a] = (loss_value(xp, v, m, u, h0, L, w, p) - loss_value(xm, v, m, u, h0, L, w, p)) / (2 * step)
        du = 1e-6 * u[i]
        up = u.copy(); up[i] += du
        um = u.copy(); um[i] -= du
        gu[t] = (loss_value(x, v, m, up, h0, L, w, p) - loss_value(x, v, m, um, h0, L, w, p)) / (2 * du)
    return gx, gu
