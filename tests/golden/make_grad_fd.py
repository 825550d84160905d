"""Writes grad_fd_differentiation.txt: FP64 central finite differences of
L = sum_i w_i . a_i for the 32,768-particle differentiation workload, with
respect to the positions (step 1e-6 of the mean spacing 1/32) and internal
energies (relative step 1e-6) of 64 seeded particles.  Calls only oracle/.

Usage: python tests/golden/make_grad_fd.py [processes]
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ics  # noqa: E402
from oracle import grad  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_fd_differentiation.txt")
N_PART = 64
SEED = 1807_01341 + 4


def particles(n_total):
    return np.sort(np.random.default_rng(SEED).choice(n_total, size=N_PART, replace=False))


def one(i):
    import torch
    torch.set_num_threads(1)
    c = ics.differentiation()
    step = 1e-6 / 32.0
    gx, gu = grad.finite_difference(c["x"], c["v"], c["m"], c["u"], c["h"], 1.0, c["w"], [i], step)
    return i, gx[0], gu[0]


if __name__ == "__main__":
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    c = ics.differentiation()
    idx = particles(c["x"].shape[0])
    with Pool(procs) as pool:
        rows = pool.map(one, idx.tolist())
    with open(OUT, "w") as f:
        f.write("# FP64 central differences of L = sum w.a (differentiation workload, 32768 particles)\n")
        f.write("# x step 1e-6/32 absolute, u step 1e-6 relative; columns: index dL/dx dL/dy dL/dz dL/du\n")
        for i, gx, gu in rows:
            f.write(f"{i} {gx[0]:.17g} {gx[1]:.17g} {gx[2]:.17g} {gu:.17g}\n")
    print("wrote", OUT)
