"""The precision scheme: the same all-active step on the clustered 20k box
with compensated and with plain FP32 accumulation of the per-particle sums,
in both loop forms (the chunk loop of dense active sets, and the
per-particle sweep that the default threshold picks for a pass of fewer than
2^18 particles), each quantity's error against the FP64 oracle reported for
every combination."""
import numpy as np
import pytest

import ics
from tests.gpu_cases import A_TOL, RHO_TOL, float_errors, oracle_all, run_gpu_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clustered20k_with_oracle():
    ic = ics.clustered(n_total=20000, n_clumps=3)
    return ic, oracle_all(ic)


@pytest.mark.parametrize("loop", ["chunk", "sweep"])
@pytest.mark.parametrize("compensated", [1, 0])
def test_errors_with_and_without_compensation(gpu_lib, clustered20k_with_oracle, compensated, loop):
    ic, (out, fo) = clustered20k_with_oracle
    kw = dict(compensated=compensated)
    if loop == "chunk":
        kw["sweep_below"] = 0
    else:
        # the default threshold: 20,000 active particles take the sweep kernels
        assert gpu_lib.default_params().sweep_below > ic["x"].shape[0]
    print(f"case clustered20k all active, {loop} loop, compensated={compensated}", flush=True)
    ctx, p, perm, snap = run_gpu_step(gpu_lib, ic, ics.N_BINS - 1, ctx_kw=kw)
    e = float_errors(p, perm, out, fo)
    print(f"{loop} loop,", "compensated" if compensated else "plain FP32",
          {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    assert e["rho"] < RHO_TOL and e["h"] < 1e-5 and e["a"] < A_TOL
