"""The entry point for callers that cannot allocate device memory,
sph_step_noalloc, through the C-ABI: its results equal those of sph_step on
a fresh context with the same parameters, bit for bit, on two calls in a
row (the second with fewer particles, so that it runs on the static scratch
array the first call left behind), and sizes beyond its limit are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import ics
from tests.gpu_cases import host

pytestmark = pytest.mark.gpu

OUTPUTS = ("x", "y", "z", "vx", "vfx", "A", "Af", "h", "time_bin", "rho", "drho_dh", "f_gradh", "divv", "curlx",
           "P", "c", "balsara", "ax", "ay", "az", "dA_dt", "du_dt", "vsig", "nngb_density", "nngb_force")


def _noalloc_fn(sg):
    return sg.lib().sph_step_noalloc


def _step_args(ic):
    # the first step of a run: every particle active, the first kick at t = 0
    return ics.N_BINS - 1, 0, ic["t_min_model"], 1


def test_noalloc_step_equals_step(gpu_lib):
    sg = gpu_lib
    f = _noalloc_fn(sg)
    for case, ic in (("clustered 60000", ics.clustered(n_total=60000, n_clumps=3)),
                     ("clustered 20000", ics.clustered(n_total=20000, n_clumps=3))):
        print(f"case step_noalloc {case}", flush=True)
        m, ti, t_min, drift = _step_args(ic)
        # the existing entry point on a fresh context
        ref = sg.Particles.from_initial(ic)
        ctx = sg.Context()
        perm_ref = torch.empty(ref.n, dtype=torch.int64, device="cuda")
        na_ref = ctx.step(ref, m, ti, t_min, drift, True, entropy_from_u=True, perm_out=perm_ref, want_count=True)
        ctx.sync()
        # the entry point that allocates nothing
        got = sg.Particles.from_initial(ic)
        prm = sg.default_params()
        perm = torch.empty(got.n, dtype=torch.int64, device="cuda")
        na = C.c_int64(-1)
        used = C.c_int64(-1)
        err = C.create_string_buffer(512)
        pc = got.c_struct()
        rc = f(C.byref(prm), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(pc), got.n,
               C.c_void_p(perm.data_ptr()), m, C.byref(na), 1, ti, t_min, drift, 1, C.byref(used), err, 512)
        torch.cuda.synchronize()
        assert rc == 0, err.value.decode()
        print(f"{case}: active {na.value}, static scratch used {used.value / 2**20:.1f} MiB", flush=True)
        assert na.value == na_ref > 0
        assert np.array_equal(perm.cpu().numpy(), perm_ref.cpu().numpy())
        for k in OUTPUTS:
            assert np.array_equal(host(got, k).view(np.uint8), host(ref, k).view(np.uint8)), (case, k)
        ctx.close()


def test_noalloc_refuses_sizes_beyond_its_limit(gpu_lib):
    sg = gpu_lib
    f = _noalloc_fn(sg)
    ic = ics.tiny_lattice(8)
    got = sg.Particles.from_initial(ic)
    prm = sg.default_params()
    err = C.create_string_buffer(512)
    pc = got.c_struct()
    # n beyond the limit is refused before any device work
    rc = f(C.byref(prm), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(pc), (1 << 18) + 1, None, 0,
           None, 1, 0, 1e-3, 1, 1, None, err, 512)
    assert rc == -1 and b"static scratch" in err.value
    rc = f(C.byref(prm), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(pc), 0, None, 0, None, 1, 0,
           1e-3, 1, 1, None, err, 512)
    assert rc == -1
