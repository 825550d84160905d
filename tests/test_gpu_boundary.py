"""The boundary's memory and batch contract, through the C-ABI:

* every device buffer of a context comes from the allocator callbacks given
  to sph_create (a counting allocator over PyTorch's caching allocator sees
  all of it, outgrown buffers are returned through it, nothing is left after
  sph_destroy), with results bitwise equal to a context on hipMalloc;
* a batch of boxes in one context (sph_batch_create, sph_batch_mark_active,
  sph_batch_density_force) gives each box bitwise the results of the same
  boxes as separate contexts in a multi-context batched pass."""
import ctypes as C

import numpy as np
import pytest
import torch

import ics
from tests.gpu_cases import host

pytestmark = pytest.mark.gpu

OUTPUTS = ("x", "h", "rho", "drho_dh", "f_gradh", "divv", "curlx", "P", "c", "balsara", "A", "ax", "ay", "az",
           "dA_dt", "du_dt", "vsig", "nngb_density", "nngb_force")


class CountingAllocator:
    """Delegates to PyTorch's caching allocator and books every block."""

    def __init__(self, sg):
        self.live = {}
        self.n_alloc = 0
        self.n_free = 0
        self.unknown_frees = 0
        self.fns = (sg.ALLOC_FN(self._alloc), sg.FREE_FN(self._free))

    def _alloc(self, nbytes, stream, user):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        self.live[int(p)] = int(nbytes)
        self.n_alloc += 1
        return p

    def _free(self, ptr, stream, user):
        if self.live.pop(int(ptr), None) is None:
            self.unknown_frees += 1
        self.n_free += 1
        torch.cuda.caching_allocator_delete(int(ptr))

    @property
    def live_bytes(self):
        return sum(self.live.values())


def _run_two_steps(sg, ctx, ic):
    p = sg.Particles.from_initial(ic)
    ctx.build_cells(p)
    ctx.sort_cells()
    ctx.mark_active(p, ics.N_BINS - 1)
    ctx.density_pass(p, True)
    ctx.force_pass(p)
    m = ics.deep_bin_for_fraction(ic["bin"], 0.05)
    ctx.step(p, m, 1 << m, ic["t_min_model"], 1 << m, False)
    ctx.step(p, m, 2 << m, ic["t_min_model"], 1 << m, False)
    ctx.sync()
    return p


def test_every_device_buffer_comes_from_the_allocator(gpu_lib):
    sg = gpu_lib
    small = ics.clustered(n_total=20000, n_clumps=3)
    large = ics.clustered(n_total=60000, n_clumps=3)
    print("case counting allocator clustered 20k then 60k", flush=True)
    ca = CountingAllocator(sg)
    ctx = sg.Context(allocator=ca.fns)
    p = _run_two_steps(sg, ctx, small)
    inf = ctx.info()
    assert ca.n_alloc > 0 and inf["device_bytes"] > 0
    assert ca.live_bytes == inf["device_bytes"]
    frees_small = ca.n_free
    # a three times larger input on the same context outgrows its buffers:
    # they go back through the callback, the new ones come from it
    _run_two_steps(sg, ctx, large)
    inf2 = ctx.info()
    assert ca.n_free > frees_small and ca.live_bytes == inf2["device_bytes"] > inf["device_bytes"]
    assert ca.unknown_frees == 0
    # the same work on a context that uses hipMalloc gives the same bits
    ref_ctx = sg.Context(allocator=None)
    ref = _run_two_steps(sg, ref_ctx, small)
    ctx2 = sg.Context(allocator=ca.fns)
    got = _run_two_steps(sg, ctx2, small)
    for k in OUTPUTS:
        assert np.array_equal(host(got, k).view(np.uint8), host(ref, k).view(np.uint8)), k
    ctx.close()
    ctx2.close()
    assert ca.live == {} and ca.unknown_frees == 0
    ref_ctx.close()


def test_one_context_batch_equals_multi_context_batch(gpu_lib):
    sg = gpu_lib
    boxes = ics.batch_of_boxes()
    ms = [ics.deep_bin_for_fraction(b["bin"], b["target_active_fraction"]) for b in boxes]
    sizes = [b["x"].shape[0] for b in boxes]
    print(f"case batch64 one context vs 64 contexts, N={sum(sizes)}", flush=True)
    # 64 contexts, batched passes (the all-active set-up pass batched too)
    cs, ps, perms = [], [], []
    for b, m in zip(boxes, ms):
        p = sg.Particles.from_initial(b)
        c = sg.Context()
        perm = torch.empty(p.n, dtype=torch.int64, device="cuda")
        c.build_cells(p, perm)
        c.sort_cells()
        c.mark_active(p, c.params.n_bins - 1)
        cs.append(c)
        ps.append(p)
        perms.append(perm)
    batch = sg.Batch(cs, ps)
    batch.density_pass(True)
    for c, p, m in zip(cs, ps, ms):
        c.mark_active(p, m)
    batch.density_pass(False)
    batch.force_pass()
    torch.cuda.synchronize()
    ref = [{k: host(p, k).copy() for k in OUTPUTS} for p in ps]
    ref_perm = [q.cpu().numpy() for q in perms]
    n_act_ref = sum(c.info()["n_active"] for c in cs)
    # one context holding the 64 boxes as slices of one set of arrays
    cat = {k: np.concatenate([b[k] for b in boxes]) for k in ("x", "v", "m", "u", "h", "bin")}
    P = sg.Particles.from_initial(cat)
    ctx = sg.Context().batch_create(sizes)
    perm = torch.empty(P.n, dtype=torch.int64, device="cuda")
    ctx.build_cells(P, perm)
    ctx.sort_cells()
    ctx.mark_active(P, ctx.params.n_bins - 1)
    ctx.density_pass(P, True)
    n_act = ctx.batch_mark_active(P, ms)
    ctx.batch_density_force(P, False)
    ctx.sync()
    assert n_act == n_act_ref
    inf = ctx.info()
    assert inf["n_active"] == n_act and inf["n"] == sum(sizes)
    off = np.concatenate([[0], np.cumsum(sizes)])
    pm = perm.cpu().numpy()
    for b in range(len(boxes)):
        sl = slice(off[b], off[b + 1])
        assert np.array_equal(pm[sl], ref_perm[b] + off[b]), b
        for k in OUTPUTS:
            assert np.array_equal(host(P, k)[sl].view(np.uint8), ref[b][k].view(np.uint8)), (b, k)
        kb = ctx.batch_box(b).info()
        assert kb["n"] == sizes[b] and kb["n_active"] == cs[b].info()["n_active"]
    # a batch context refuses the per-box introspection calls and the adjoint
    with pytest.raises(sg.SPHError):
        ctx.copy_leaves()
