"""Python binding of libsphgpu (the C-ABI in include/sphgpu.h).

Argument marshalling only: every step of the SPH path runs in the HIP kernels
of the shared library.  PyTorch supplies device memory and the stream.  The
binding raises if the library has not been built or no GPU is present; there
is no CPU fallback.

Names follow the C functions without their `sph_` prefix.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsphgpu.so")

STATUS = {0: "SPH_OK", -1: "SPH_EINVAL", -2: "SPH_ENOMEM", -3: "SPH_EDEVICE", -4: "SPH_ENOCONV",
          -5: "SPH_EREBUILD", -6: "SPH_ESTATE"}


class SPHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("gamma", C.c_double), ("cfl", C.c_double),
                ("eta", C.c_float), ("alpha", C.c_float), ("balsara_eps", C.c_float), ("h_tol", C.c_float),
                ("n_bins", C.c_int), ("split_count", C.c_int), ("morton_depth", C.c_int), ("top_cap", C.c_int),
                ("h_max_iter", C.c_int), ("compensated", C.c_int), ("cand_cap", C.c_int), ("list_cap", C.c_int),
                ("waves_per_chunk", C.c_int), ("chunk_split", C.c_int), ("sweep_below", C.c_int),
                ("sweep_waves", C.c_int), ("rebuild_frac", C.c_float), ("pair_slack", C.c_float),
                ("lazy_drift", C.c_int)]


# field name, dtype, role
PARTICLE_FIELDS = [
    ("x", torch.float64), ("y", torch.float64), ("z", torch.float64),
    ("vx", torch.float64), ("vy", torch.float64), ("vz", torch.float64),
    ("vfx", torch.float64), ("vfy", torch.float64), ("vfz", torch.float64),
    ("m", torch.float32), ("u", torch.float32), ("A", torch.float32), ("Af", torch.float32),
    ("h", torch.float32), ("time_bin", torch.int8),
    ("rho", torch.float32), ("drho_dh", torch.float32), ("f_gradh", torch.float32), ("divv", torch.float32),
    ("curlx", torch.float32), ("curly", torch.float32), ("curlz", torch.float32), ("P", torch.float32),
    ("c", torch.float32), ("balsara", torch.float32),
    ("ax", torch.float32), ("ay", torch.float32), ("az", torch.float32), ("dA_dt", torch.float32),
    ("du_dt", torch.float32), ("vsig", torch.float32),
    ("nngb_density", torch.int32), ("nngb_force", torch.int32),
]


class ParticlesC(C.Structure):
    _fields_ = [(name, C.c_void_p) for name, _ in PARTICLE_FIELDS]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_leaves", C.c_int64), ("top_level", C.c_int32),
                ("n_active", C.c_int64), ("n_active_leaves", C.c_int64), ("n_density_pairs", C.c_int64),
                ("n_force_pairs", C.c_int64), ("density_iterations", C.c_int32), ("n_unconverged", C.c_int64),
                ("interactions_density", C.c_int64), ("interactions_force", C.c_int64),
                ("unconverged_after_pass", C.c_int32 * 32), ("pair_rebuilds", C.c_int32),
                ("full_builds", C.c_int64), ("cell_updates", C.c_int64), ("dx_max", C.c_float),
                ("device_bytes", C.c_int64)]


_lib = None

# device memory of the contexts: the allocator callbacks of sph_create
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def _torch_alloc(nbytes, stream, user):
    """PyTorch's caching allocator, stream-ordered on the context's stream;
    NULL (the library reports SPH_ENOMEM) when it has no memory."""
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # noqa: BLE001 -- no exception may cross the C boundary
        return None


def _torch_free(ptr, stream, user):
    torch.cuda.caching_allocator_delete(int(ptr))


TORCH_ALLOC = ALLOC_FN(_torch_alloc)
TORCH_FREE = FREE_FN(_torch_free)

_live = weakref.WeakSet()


@atexit.register
def _destroy_live_contexts():
    # destroy contexts while torch (their allocator) is still alive
    for c in list(_live):
        c.close()


def lib():
    """The loaded shared library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsphgpu.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        sigs = {
            "sph_default_params": (None, [vp]),
            "sph_create": (i32, [vp, vp, ALLOC_FN, FREE_FN, vp, vp]),
            "sph_batch_create": (i32, [vp, i32, vp, vp]),
            "sph_batch_mark_active": (i32, [vp, vp, vp, vp]),
            "sph_batch_density_force": (i32, [vp, vp, i32]),
            "sph_batch_box": (vp, [vp, i32]),
            "sph_step_noalloc": (i32, [vp, vp, vp, i64, vp, i32, vp, i32, i64, C.c_double, i64, i32, vp,
                                       C.c_char_p, C.c_size_t]),
            "sph_destroy": (None, [vp]),
            "sph_build_cells": (i32, [vp, vp, i64, vp]),
            "sph_sort_cells": (i32, [vp]),
            "sph_mark_active": (i32, [vp, vp, i32, vp]),
            "sph_density_pass": (i32, [vp, vp, i32]),
            "sph_force_pass": (i32, [vp, vp]),
            "sph_kick_drift": (i32, [vp, vp, i64, C.c_double, i64, i32]),
            "sph_step": (i32, [vp, vp, i64, vp, i32, vp, i32, i64, C.c_double, i64, i32]),
            "sph_drift_all": (i32, [vp, vp]),
            "sph_next_active_time": (i32, [vp, vp, i64, vp]),
            "sph_drift": (i32, [vp, vp, C.c_double, i64]),
            "sph_sync": (i32, [vp]),
            "sph_last_error": (C.c_char_p, [vp]),
            "sph_info": (i32, [vp, vp]),
            "sph_copy_leaves": (i32, [vp] * 9),
            "sph_copy_particles": (i32, [vp] * 5),
            "sph_copy_axis_order": (i32, [vp, vp]),
            "sph_copy_active": (i32, [vp] * 4),
            "sph_copy_pairs": (i32, [vp, i32] + [vp] * 5),
            "sph_profile": (i32, [vp, i32]),
            "sph_profile_read": (i64, [vp, vp, i64]),
            "sph_autotune": (i32, [vp, vp, C.c_char_p]),
            "sph_load_tuning": (i32, [vp, C.c_char_p]),
            "sph_adjoint": (i32, [vp] * 9),
            "sph_batch_density_pass": (i32, [vp, vp, i32, i32]),
            "sph_batch_force_pass": (i32, [vp, vp, i32]),
            "sph_batch_autotune": (i32, [vp, vp, i32, C.c_char_p]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return ["sph_default_params", "sph_create", "sph_destroy", "sph_build_cells", "sph_sort_cells",
            "sph_mark_active", "sph_density_pass", "sph_force_pass", "sph_kick_drift", "sph_sync",
            "sph_last_error", "sph_info", "sph_copy_leaves", "sph_copy_particles", "sph_copy_axis_order",
            "sph_copy_active", "sph_copy_pairs", "sph_profile", "sph_profile_read", "sph_autotune",
            "sph_load_tuning", "sph_adjoint", "sph_batch_density_pass", "sph_batch_force_pass",
            "sph_batch_autotune", "sph_step", "sph_drift_all", "sph_batch_create", "sph_batch_mark_active",
            "sph_batch_density_force", "sph_batch_box", "sph_step_noalloc", "sph_next_active_time", "sph_drift"]


def require_device():
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the SPH path runs only on the HIP device")
    lib()


def default_params(**overrides) -> Params:
    p = Params()
    lib().sph_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class Particles:
    """Device arrays of the particle state (structure of arrays, cell order
    after build_cells)."""
    arrays: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.arrays["x"].shape[0]

    def __getitem__(self, k):
        return self.arrays[k]

    def __setitem__(self, k, v):
        self.arrays[k] = v
        self.__dict__.pop("_c", None)

    def c_struct(self) -> ParticlesC:
        """The C view of the arrays, built once (until an array is replaced)."""
        s = self.__dict__.get("_c")
        if s is None:
            s = self.to_c()
            self.__dict__["_c"] = s
        return s

    @classmethod
    def from_initial(cls, ic: dict, device="cuda", counts=True):
        """From a generator dict (x (N,3), v (N,3), m, u, h, bin); outputs
        zero-filled; A and Af are filled by the first density pass."""
        N = ic["x"].shape[0]
        a = {}
        dev = torch.device(device)
        for d, k in enumerate("xyz"):
            a[k] = torch.tensor(np.ascontiguousarray(ic["x"][:, d]), dtype=torch.float64, device=dev)
        v = ic.get("v", np.zeros((N, 3)))
        for d, k in enumerate(("vx", "vy", "vz")):
            a[k] = torch.tensor(np.ascontiguousarray(v[:, d]), dtype=torch.float64, device=dev)
            a["vf" + k[1]] = a[k].clone()
        a["m"] = torch.tensor(ic["m"], dtype=torch.float32, device=dev)
        a["u"] = torch.tensor(ic["u"], dtype=torch.float32, device=dev)
        a["h"] = torch.tensor(ic["h"], dtype=torch.float32, device=dev)
        a["time_bin"] = torch.tensor(ic.get("bin", np.zeros(N, np.int8)), dtype=torch.int8, device=dev)
        for name, dt in PARTICLE_FIELDS:
            if name in a:
                continue
            if name.startswith("nngb") and not counts:
                continue
            a[name] = torch.zeros(N, dtype=dt, device=dev)
        return cls(a)

    @classmethod
    def from_tensors(cls, x, v, m, u, h, counts=True):
        """From device tensors: x, v (N,3), m, u, h (N,).  Copies them into
        the library's layout (x, v as FP64 columns; m, u, h as FP32), so the
        caller's tensors are not modified by the calls."""
        N = x.shape[0]
        dev = x.device
        a = {}
        for d, k in enumerate("xyz"):
            a[k] = x[:, d].to(torch.float64).contiguous().clone()
        for d, k in enumerate(("vx", "vy", "vz")):
            a[k] = v[:, d].to(torch.float64).contiguous().clone()
            a["vf" + k[1]] = a[k].clone()
        a["m"] = m.to(torch.float32).contiguous().clone()
        a["u"] = u.to(torch.float32).contiguous().clone()
        a["h"] = h.to(torch.float32).contiguous().clone()
        a["time_bin"] = torch.zeros(N, dtype=torch.int8, device=dev)
        for name, dt in PARTICLE_FIELDS:
            if name in a:
                continue
            if name.startswith("nngb") and not counts:
                continue
            a[name] = torch.zeros(N, dtype=dt, device=dev)
        return cls(a)

    def to_c(self) -> ParticlesC:
        s = ParticlesC()
        for name, dt in PARTICLE_FIELDS:
            t = self.arrays.get(name)
            if t is not None:
                if t.dtype != dt or not t.is_contiguous() or t.device.type != "cuda":
                    raise TypeError(f"particle array {name}: need contiguous {dt} on the GPU")
                setattr(s, name, t.data_ptr())
        return s


class Context:
    """One sph_ctx bound to a torch stream (the current one by default).

    allocator: "torch" (default) takes every device buffer of the context
    from PyTorch's caching allocator on the context's stream; None lets the
    library use hipMalloc / hipFree; or a pair (alloc, free) of ALLOC_FN /
    FREE_FN callbacks."""

    def __init__(self, params: Params | None = None, stream=None, allocator="torch", **overrides):
        require_device()
        self.params = params if params is not None else default_params(**overrides)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if allocator == "torch":
            self._alloc = (TORCH_ALLOC, TORCH_FREE)
        elif allocator is None:
            self._alloc = (ALLOC_FN(), FREE_FN())
        else:
            self._alloc = tuple(allocator)
        h = C.c_void_p()
        self._check(lib().sph_create(C.byref(self.params), C.c_void_p(self.stream.cuda_stream), self._alloc[0],
                                     self._alloc[1], None, C.byref(h)), ctx=None)
        self.h = h
        self._owns = True
        self._pc = None
        # counts the calls that change the context's derived structures or
        # step state; a saved forward evaluation checks it before its backward
        self.generation = 0
        _live.add(self)

    def close(self):
        if getattr(self, "h", None) and getattr(self, "_owns", False) and callable(lib):
            lib().sph_destroy(self.h)
        self.h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        self.close()

    def _check(self, code, ctx="self"):
        if code != 0:
            msg = lib().sph_last_error(self.h).decode() if ctx == "self" and getattr(self, "h", None) else ""
            raise SPHError(code, msg)
        return code

    def _pcs(self, p: Particles, changes=True):
        self._pc = p.c_struct()   # kept alive while queued work reads the pointers
        if changes:
            self.generation += 1
        return C.byref(self._pc)

    # ---- the path
    def build_cells(self, p: Particles, perm_out: torch.Tensor | None = None):
        return self._check(lib().sph_build_cells(self.h, self._pcs(p), p.n, _ptr(perm_out)))

    def sort_cells(self):
        self.generation += 1
        return self._check(lib().sph_sort_cells(self.h))

    def mark_active(self, p: Particles, max_active_bin: int, want_count=True):
        n = C.c_int64(-1)
        self._check(lib().sph_mark_active(self.h, self._pcs(p), int(max_active_bin),
                                          C.byref(n) if want_count else None))
        return n.value

    def density_pass(self, p: Particles, entropy_from_u: bool):
        return self._check(lib().sph_density_pass(self.h, self._pcs(p), int(bool(entropy_from_u))))

    def force_pass(self, p: Particles):
        return self._check(lib().sph_force_pass(self.h, self._pcs(p)))

    def kick_drift(self, p: Particles, ti: int, t_min: float, drift_int: int, first_step: bool):
        return self._check(lib().sph_kick_drift(self.h, self._pcs(p), int(ti), float(t_min), int(drift_int),
                                                int(bool(first_step))))

    def step(self, p: Particles, max_active_bin: int, ti: int, t_min: float, drift_int: int, first_step: bool,
             entropy_from_u: bool = False, perm_out: torch.Tensor | None = None, want_count: bool = False):
        """build_cells, sort_cells, mark_active, density_pass, force_pass and
        kick_drift in one library call; returns the number of active
        particles with want_count (else -1)."""
        n = C.c_int64(-1)
        self._check(lib().sph_step(self.h, self._pcs(p), p.n, _ptr(perm_out), int(max_active_bin),
                                   C.byref(n) if want_count else None, int(bool(entropy_from_u)), int(ti),
                                   float(t_min), int(drift_int), int(bool(first_step))))
        return n.value

    def next_active_time(self, p: Particles, ti: int) -> int:
        """First time after ti (units of t_min) at which some particle is
        active: the next multiple of 2^(smallest time-bin)."""
        out = C.c_int64(-1)
        self._check(lib().sph_next_active_time(self.h, self._pcs(p, changes=False), int(ti), C.byref(out)))
        return out.value

    def drift(self, p: Particles, t_min: float, drift_int: int):
        """Move the time line on by drift_int units of t_min with no kick."""
        return self._check(lib().sph_drift(self.h, self._pcs(p), float(t_min), int(drift_int)))

    def drift_all(self, p: Particles):
        """With lazy drift: bring every particle to the current time."""
        return self._check(lib().sph_drift_all(self.h, self._pcs(p)))

    def adjoint(self, p: Particles, w: torch.Tensor):
        """dL/dx (N,3) float64 and dL/du (N,) float32 of L = sum_i w_i . a_i
        after an all-active force pass (cell order, as the particle arrays)."""
        w = w.to(torch.float32)
        wx, wy, wz = (w[:, d].contiguous() for d in range(3))
        n = p.n
        dev = w.device
        gx, gy, gz = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        gu = torch.empty(n, dtype=torch.float32, device=dev)
        self._check(lib().sph_adjoint(self.h, self._pcs(p, changes=False), _ptr(wx), _ptr(wy), _ptr(wz), _ptr(gx), _ptr(gy),
                                      _ptr(gz), _ptr(gu)))
        self._keep = (wx, wy, wz)
        return torch.stack([gx, gy, gz], 1), gu

    def sync(self):
        return self._check(lib().sph_sync(self.h))

    # ---- batches of boxes in this context
    def batch_create(self, box_sizes, box_L=None):
        """Turns this (unused) context into a batch of len(box_sizes) boxes
        whose particles are consecutive slices of the particle arrays."""
        nb = len(box_sizes)
        off = (C.c_int64 * (nb + 1))(*np.concatenate([[0], np.cumsum(np.asarray(box_sizes, np.int64))]).tolist())
        L = (C.c_double * nb)(*([1.0] * nb if box_L is None else [float(v) for v in box_L]))
        self.generation += 1
        self._check(lib().sph_batch_create(self.h, nb, off, L))
        self.n_boxes = nb
        return self

    def batch_mark_active(self, p: Particles, max_active_bins):
        m = (C.c_int * len(max_active_bins))(*[int(v) for v in max_active_bins])
        n = C.c_int64(-1)
        self._check(lib().sph_batch_mark_active(self.h, self._pcs(p), m, C.byref(n)))
        return n.value

    def batch_density_force(self, p: Particles, entropy_from_u: bool):
        return self._check(lib().sph_batch_density_force(self.h, self._pcs(p), int(bool(entropy_from_u))))

    def batch_box(self, b: int) -> "Context":
        """A view of box b's context (owned by this batch) for introspection."""
        k = lib().sph_batch_box(self.h, int(b))
        if not k:
            raise IndexError(b)
        v = Context.__new__(Context)
        v.params, v.stream, v._alloc = self.params, self.stream, self._alloc
        v.h, v._owns, v._pc, v.generation = C.c_void_p(k), False, None, 0
        v._parent = self
        return v

    def info(self) -> dict:
        inf = Info()
        self._check(lib().sph_info(self.h, C.byref(inf)))
        out = {k: getattr(inf, k) for k, _ in Info._fields_}
        out["unconverged_after_pass"] = list(out["unconverged_after_pass"])[:max(0, out["density_iterations"])]
        return out

    def autotune(self, p: Particles, path: str | None = None):
        return self._check(lib().sph_autotune(self.h, self._pcs(p), path.encode() if path else None))

    def load_tuning(self, path: str):
        return self._check(lib().sph_load_tuning(self.h, path.encode()))

    def profile(self, enable: bool):
        return self._check(lib().sph_profile(self.h, int(bool(enable))))

    def profile_read(self) -> dict:
        n = lib().sph_profile_read(self.h, None, 0)
        buf = C.create_string_buffer(int(n) + 1)
        lib().sph_profile_read(self.h, buf, int(n) + 1)
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    # ---- introspection
    def copy_leaves(self):
        nl = self.info()["n_leaves"]
        dev = torch.device("cuda")
        out = {k: torch.empty(nl, dtype=torch.int32, device=dev)
               for k in ("level", "ix", "iy", "iz", "begin", "count")}
        out["hmax"] = torch.empty(nl, dtype=torch.float32, device=dev)
        out["drift"] = torch.empty(nl, dtype=torch.float32, device=dev)
        self._check(lib().sph_copy_leaves(self.h, *[_ptr(out[k]) for k in
                                                    ("level", "ix", "iy", "iz", "begin", "count", "hmax", "drift")]))
        return out

    def copy_particles(self):
        n = self.info()["n"]
        dev = torch.device("cuda")
        keys = torch.empty(n, dtype=torch.int64, device=dev)
        o = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3)]
        self._check(lib().sph_copy_particles(self.h, _ptr(keys), *[_ptr(t) for t in o]))
        return keys, o

    def copy_axis_order(self):
        n = self.info()["n"]
        order = torch.empty(13 * n, dtype=torch.int16, device="cuda")
        self._check(lib().sph_copy_axis_order(self.h, _ptr(order)))
        return order.view(13, n)

    def copy_active(self):
        inf = self.info()
        dev = torch.device("cuda")
        act = torch.empty(inf["n"], dtype=torch.uint8, device=dev)
        al = torch.empty(max(1, inf["n_active_leaves"]), dtype=torch.int32, device=dev)
        hm = torch.empty(max(1, inf["n_active_leaves"]), dtype=torch.float32, device=dev)
        self._check(lib().sph_copy_active(self.h, _ptr(act), _ptr(al), _ptr(hm)))
        k = inf["n_active_leaves"]
        return act, al[:k], hm[:k]

    def copy_pairs(self, which: int):
        inf = self.info()
        np_ = inf["n_density_pairs"] if which == 0 else inf["n_force_pairs"]
        dev = torch.device("cuda")
        a = torch.empty(max(1, np_), dtype=torch.int32, device=dev)
        b = torch.empty(max(1, np_), dtype=torch.int32, device=dev)
        s = [torch.empty(max(1, np_), dtype=torch.float32, device=dev) for _ in range(3)]
        self._check(lib().sph_copy_pairs(self.h, int(which), _ptr(a), _ptr(b), *[_ptr(t) for t in s]))
        return a[:np_], b[:np_], torch.stack([t[:np_] for t in s], 1)


class Batch:
    """Batched passes over several contexts that share one stream: each loop
    pass of the density / force pass is one launch over all boxes' active
    chunks.  contexts[0] leads (work list, batch tuning table, errors)."""

    def __init__(self, contexts, particles):
        if len(contexts) != len(particles) or not contexts:
            raise ValueError("one particle set per context")
        self.contexts = list(contexts)
        self.particles = list(particles)
        self._h = (C.c_void_p * len(contexts))(*[c.h.value for c in contexts])

    def _ps(self):
        self._pc = (ParticlesC * len(self.particles))(*[p.to_c() for p in self.particles])
        return self._pc

    def density_pass(self, entropy_from_u: bool):
        return self.contexts[0]._check(lib().sph_batch_density_pass(self._h, self._ps(), len(self.contexts),
                                                                    int(bool(entropy_from_u))))

    def force_pass(self):
        return self.contexts[0]._check(lib().sph_batch_force_pass(self._h, self._ps(), len(self.contexts)))

    def autotune(self, path: str | None = None):
        return self.contexts[0]._check(lib().sph_batch_autotune(
            self._h, self._ps(), len(self.contexts), path.encode() if path else None))


class SPHForce(torch.autograd.Function):
    """a = SPHForce.apply(x, u, v, m, h0[, context]): accelerations (N,3,
    FP32) of one all-active density + force evaluation at positions x (N,3)
    and internal energies u, with velocities v, masses m and initial
    smoothing lengths h0 (solved for in the density pass).  The backward
    runs the library's adjoint and returns dL/dx (FP64) and dL/du; v, m and
    h0 get no gradient.  The forward keeps the context and the per-particle
    state of the evaluation for the backward."""

    @staticmethod
    def forward(fctx, x, u, v, m, h0, context=None):
        c = context if context is not None else Context()
        p = Particles.from_tensors(x.detach(), v.detach(), m.detach(), u.detach(), h0.detach())
        n = p.n
        perm = torch.empty(n, dtype=torch.int64, device=x.device)
        c.build_cells(p, perm)
        c.sort_cells()
        c.mark_active(p, c.params.n_bins - 1, want_count=False)
        c.density_pass(p, entropy_from_u=True)
        c.force_pass(p)
        a = torch.empty(n, 3, dtype=torch.float32, device=x.device)
        a[perm] = torch.stack([p["ax"], p["ay"], p["az"]], 1)
        fctx.sph = (c, p, perm, c.generation)
        fctx.x_dtype, fctx.u_dtype = x.dtype, u.dtype
        return a

    @staticmethod
    def backward(fctx, ga):
        c, p, perm, gen = fctx.sph
        if c.generation != gen:
            # the adjoint reads the context's current cells and pair lists
            raise RuntimeError("SPHForce backward: the context was used by another call after this forward "
                               "evaluation; give each evaluation its own context or run backward first")
        gx_s, gu_s = c.adjoint(p, ga[perm])
        gx = torch.empty(p.n, 3, dtype=torch.float64, device=ga.device)
        gu = torch.empty(p.n, dtype=torch.float32, device=ga.device)
        gx[perm] = gx_s
        gu[perm] = gu_s
        return gx.to(fctx.x_dtype), gu.to(fctx.u_dtype), None, None, None, None
