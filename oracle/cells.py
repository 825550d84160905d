"""ctypes front of oracle/cells.c (test infrastructure only).

`build_library()` compiles cells.c with gcc (-O2 -ffp-contract=off); the
loader compiles it on first use if the shared object is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cells.c")
_LIB = os.path.join(_HERE, "libsphoracle_cells.so")
_lib = None


def build_library() -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library()
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def build_cells(x, h, L=1.0, split=400, D=21, top_cap=7):
    """Cell build of the C definitions; see cells.c.  x (N,3) f64, h (N,) f32
    in original order.  Returns a dict of sorted-order arrays and the leaf table."""
    x = np.ascontiguousarray(x, np.float64)
    h = np.ascontiguousarray(h, np.float32)
    n = x.shape[0]
    xs, ys, zs = (np.ascontiguousarray(x[:, a]) for a in range(3))
    out = dict(perm=np.empty(n, np.int64), key=np.empty(n, np.uint64),
               xw=np.empty(n), yw=np.empty(n), zw=np.empty(n),
               ox=np.empty(n, np.float32), oy=np.empty(n, np.float32), oz=np.empty(n, np.float32),
               H=np.empty(n, np.float32), leaf_of=np.empty(n, np.int64),
               leaf_level=np.empty(n, np.int32), leaf_ix=np.empty(n, np.int64),
               leaf_iy=np.empty(n, np.int64), leaf_iz=np.empty(n, np.int64),
               leaf_begin=np.empty(n, np.int64), leaf_count=np.empty(n, np.int32),
               leaf_hmax=np.empty(n, np.float32))
    k0 = C.c_int32()
    nl = C.c_int64()
    f = lib().emu_build_cells
    f.restype = C.c_int
    rc = f(C.c_int64(n), _p(xs), _p(ys), _p(zs), _p(h), C.c_double(L), C.c_int(split), C.c_int(D),
           C.c_int(top_cap), _p(out["perm"]), _p(out["key"]), _p(out["xw"]), _p(out["yw"]), _p(out["zw"]),
           _p(out["ox"]), _p(out["oy"]), _p(out["oz"]), _p(out["H"]), _p(out["leaf_of"]),
           _p(out["leaf_level"]), _p(out["leaf_ix"]), _p(out["leaf_iy"]), _p(out["leaf_iz"]),
           _p(out["leaf_begin"]), _p(out["leaf_count"]), _p(out["leaf_hmax"]), C.byref(k0), C.byref(nl))
    if rc != 0:
        raise ValueError("max smoothing length exceeds a quarter of the box")
    nl = nl.value
    for k in ("leaf_level", "leaf_ix", "leaf_iy", "leaf_iz", "leaf_begin", "leaf_count", "leaf_hmax"):
        out[k] = out[k][:nl].copy()
    out.update(n_leaves=nl, top_level=k0.value, L=L, D=D, split=split)
    return out


def axis_vectors():
    e = np.empty(39, np.float32)
    lib().emu_axis_vectors(_p(e))
    return e.reshape(13, 3)


def axis_sort(cells):
    n = cells["ox"].size
    order = np.empty(13 * n, np.uint16)
    keys = np.empty(13 * n, np.float32)
    f = lib().emu_axis_sort
    f.restype = C.c_int
    rc = f(C.c_int64(n), C.c_int64(cells["n_leaves"]), _p(cells["leaf_begin"]), _p(cells["leaf_count"]),
           _p(cells["ox"]), _p(cells["oy"]), _p(cells["oz"]), _p(order), _p(keys))
    if rc != 0:
        raise ValueError("leaf larger than 65535 particles")
    return order.reshape(13, n), keys.reshape(13, n)


def mark_active(cells, bin_sorted, m, H=None):
    """Active particles (bin <= m), active leaves and their max active H.
    H defaults to the build's H (sorted order)."""
    n = cells["ox"].size
    H = cells["H"] if H is None else np.ascontiguousarray(H, np.float32)
    b = np.ascontiguousarray(bin_sorted, np.int8)
    active = np.empty(n, np.uint8)
    al = np.empty(cells["n_leaves"], np.int64)
    hm = np.empty(cells["n_leaves"], np.float32)
    f = lib().emu_mark_active
    f.restype = C.c_int64
    na = f(C.c_int64(n), _p(b), C.c_int(m), C.c_int64(cells["n_leaves"]), _p(cells["leaf_begin"]),
           _p(cells["leaf_count"]), _p(H), _p(active), _p(al), _p(hm))
    return dict(active=active.astype(bool), active_leaves=al[:na].copy(), hmax_act=hm[:na].copy())


def leaf_hmax(cells, H):
    """Max H per leaf for an H array in sorted order."""
    H = np.asarray(H, np.float32)
    out = np.zeros(cells["n_leaves"], np.float32)
    for l in range(cells["n_leaves"]):
        b, c = cells["leaf_begin"][l], cells["leaf_count"][l]
        out[l] = H[b:b + c].max()
    return out


def pairs(cells, act, mode, leaf_hmax_arr=None, leaf_dx=None):
    """All-pairs cell test (mode 'density' or 'force'), widened by the leaves'
    drift margins when leaf_dx is given.  Returns (A, B, s) with s (P,3)
    float32 shifts, in (A, B) order."""
    md = {"density": 0, "force": 1}[mode]
    lh = cells["leaf_hmax"] if leaf_hmax_arr is None else np.ascontiguousarray(leaf_hmax_arr, np.float32)
    f = lib().emu_pairs
    f.restype = C.c_int64
    cap = max(1, 64 * len(act["active_leaves"]))
    while True:
        pa = np.empty(cap, np.int64)
        pb = np.empty(cap, np.int64)
        s = np.empty((3, cap), np.float32)
        np_ = f(C.c_int(md), C.c_double(cells["L"]), C.c_int(cells["D"]),
                C.c_int64(len(act["active_leaves"])), _p(act["active_leaves"]), _p(act["hmax_act"]),
                C.c_int64(cells["n_leaves"]), _p(cells["leaf_level"]), _p(cells["leaf_ix"]),
                _p(cells["leaf_iy"]), _p(cells["leaf_iz"]), _p(lh),
                None if leaf_dx is None else _p(np.ascontiguousarray(leaf_dx, np.float32)), C.c_int64(cap),
                _p(pa), _p(pb), _p(s[0]), _p(s[1]), _p(s[2]))
        if np_ <= cap:
            return pa[:np_].copy(), pb[:np_].copy(), s[:, :np_].T.copy()
        cap = int(np_)


def counts(cells, mode, samples, H=None):
    """FP32 neighbour counts (j != i) for sampled sorted indices."""
    md = {"density": 0, "force": 1}[mode]
    H = cells["H"] if H is None else np.ascontiguousarray(H, np.float32)
    samples = np.ascontiguousarray(samples, np.int64)
    out = np.empty(samples.size, np.int64)
    lib().emu_counts(C.c_int(md), C.c_double(cells["L"]), C.c_int(cells["D"]), C.c_int64(cells["ox"].size),
                     _p(cells["ox"]), _p(cells["oy"]), _p(cells["oz"]), _p(H), _p(cells["leaf_of"]),
                     _p(cells["leaf_level"]), _p(cells["leaf_ix"]), _p(cells["leaf_iy"]), _p(cells["leaf_iz"]),
                     C.c_int64(samples.size), _p(samples), _p(out))
    return out


def counts_grid(cells, mode, samples, H=None):
    """The counts of `counts`, with candidates from a grid over the wrapped
    positions (fast for large inputs; equal to `counts` by construction and
    by test)."""
    md = {"density": 0, "force": 1}[mode]
    H = cells["H"] if H is None else np.ascontiguousarray(H, np.float32)
    samples = np.ascontiguousarray(samples, np.int64)
    out = np.empty(samples.size, np.int64)
    xw, yw, zw = (np.ascontiguousarray(cells[k], np.float64) for k in ("xw", "yw", "zw"))
    f = lib().emu_counts_grid
    f.restype = C.c_int
    rc = f(C.c_int(md), C.c_double(cells["L"]), C.c_int(cells["D"]), C.c_int64(cells["ox"].size), _p(xw), _p(yw),
           _p(zw), _p(cells["ox"]), _p(cells["oy"]), _p(cells["oz"]), _p(H), _p(cells["leaf_of"]),
           _p(cells["leaf_level"]), _p(cells["leaf_ix"]), _p(cells["leaf_iy"]), _p(cells["leaf_iz"]),
           C.c_int64(samples.size), _p(samples), _p(out))
    if rc != 0:
        raise MemoryError("emu_counts_grid: allocation failed")
    return out


def update(cells, x_sorted, h_sorted, x_build, frac=0.125):
    """The cells of `cells` kept for new positions (sorted order): wrapped
    positions, offsets by the minimum image, H, leaf max H, leaf drift
    margins and the rebuild flag, as the C definitions compute them."""
    x = np.ascontiguousarray(x_sorted, np.float64).copy()
    xs, ys, zs = (np.ascontiguousarray(x[:, a]) for a in range(3))
    xb = np.ascontiguousarray(x_build, np.float64)
    xbs, ybs, zbs = (np.ascontiguousarray(xb[:, a]) for a in range(3))
    h = np.ascontiguousarray(h_sorted, np.float32)
    n = x.shape[0]
    nl = cells["n_leaves"]
    out = dict(ox=np.empty(n, np.float32), oy=np.empty(n, np.float32), oz=np.empty(n, np.float32),
               H=np.empty(n, np.float32), leaf_hmax=np.empty(nl, np.float32), leaf_dx=np.empty(nl, np.float32))
    f = lib().emu_update
    f.restype = C.c_int
    flag = f(C.c_int64(n), _p(xs), _p(ys), _p(zs), _p(h), _p(xbs), _p(ybs), _p(zbs), C.c_double(cells["L"]),
             C.c_int(cells["D"]), C.c_int64(nl), _p(cells["leaf_begin"]), _p(cells["leaf_count"]),
             _p(cells["leaf_level"]), _p(cells["leaf_ix"]), _p(cells["leaf_iy"]), _p(cells["leaf_iz"]),
             C.c_float(frac), _p(out["ox"]), _p(out["oy"]), _p(out["oz"]), _p(out["H"]), _p(out["leaf_hmax"]),
             _p(out["leaf_dx"]))
    new = dict(cells)
    new.update(out)
    new["xw"], new["yw"], new["zw"] = xs, ys, zs
    return new, bool(flag)
