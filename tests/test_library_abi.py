"""CPU checks of the C-ABI library: it loads and exports every function the
header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sphgpu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for f in ("sph_build_cells", "sph_sort_cells", "sph_mark_active", "sph_density_pass", "sph_force_pass",
              "sph_kick_drift", "sph_create", "sph_destroy"):
        assert f in names


def test_header_declares_the_boundary_calls():
    """The calls of the boundary: the path, the allocator callbacks of
    sph_create, the one-context batch and the adjoint."""
    text = open(os.path.join(ROOT, "include", "sphgpu.h")).read()
    flat = re.sub(r"\s+", " ", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
    assert "typedef void *(*sph_alloc_fn)(size_t bytes, void *hip_stream, void *user);" in flat
    assert "typedef void (*sph_free_fn)(void *ptr, void *hip_stream, void *user);" in flat
    assert ("sph_status sph_create(const sph_params *p, void *hip_stream, sph_alloc_fn alloc, sph_free_fn free, "
            "void *user, sph_ctx **out);") in flat
    names = declared_functions()
    for f in ("sph_batch_create", "sph_batch_density_force", "sph_batch_mark_active", "sph_batch_box",
              "sph_adjoint", "sph_step", "sph_sync", "sph_last_error"):
        assert f in names, f


def test_library_exports_every_declared_symbol():
    import paper_1807_01341_amd as sg
    if not os.path.exists(sg.LIB_PATH):
        pytest.fail("libsphgpu.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(sg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(sg.exported_symbols()) == declared_functions()


def test_default_params_and_struct_layout():
    import paper_1807_01341_amd as sg
    p = sg.default_params()
    assert p.split_count == 400 and p.morton_depth == 16 and abs(p.cfl - 0.2) == 0.0
    assert abs(p.eta - 1.2348) < 1e-6 and p.n_bins == 14
    # the ctypes mirror has the C field order and sizes
    text = open(os.path.join(ROOT, "include", "sphgpu.h")).read()
    body = text[text.index("typedef struct {\n  double *x"):text.index("} sph_particles;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\*(\w+)", body)
    assert names == [n for n, _ in sg.PARTICLE_FIELDS]
    pbody = text[text.index("typedef struct {\n  double box"):text.index("} sph_params;")]
    pbody = re.sub(r"/\*.*?\*/", "", pbody, flags=re.S)
    pnames = re.findall(r"(\w+);", pbody)
    assert pnames == [n for n, _ in sg.Params._fields_]


def test_binding_refuses_without_device():
    import torch

    import paper_1807_01341_amd as sg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        sg.Context()
