"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports
every entry point declared in include/flexipart.h; the binding refuses to run
without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flexipart.h")
LIB = os.path.join(ROOT, "paper_2211_05458_amd", "libflexipart.so")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fp_[a-z0-9_]+)\s*\(", txt)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_export_list_matches_header():
    from paper_2211_05458_amd import lib
    assert sorted(lib.EXPORTS) == _declared()
    assert lib.load().fp_mlp_n_weights() == 64 * 84 + 64 + 2 * (64 * 64 + 64) + 3 * 64 + 3


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_validation_without_gpu():
    """Argument checks that run before any device call."""
    import numpy as np
    from paper_2211_05458_amd import lib, workloads as W
    L = lib.load()
    ctx = ctypes.c_void_p()
    assert L.fp_create(ctypes.byref(ctx), None) == 0
    mesh = W.config1(n_particles=1, cells=2).mesh
    keep = [np.ascontiguousarray(mesh.X), mesh.nbr_elem.copy(), mesh.nbr_face.copy(), mesh.bc.copy(),
            np.ascontiguousarray(mesh.shift)]
    desc = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep], 3, 0)
    assert L.fp_init_mesh(ctx, ctypes.byref(desc)) == 0
    # unsupported degree
    bad = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep], 9, 0)
    assert L.fp_init_mesh(ctx, ctypes.byref(bad)) == lib.FP_EINVAL
    # non-reciprocal neighbour table
    ne = keep[1].copy()
    ne[0, 1] = 3
    keep2 = [keep[0], ne, keep[2], keep[3], keep[4]]
    bad = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep2], 3, 0)
    assert L.fp_init_mesh(ctx, ctypes.byref(bad)) == lib.FP_EMESH
    assert b"reciprocal" in L.fp_last_error(ctx)
    # calls out of order
    assert L.fp_init_mesh(ctx, ctypes.byref(desc)) == 0
    o = lib.StepOpts(1, 1, 0, 0, 1, 50, 64, 0, 0, (ctypes.c_double * 3)(0, 0, 0))
    assert L.fp_step(ctx, 1e-3, 1, ctypes.byref(o)) == lib.FP_ESTATE
    sz = ctypes.c_size_t(0)
    assert L.fp_workspace_size(ctx, 1000, ctypes.byref(sz)) == 0 and sz.value > 0
    L.fp_destroy(ctx)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2211_05458_amd import lib
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(lib.FPError):
        lib.load()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_mortar_table_validation_without_gpu():
    """A non-conforming mesh is accepted with its mortar table; a table that
    lists a small face of another big face, or a missing table, is rejected."""
    import numpy as np
    from paper_2211_05458_amd import lib, workloads as W
    L = lib.load()
    ctx = ctypes.c_void_p()
    assert L.fp_create(ctypes.byref(ctx), None) == 0
    mesh = W.mortar_box(n_geo=1, N=1, refine=(2, 2), n_particles=1).mesh
    keep = [np.ascontiguousarray(mesh.X), mesh.nbr_elem.copy(), mesh.nbr_face.copy(), mesh.bc.copy(),
            np.ascontiguousarray(mesh.shift)]
    tab = np.ascontiguousarray(mesh.mortar, np.int32)
    desc = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep], 1, 0, tab.shape[0], lib._ptr(tab))
    assert L.fp_init_mesh(ctx, ctypes.byref(desc)) == 0
    wrong = tab.copy()
    wrong[0, 1] = wrong[1, 1]
    bad = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep], 1, 0, wrong.shape[0], lib._ptr(wrong))
    assert L.fp_init_mesh(ctx, ctypes.byref(bad)) == lib.FP_EMESH
    bad = lib.MeshDesc(mesh.n_elem, 1, *[lib._ptr(a) for a in keep], 1, 0, 0, None)
    assert L.fp_init_mesh(ctx, ctypes.byref(bad)) == lib.FP_EMESH
    L.fp_destroy(ctx)
