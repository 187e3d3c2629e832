"""The C-ABI library: loads without a GPU, exports every symbol include/glbm.h
declares, and validates descriptors on the host (no device calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(glbm_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported():
    import paper_1601_00704_amd.glbm as g
    lib = ctypes.CDLL(g.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(g.EXPORTS) <= names | {"glbm_last_error"}


def test_binding_has_same_names():
    import paper_1601_00704_amd.glbm as g
    for n in declared_functions():
        assert hasattr(g, n), n


def _desc(lib, **kw):
    base = dict(shape=(32, 64))
    base.update(kw)
    shape = base.pop("shape")
    return lib.make_desc(shape, **base)


def test_required_bytes_and_validation():
    import paper_1601_00704_amd.glbm as g
    ok = _desc(g)
    nb = g.glbm_required_bytes([ok])
    assert nb >= 2 * 9 * 32 * 64 * 4 and nb % 256 == 0
    nb64 = g.glbm_required_bytes([_desc(g, store=g.GLBM_STORE_F64)])
    nb16 = g.glbm_required_bytes([_desc(g, store=g.GLBM_STORE_F16DEV, flags=g.GLBM_FLAG_F16DEV_OPT_IN)])
    nb16l = g.glbm_required_bytes([_desc(g, store=g.GLBM_STORE_F16LOC)])
    assert nb64 > nb > nb16l > nb16
    bad = [
        _desc(g, tau=0.5),
        _desc(g, check_every=7),
        _desc(g, wall_faces=0b0100),            # one-sided wall
        _desc(g, shape=(2, 8, 8)),              # D2Q9 with nz = 2
        _desc(g, lattice=7),
        _desc(g, store=5),
        _desc(g, shape=(0, 8)),
        _desc(g, store=g.GLBM_STORE_F16DEV, dev_scale_log2=40, flags=g.GLBM_FLAG_F16DEV_OPT_IN),
        _desc(g, g=(float("nan"), 0, 0)),
        _desc(g, flags=2),                      # unknown flag bit
    ]
    for d in bad:
        assert g.glbm_required_bytes([d]) == 0
        assert g.glbm_last_error() != ""
    # the literal FP16 deviation store needs its explicit opt-in, and the message says why
    assert g.glbm_required_bytes([_desc(g, store=g.GLBM_STORE_F16DEV)]) == 0
    assert "F16LOC" in g.glbm_last_error() and "OPT_IN" in g.glbm_last_error()
    # mixed lattices / stores in one context are rejected
    assert g.glbm_required_bytes([ok, _desc(g, store=g.GLBM_STORE_F64)]) == 0
    assert g.glbm_required_bytes([ok, _desc(g, shape=(16, 16))]) > nb


def test_velocity_sets_match_oracle():
    import oracle
    import paper_1601_00704_amd.glbm as g
    for q in (9, 19):
        e, w = g.glbm_velocity_set(q)
        eo, wo, _ = oracle.lattice(q)
        a = sorted((tuple(v), x) for v, x in zip(e.tolist(), w.tolist()))
        b = sorted((tuple(v), x) for v, x in zip(eo.tolist(), wo.tolist()))
        assert [x[0] for x in a] == [x[0] for x in b]
        assert np.allclose([x[1] for x in a], [x[1] for x in b], rtol=0, atol=1e-16)
    with pytest.raises(g.GlbmError):
        g.glbm_velocity_set(7)


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    """The binding refuses to import when libglbm.so is absent (no fallback)."""
    import importlib.util
    src = os.path.join(ROOT, "paper_1601_00704_amd", "glbm.py")
    pkg = tmp_path / "fakepkg"
    pkg.mkdir()
    (pkg / "glbm.py").write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("fakeglbm", str(pkg / "glbm.py"))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_largest_lattice_limit():
    """Population indices are 32-bit: (q + 3) x the node count, rounded up to whole node
    blocks, must stay below 2^31.  Sizes are computed only; nothing is allocated."""
    import paper_1601_00704_amd.glbm as g
    ny = 16384                                    # D2Q9: q + 3 = 12
    assert 12 * ny * 10240 < 1 << 31 <= 12 * ny * 11264
    assert g.glbm_required_bytes([_desc(g, shape=(ny, 10240))]) > 0
    assert g.glbm_required_bytes([_desc(g, shape=(ny, 11264))]) == 0
    assert "32-bit" in g.glbm_last_error()
    # D3Q19 (q + 3 = 22): 448^3 fits, 480^3 does not
    assert g.glbm_required_bytes([_desc(g, shape=(448, 448, 448), lattice=g.GLBM_D3Q19)]) > 0
    assert g.glbm_required_bytes([_desc(g, shape=(480, 480, 480), lattice=g.GLBM_D3Q19)]) == 0


def test_host_queries_reject_null_arguments():
    """The host-only queries answer without a device: a null context or output is an
    argument error, not a crash."""
    import paper_1601_00704_amd.glbm as g
    lib = ctypes.CDLL(g.LIB_PATH)
    lib.glbm_sweeps_per_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.glbm_sweeps_per_launch(None, None) == g.GLBM_EINVAL
    out = ctypes.c_int32(7)
    assert lib.glbm_sweeps_per_launch(None, ctypes.byref(out)) == g.GLBM_EINVAL and out.value == 7
    lib.glbm_pore_percolates.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    assert lib.glbm_pore_percolates(9, 4, 4, 1, None, 1, ctypes.byref(out)) == g.GLBM_EINVAL
    cls = np.zeros(16, np.uint8)
    assert lib.glbm_pore_percolates(9, 4, 4, 1, cls.ctypes.data, 1, None) == g.GLBM_EINVAL
    assert lib.glbm_pore_percolates(9, 4, 4, 1, cls.ctypes.data, 1, ctypes.byref(out)) == g.GLBM_OK
    assert out.value == 1
