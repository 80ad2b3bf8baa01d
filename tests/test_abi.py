"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bhfwi.h")
LIB = os.path.join(ROOT, "paper_2005_00281_amd", "libbhfwi.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bhfwi_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_path_entry_points():
    names = declared()
    for verb in ("bhfwi_fwd_model", "bhfwi_adjoint_model", "bhfwi_gradient",
                 "bhfwi_precondition", "bhfwi_update", "bhfwi_misfit", "bhfwi_moduli"):
        assert verb in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbhfwi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbhfwi.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_2005_00281_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbhfwi.so not built")
def test_create_rejects_bad_geometry_without_gpu_work():
    """Validation happens before any device call: a receiver outside the
    grid, a CFL violation, a window outside the model and two receivers on
    one row are refused with their codes."""
    from paper_2005_00281_amd import _lib
    L = _lib.load()
    sh = (_lib.Shot * 1)()
    sh[0] = _lib.Shot(16, 32, 4, 4, 5e-3, 5e-3, 0.5e-6, 10, 1e4, 4000.0, 10, 1, 0, 0, 0, 40)
    rec = (ctypes.c_int32 * 1)(999)
    h = ctypes.c_void_p()
    rc = L.bhfwi_create(ctypes.byref(h), 0, sh, 1, rec, 1, 20 * 40, 10)
    assert rc == -1 and b"receiver" in L.bhfwi_last_error(None)
    rec[0] = 12
    sh[0].dt = 1e-6  # 4000 * 1e-6 * sqrt(2) / 5e-3 = 1.13
    rc = L.bhfwi_create(ctypes.byref(h), 0, sh, 1, rec, 1, 20 * 40, 10)
    assert rc == -2 and b"vmax" in L.bhfwi_last_error(None)
    sh[0].dt = 0.5e-6
    sh[0].model_off = 5  # window runs past the model
    rc = L.bhfwi_create(ctypes.byref(h), 0, sh, 1, rec, 1, 20 * 40, 10)
    assert rc == -1 and b"model window" in L.bhfwi_last_error(None)
    sh[0].model_off = 0
    two = (ctypes.c_int32 * 2)(12, 12)  # two receivers on one row
    sh[0].nrec = 2
    rc = L.bhfwi_create(ctypes.byref(h), 0, sh, 1, two, 2, 20 * 40, 10)
    assert rc == -1 and b"two receivers" in L.bhfwi_last_error(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbhfwi.so not built")
def test_library_build_id_matches_the_sources(monkeypatch):
    """The library carries the hash of the sources it was built from; the
    loader refuses a library whose sources have changed since."""
    from paper_2005_00281_amd import _lib, build
    lib = ctypes.CDLL(LIB)
    lib.bhfwi_build_id.restype = ctypes.c_char_p
    assert lib.bhfwi_build_id().decode() == build.source_id()
    saved = _lib._lib
    try:
        _lib._lib = None
        monkeypatch.setattr(build, "source_id", lambda: "0" * 64)
        with pytest.raises(RuntimeError, match="stale"):
            _lib.load()
    finally:
        _lib._lib = saved


def _header_struct_fields(name):
    """Field names and C types of `typedef struct { ... } name;` in the header,
    in order (comments dropped; `int32_t a, b;` gives both names)."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*%s;" % name, txt).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        out += [(n.strip(), ctype) for n in names.split(",")]
    return out


@pytest.mark.parametrize("struct,cls", [("bhfwi_shot", "Shot"), ("bhfwi_sizes_t", "Sizes"),
                                        ("bhfwi_tune", "Tune"),
                                        ("bhfwi_plan_bytes_t", "PlanBytes"),
                                        ("bhfwi_plan_info", "PlanInfo"),
                                        ("bhfwi_kernel_times_t", "KernelTimes"),
                                        ("bhfwi_bounds", "Bounds")])
def test_binding_structs_match_the_header(struct, cls):
    # the ctypes mirrors of the ABI structs: same fields, order and widths
    from paper_2005_00281_amd import _lib
    width = {"int32_t": 4, "int64_t": 8, "float": 4, "double": 8}
    hdr = _header_struct_fields(struct)
    py = getattr(_lib, cls)._fields_
    assert [n for n, _ in hdr] == [n for n, _ in py]
    for (n, ctype), (_, pytype) in zip(hdr, py):
        assert width[ctype] == ctypes.sizeof(pytype), (struct, n)
