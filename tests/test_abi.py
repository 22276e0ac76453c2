"""The C-ABI library loads and exports every entry point include/fmm.h
declares; host-only entry points behave (no GPU needed, no kernel launched)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1405_2255_amd", "libfmm.so")
HDR = os.path.join(ROOT, "include", "fmm.h")


def _declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfmm.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("fmm_build", "fmm_forces", "fmm_forces_batched", "fmm_direct", "fmm_stats",
                 "fmm_footprint_bytes", "fmm_last_error", "fmm_destroy", "fmm_export",
                 "fmm_order_for_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_lists_the_same_symbols():
    from paper_1405_2255_amd import fmm
    assert sorted(fmm.SYMBOLS) == _declared()


def test_host_only_entry_points(lib):
    lib.fmm_order_for_error.restype = C.c_int
    lib.fmm_order_for_error.argtypes = [C.c_double]
    # two above the paper's CPU optimum p = 10 at eps = 10^-6.25 (Sec. 6.2, Fig. 10)
    assert lib.fmm_order_for_error(10 ** -6.25) == 12
    assert lib.fmm_order_for_error(0.0) == -1
    assert lib.fmm_order_for_error(float("nan")) == -1
    assert 3 <= lib.fmm_order_for_error(1e-3) <= lib.fmm_order_for_error(1e-9) <= 20
    lib.fmm_footprint_bytes.restype = C.c_size_t
    lib.fmm_footprint_bytes.argtypes = [C.c_int64, C.c_int, C.c_void_p]
    a = lib.fmm_footprint_bytes(10 ** 5, 10, None)
    b = lib.fmm_footprint_bytes(10 ** 6, 10, None)
    assert 0 < a < b
    assert lib.fmm_footprint_bytes(0, 10, None) == 0
    lib.fmm_last_error.restype = C.c_char_p
    lib.fmm_last_error.argtypes = [C.c_void_p]
    assert lib.fmm_last_error(None) == b"null context"
    lib.fmm_destroy.argtypes = [C.c_void_p]
    lib.fmm_destroy(None)
    lib.fmm_build.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.fmm_build(None, None) == 1          # FMM_E_INVAL
    lib.fmm_stats.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.fmm_stats(None, None) == 1
    lib.fmm_forces.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_double,
                               C.c_int, C.c_double, C.c_void_p, C.c_void_p]
    assert lib.fmm_forces(None, 10, None, None, 1.0, 8, 1e-7, None, None) == 1


def test_option_and_stats_layouts_match_header():
    """The binding's ctypes structures list the header's members in order."""
    import re
    from paper_1405_2255_amd import fmm
    hdr = open(HDR).read()

    def members(name):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", hdr).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(None, 1)[1] if " " in decl else decl
            for v in names.split(","):
                out.append(v.strip().lstrip("*").strip())
        return out

    assert [f[0] for f in fmm.Opts._fields_] == members("fmm_opts")
    assert [f[0] for f in fmm.Stats._fields_] == members("fmm_stats_t")


def test_destroy_releases_every_device_buffer():
    """Every DevBuf member of the context is in fmm_destroy's release list."""
    src = open(os.path.join(ROOT, "paper_1405_2255_amd", "csrc", "api.hip")).read()
    body = src[src.index("struct fmm_ctx {"):]
    body = body[:body.index("\n};")]
    body = re.sub(r"//[^\n]*", "", body)
    members = [v.strip() for d in re.findall(r"DevBuf\s+([^;]*);", body) for v in d.split(",")]
    listed = re.search(r"DevBuf \*bufs\[\] = \{(.*?)\};", src, re.S).group(1)
    listed = {v.strip().replace("&c->", "") for v in listed.split(",")}
    assert members and not [m for m in members if m not in listed]
