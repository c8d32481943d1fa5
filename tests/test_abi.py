"""The C-ABI library loads and exports every entry point the public header
declares, and the Python binding covers exactly that set (no compute calls:
these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spvar.h")
LIB = os.path.join(ROOT, "paper_1706_07826_amd", "libspvar.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(spv_[a-z_0-9]+)\s*\(", text,
                          flags=re.M))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: build with __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    d = _declared()
    for name in ("spv_ctx_create", "spv_sample", "spv_persist_fix", "spv_ispvar", "spv_pt_sample",
                 "spv_top_sample", "spv_sample_batch", "spv_server_submit"):
        assert name in d


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_exported_set_matches_header():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T spv_" in l}
    assert exported == _declared()


def test_binding_covers_header():
    import paper_1706_07826_amd as spv
    assert set(spv.EXPORTED) == _declared()


def test_version_string(lib):
    lib.spv_version.restype = ctypes.c_char_p
    assert lib.spv_version().decode().startswith("spvar-mi355x")


def test_null_context_is_rejected_without_device(lib):
    """Argument checks that fire before any device work."""
    lib.spv_sample.restype = ctypes.c_int
    assert lib.spv_sample(None, None, None, 0, 0, ctypes.c_uint64(0), 0, None, None, None, None) == -1
    lib.spv_server_submit.restype = ctypes.c_int
    assert lib.spv_server_submit(None, None, None) == -1
    lib.spv_last_error.restype = ctypes.c_char_p
    assert lib.spv_last_error(None) == b"no context"
