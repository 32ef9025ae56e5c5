"""The C ABI library loads and exports every entry point that include/dottt.h declares (no GPU
needed: nothing here launches device work)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dottt.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(dt_[a-z_]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2106_02762_amd as dt
    return dt.library()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("dt_ctx_create", "dt_graph_load", "dt_graph_build", "dt_count",
                     "dt_count_batch", "dt_server_start", "dt_server_submit", "dt_server_wait"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2106_02762_amd as dt
    out = subprocess.run(["nm", "-D", "--defined-only", dt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (dt_[a-z_]+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert sorted(dt.ENTRY_POINTS) == _declared()


def test_host_only_calls(lib):
    import paper_2106_02762_amd as dt
    assert dt.dt_strerror(dt.DT_EINVAL) == "invalid argument"
    assert dt.dt_strerror(0) == "ok"
    assert isinstance(dt.dt_last_error(), str)


def test_library_is_built_for_gfx950():
    import paper_2106_02762_amd as dt
    data = open(dt.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
