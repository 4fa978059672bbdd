"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host (no GPU needed;
no kernel is launched by these calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "graphreduce.h")


def _lib():
    from paper_1812_08942_amd import build, graphreduce

    if not os.path.exists(graphreduce.LIB_PATH):
        build.build(force=False)
    return graphreduce


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gr_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_are_exported():
    G = _lib()
    lib = G.load()
    names = declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), f"{name} declared but not exported"
    # the binding wraps every declared entry point under the same name
    assert set(names) <= set(G.exported_symbols())
    for name in names:
        assert hasattr(G, name), f"binding lacks {name}"


def test_status_strings_and_version():
    G = _lib()
    lib = G.load()
    assert lib.gr_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.gr_status_string(code)
    assert lib.gr_status_string(-99) == b"unknown status"


def test_workspace_size_argument_checks():
    G = _lib()
    assert G.gr_workspace_size(1000, 8000, 16, G.GR_F32) > 0
    big = G.gr_workspace_size(256**3, 100270080, 32, G.GR_BF16)
    assert big < 16 * 2**30          # fits easily in 288 GB
    with pytest.raises(G.GraphReduceError) as e:
        G.gr_workspace_size(10, 10, 6, G.GR_F32)     # 24-byte rows
    assert e.value.code == -6
    out = ctypes.c_size_t(0)
    assert G.load().gr_workspace_size(10, 10, 8, 7, ctypes.byref(out)) == -6
    with pytest.raises(G.GraphReduceError):
        G.gr_workspace_size(10, 10, 12, G.GR_BF16)   # bf16 needs K % 8
    with pytest.raises(G.GraphReduceError):
        G.gr_workspace_size(-1, 10, 8, G.GR_F32)


def test_null_arguments_rejected_before_any_launch():
    G = _lib()
    lib = G.load()
    assert lib.gr_validate(None, None, 0, None) == -1
    assert b"NULL" in lib.gr_last_error()
    g = G.gr_graph(4, 6, None, None, None)           # null row_ptr
    assert lib.gr_validate(ctypes.byref(g), None, 0, None) == -1
    g = G.gr_graph(-1, 0, 8, None, None)
    assert lib.gr_validate(ctypes.byref(g), None, 0, None) == -1
    p = G.gr_params(8, 5, 0.5, 1, 1, 0, None, 0, 0, 0)   # ratio < 1
    r = G.gr_result()
    g = G.gr_graph(4, 0, 16, None, None)
    assert lib.gr_reduce(ctypes.byref(g), ctypes.byref(p), ctypes.byref(r),
                         None, 0, None) == -1
    assert b"ratio" in lib.gr_last_error()
    p = G.gr_params(8, -1, 2.0, 1, 1, 0, None, 0, 0, 0)  # negative sweeps
    assert lib.gr_reduce(ctypes.byref(g), ctypes.byref(p), ctypes.byref(r),
                         None, 0, None) == -1
    p = G.gr_params(10, 5, 2.0, 1, 1, 0, None, 0, 0, 0)  # K=10 unsupported
    assert lib.gr_reduce(ctypes.byref(g), ctypes.byref(p), ctypes.byref(r),
                         None, 0, None) == -6


def test_package_does_not_reach_the_oracle():
    """The product path never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1812_08942_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
