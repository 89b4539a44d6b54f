"""The C-ABI library on the host, without a GPU: it loads, its dynamic
symbol table exports every entry point that include/lbmswim.h declares, the
binding's symbol list and struct layouts match the header, and entry points
that check their arguments before any device work reject null or invalid
ones with LBM_E_ARG."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1108_0786_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmswim.h")


def _declared():
    """Names of the functions the header declares (comments stripped)."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi._LIB_PATH):       # nothing built yet: build it (hipcc needs no GPU)
        from paper_1108_0786_amd import build
        build.build()
    return _abi.load()


def test_header_declares_the_entry_points():
    names = _declared()
    assert len(names) >= 25
    for name in ("lbm_init", "lbm_init_batch", "lbm_step", "lbm_body_forces", "lbm_adjoint", "lbm_vacuum_run"):
        assert name in names


def test_binding_lists_every_declared_entry_point():
    assert sorted(_abi.SYMBOLS) == _declared()


def test_library_exports_every_declared_entry_point(lib):
    for name in _declared():
        assert getattr(lib, name) is not None
    out = subprocess.run(["nm", "-D", "--defined-only", _abi._LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if line.split()[-2:-1] == ["T"]}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_struct_layouts_match_the_binding(lib):
    sizes = (C.c_int64 * 4)()
    assert lib.lbm_struct_sizes(sizes) == _abi.LBM_OK
    assert list(sizes) == [C.sizeof(_abi.LbmParams), C.sizeof(_abi.LbmBody), C.sizeof(_abi.LbmSpring),
                           C.sizeof(_abi.LbmDrive)]


def test_null_and_invalid_arguments_are_rejected_on_the_host(lib):
    E = _abi.LBM_E_ARG
    ctx = C.c_void_p()
    assert lib.lbm_init(None, C.byref(ctx)) == E
    assert lib.lbm_init_batch(None, 0, C.byref(ctx)) == E
    assert not ctx
    assert lib.lbm_step(None, 1) == E
    assert lib.lbm_status(None) == E
    assert lib.lbm_tune(None, _abi.TUNE["block"], 256) == E
    n = C.c_int64()
    assert lib.lbm_step_count(None, 0, C.byref(n)) == E
    assert lib.lbm_flow_average_begin(None, 0, 1) == E
    assert lib.lbm_last_error(None) == b"null context"
    lib.lbm_destroy(None)
    assert lib.lbm_vacuum_run(None, 3, None, 0, None, 0, 1, 10, None, 0, None, None) == E
    assert lib.lbm_copy_kernel(None, None, 16, 0, 0, None) == E
    # measurement aids: pointers are checked first, then sizes (no launch happens)
    assert lib.lbm_stream_copy(None, None, 16, 16, 4, 0, None) == E
    fake = C.c_void_p(16)     # never dereferenced: every call below fails its size check
    assert lib.lbm_copy_kernel(fake, fake, 15, 0, 0, None) == E
    assert lib.lbm_stream_copy(fake, fake, 0, 16, 4, 0, None) == E
    assert lib.lbm_stream_copy(fake, fake, 32, 16, 4, 0, None) == E
    assert lib.lbm_stream_copy(fake, fake, 16, 16, 3, 0, None) == E
    assert lib.lbm_stream_copy(fake, fake, 16, 1 << 62, 8, 0, None) == E
