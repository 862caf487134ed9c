"""CPU checks of the C ABI library: it loads and exports every declared symbol.

No compute call is made here (there is no GPU in the CPU test run).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ldpc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    from paper_1702_07740_amd import ldpc
    assert set(_declared_functions()) == set(ldpc.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1702_07740_amd import ldpc
    if not os.path.exists(ldpc.LIB_PATH):
        pytest.skip("libldpc.so not built")
    lib = ctypes.CDLL(ldpc.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_opts_defaults():
    from paper_1702_07740_amd import ldpc
    if not os.path.exists(ldpc.LIB_PATH):
        pytest.skip("libldpc.so not built")
    lib = ldpc.load()
    assert lib.ldpc_status_string(0) == b"ok"
    assert lib.ldpc_status_string(-5).startswith(b"workspace")
    o = ldpc.DecodeOpts()
    o.schedule, o.streams, o.graphs = 7, 7, 7   # the last fields: init must reach them
    lib.ldpc_decode_opts_init(ctypes.byref(o))
    assert (o.early_stop, o.check_from_iter, o.msg_fp16, o.checks_per_thread, o.llr_out) == (1, 0, 0, 0, None)
    assert not o.timing_events and o.n_timing_events == 0
    assert (o.schedule, o.streams, o.graphs) == (0, 0, 0)
    # host-only argument checks fail before any device call
    h = ctypes.c_void_p()
    assert lib.ldpc_code_create(1, 1, None, 4, ctypes.byref(h)) == ldpc.LDPC_EINVAL
    assert lib.ldpc_decode_batch(None, 1, None, None, 1, None, None, None, None, None, 0,
                                 None) == ldpc.LDPC_EINVAL
    assert b"null" in lib.ldpc_last_error()
    assert lib.ldpc_workspace_bytes(None, 1, 1, None) == 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1702_07740_amd import ldpc
    with pytest.raises(RuntimeError):
        ldpc._lib_saved = ldpc._lib
        try:
            ldpc._lib = None
            ldpc.load(str(tmp_path / "missing.so"))
        finally:
            ldpc._lib = ldpc._lib_saved
