"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/cshydro.h declares, and rejects bad arguments before
touching the device.  Also checks the separation of the product and the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cshydro.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csh3?_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1210_5246_amd as csh
    L = csh.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in csh._SIGNATURES}
    assert set(names) == bound


def test_argument_validation_without_gpu():
    import paper_1210_5246_amd as csh
    L = csh.lib()
    h = ctypes.c_void_p()
    assert L.csh_init_state(ctypes.byref(h), 0, 1, 1.0, 1.0, 0, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert b"nx" in L.csh_last_error()
    assert L.csh_init_state(ctypes.byref(h), 4, 4, 1.0, 1.0, 7, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert L.csh_init_state(ctypes.byref(h), 4, 4, -1.0, 1.0, 0, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert L.csh_step(None, 0.1, None, None) == csh.CSH_ERR_ARG
    assert L.csh_run_cfl_states(None, 4, 0.8, None, None, None) == csh.CSH_ERR_ARG
    assert L.csh_fourier_amplitudes_noalloc(None, None, 0.0, 0.0, 1.0, 1.0, 4, None) == csh.CSH_ERR_ARG
    assert L.csh_batch_init(ctypes.byref(h), 0, None, 0, None, None, None) == csh.CSH_ERR_ARG
    assert L.csh_batch_status(None) == csh.CSH_ERR_ARG
    assert L.csh3_init_state(ctypes.byref(h), 4, 0, 4, 1.0, 1.0, 1.0, 0, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert b"nz" in L.csh3_last_error()
    assert L.csh3_init_state(ctypes.byref(h), 4, 4, 4, 1.0, 0.0, 1.0, 0, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert L.csh3_step(None, 0.1, None, None) == csh.CSH_ERR_ARG
    # the largest grids: one plane of the state must stay below 4 GiB (32-bit
    # offsets); the limit is checked before any device work
    assert L.csh_init_state(ctypes.byref(h), 1 << 15, 1 << 14, 1.0, 1.0, 0, 0, 0, None, None, None) == csh.CSH_ERR_ARG
    assert b"4 GiB" in L.csh_last_error()
    assert L.csh_init_state(ctypes.byref(h), 1 << 16, 1 << 14, 1.0, 1.0, 0, 0, 1, None, None, None) == csh.CSH_ERR_ARG
    assert b"4 GiB" in L.csh_last_error()
    # just below the limit the size passes and the missing buffers are reported
    assert L.csh_init_state(ctypes.byref(h), 1 << 15, 1 << 14, 1.0, 1.0, 0, 0, 1, None, None, None) == csh.CSH_ERR_ARG
    assert b"device pointers" in L.csh_last_error()
    assert L.csh3_init_state(ctypes.byref(h), 1024, 1024, 512, 1.0, 1.0, 1.0, 0, 0, 0, None, None, None) == \
        csh.CSH_ERR_ARG
    assert b"4 GiB" in L.csh3_last_error()


def _sources(folder, exts):
    for dp, _, fns in os.walk(os.path.join(ROOT, folder)):
        for fn in fns:
            if fn.endswith(exts):
                yield os.path.join(dp, fn)


def test_product_and_oracle_share_nothing():
    for f in _sources("paper_1210_5246_amd", (".py", ".hip", ".h", ".cpp")):
        txt = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
        assert "cshoracle" not in txt, f
    for f in _sources("oracle", (".py", ".c", ".h")):
        txt = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+paper_1210_5246_amd\b", txt, re.M), f
        assert not re.search(r"#include\s+\"csh_", txt), f
