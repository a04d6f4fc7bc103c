"""C-ABI checks that need no GPU: the library loads, exports every symbol include/curob.h
declares, rejects misuse with the documented codes, and its host-side problem generator
agrees with the oracle's independent implementation."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "curob.h")


@pytest.fixture(scope="module")
def curob():
    import paper_1407_7737_amd as c
    return c


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_paper_interface():
    names = declared_functions()
    for n in ["initialize", "dispose", "func_evaluate", "func_evaluatef", "h_func_evaluate", "h_func_evaluatef"]:
        assert n in names


def test_every_declared_symbol_is_exported(curob):
    lib = ctypes.CDLL(curob._native.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(curob._native.EXPORTED)


def test_calls_before_initialize_report_state(curob):
    lib = curob.lib
    assert lib.func_evaluate(0, None, 0, None) == curob.CUROB_E_STATE
    assert lib.func_evaluatef(0, None, 10, None) == curob.CUROB_E_STATE
    assert lib.h_func_evaluate(0, None, 1, None) == curob.CUROB_E_STATE
    assert lib.curob_set_mode(0) == curob.CUROB_E_STATE
    out = ctypes.c_double()
    assert lib.curob_probe_read(None, 16, 1, ctypes.byref(out)) == curob.CUROB_E_STATE
    assert lib.curob_probe_mfma_bf16(1, ctypes.byref(out)) == curob.CUROB_E_STATE
    assert lib.dispose() == curob.CUROB_E_STATE
    assert "not initialised" in curob.last_error() or "nothing to dispose" in curob.last_error()


def test_initialize_argument_checks(curob):
    lib = curob.lib
    assert lib.initialize(1, 10, 0) == curob.CUROB_E_ARG
    assert lib.initialize(10, 0, 0) == curob.CUROB_E_ARG
    assert "max_concurrency" in curob.last_error()


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_initialize_without_device_fails_cleanly(curob):
    assert curob.lib.initialize(10, 10, 0) == curob.CUROB_E_HIP
    assert curob.last_error()


def test_generate_basic_argument_checks(curob):
    dp = ctypes.POINTER(ctypes.c_double)
    assert curob.lib.curob_generate_basic(23, 10, 0, None, None) == curob.CUROB_E_FID
    assert curob.lib.curob_generate_basic(0, 1, 0, None, None) == curob.CUROB_E_ARG


@pytest.mark.parametrize("fid,dim,seed", [(0, 2, 0), (11, 10, 0), (2, 30, 1), (19, 100, 7), (16, 128, 3),
                                          (10, 50, 0), (14, 1000, 0)])
def test_generator_agrees_with_the_oracle(curob, orc, fid, dim, seed):
    """Both sides implement SplitMix64 / polar normals / Fisher-Yates independently; the
    library orthonormalises with Householder QR, the oracle with CGS2."""
    o, R = curob.generate_basic(fid, dim, seed)
    p = orc.basic(fid, dim, seed)
    assert np.array_equal(o, p.shift())
    assert np.abs(R - p.rotation()).max() <= 1e-13


def test_batch_handle_checks(curob):
    assert curob.lib.curob_batch_destroy(None) == curob.CUROB_OK
