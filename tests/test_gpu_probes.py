"""Measured-peak probes (curob_probe_read, curob_probe_mfma_bf16): argument checks, and rates
in the range an MI355X can reach (the nominal peaks are 8 TB/s HBM and 2.5 PFLOP/s dense
BF16; a probe can neither exceed them by much nor read as idle)."""
import ctypes
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_probes_report_plausible_peaks():
    import torch
    assert torch.cuda.is_available()
    import paper_1407_7737_amd as c
    c.initialize(10, 16, 0)
    try:
        x = torch.empty(1 << 26, dtype=torch.float32, device="cuda").fill_(1.0)  # 256 MiB
        gbs = c.probe_read_gbs(x, reps=5)
        tf = c.probe_mfma_bf16_tflops(reps=3)
        say(f"probe: read {gbs:.0f} GB/s, bf16 MFMA {tf:.0f} TFLOP/s")
        assert 1000.0 < gbs < 9000.0
        assert 200.0 < tf < 2800.0
        lib, out = c.lib, ctypes.c_double()
        assert lib.curob_probe_read(None, 16, 1, ctypes.byref(out)) == c.CUROB_E_ARG
        assert lib.curob_probe_read(ctypes.c_void_p(x.data_ptr()), 24, 1, ctypes.byref(out)) == c.CUROB_E_ARG
        assert lib.curob_probe_read(ctypes.c_void_p(x.data_ptr()), 16, 0, ctypes.byref(out)) == c.CUROB_E_ARG
        assert lib.curob_probe_mfma_bf16(0, ctypes.byref(out)) == c.CUROB_E_ARG
    finally:
        c.dispose()
