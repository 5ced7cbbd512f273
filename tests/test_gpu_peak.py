"""Measured device peaks (ibf_measure_peak), used by bench.py for the
roofline fraction against this device: both are positive and below twice
the published MI355X figures (8 TB/s HBM, 157.3 TFLOP/s dense FP32)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1605_03616_amd import ibf
    print("[gpu-case] measured peaks", flush=True)
    sys.stdout.flush()
    hbm = ibf.measure_peak(ibf.PEAK_HBM_COPY)
    mfma = ibf.measure_peak(ibf.PEAK_MFMA_F32)
    print(f"[gpu-case] copy {hbm:.1f} GB/s, fp32 4x4x1 MFMA {mfma:.2f} TFLOP/s", flush=True)
    assert 0 < hbm < 16000
    assert 0 < mfma < 2 * 157.3
    with pytest.raises(ibf.IBFError):
        ibf.measure_peak(7)
