"""Achievable-peak micro-benchmarks (the denominators of measured roofline
fractions): every figure is finite, positive and below the device's published
peak (MI355X: float32 MFMA 157.3, bf16 2500, float64 78.6 TFLOP/s; HBM 8 TB/s,
a copy moving each byte twice counts both)."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_measure_peaks_plausible():
    from paper_2307_14123_amd import qmc
    p = qmc.measure_peaks(512 << 20)
    print(f"[peaks] {p}", flush=True)
    bounds = {"fp32_mfma": 157.3, "bf16_mfma": 2500.0, "fp64_mfma": 78.6, "copy": 8000.0}
    for k, hi in bounds.items():
        assert math.isfinite(p[k]) and 0.05 * hi < p[k] <= 1.02 * hi, (k, p[k])
