"""Lane layouts of the matrix-core products the HGEMV leaf kernel relies on:
operand A[i][k] in lane i + 16 (k / kpl), B[k][j] in lane j + 16 (k / kpl);
the 16x16 result D[i][j] sits in lane j + 16 (i / 4), register i % 4 for the
f32 and bf16 products, and in lane j + 16 (i % 4), register i / 4 for f64."""
import numpy as np
import pytest

import paper_2003_10173_amd as h2
from paper_2003_10173_amd._lib import lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_mfma_result_layout(kind):
    out = np.zeros(256)
    h2.check(lib().h2_test_mfma_layout(kind, out.ctypes.data), "mfma probe")
    # which (i, j) each (lane, register) holds: D[i][j] = (i + 1) + 32 (j + 1)
    for lane in range(64):
        for reg in range(4):
            v = int(round(out[lane * 4 + reg]))
            got = (v % 32 - 1, v // 32 - 1)
            row = 4 * reg + lane // 16 if kind == 0 else 4 * (lane // 16) + reg
            assert got == (row, lane % 16), (kind, lane, reg, got)


def test_wave_sum_dpp():
    """The data-parallel wave reduction returns the same total to every lane,
    equal to the exact sum within the rounding of a 64-term sum."""
    import math
    g = np.random.default_rng(5)
    for scale in (1.0, 1e-300, 1e300):
        x = g.standard_normal(64) * np.exp(g.uniform(-5, 5, 64)) * scale
        out = np.zeros(64)
        h2.check(lib().h2_test_wave_sum(x.ctypes.data, out.ctypes.data), "wave sum")
        assert np.all(out == out[0])
        exact = math.fsum(x)
        assert abs(out[0] - exact) <= 64 * 2.0 ** -53 * np.abs(x).sum()
    x = np.zeros(64)
    x[63] = 1.5
    x[0] = -0.25
    out = np.zeros(64)
    h2.check(lib().h2_test_wave_sum(x.ctypes.data, out.ctypes.data), "wave sum")
    assert np.all(out == 1.25)
