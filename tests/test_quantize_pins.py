"""Pins of the test-side bfloat16 / fp8-e4m3 rounding used to feed the oracle
the exact feature values the low-precision paths compute with (values fixed by
the formats: 8 significant bits for bfloat16; 4 for e4m3, exponent bias 7,
subnormal step 2^-9, largest finite 448)."""
import numpy as np

from helpers import bf16_round, e4m3_round


def test_bf16_round():
    u = 2.0 ** -8  # half an ulp at 1
    cases = {1.0: 1.0, 1 + u: 1.0, 1 + 3 * u: 1 + 4 * u, 1 + 2 * u: 1 + 2 * u, -(1 + 3 * u): -(1 + 4 * u),
             0.0: 0.0, 3.0: 3.0, 1 + 1.01 * u: 1 + 2 * u, 255.5: 256.0, 257.0: 256.0, 259.0: 260.0}
    for x, want in cases.items():
        assert bf16_round(np.float32(x)) == np.float32(want), x
    r = np.random.default_rng(0).normal(size=10000).astype(np.float32)
    q = bf16_round(r)
    assert np.all(q.view(np.uint32) & 0xFFFF == 0)             # representable in bfloat16
    assert np.all(np.abs(q - r) <= np.abs(r) * 2.0 ** -8 + 0)  # within half an ulp


def test_e4m3_round():
    cases = {1.0: 1.0, 448.0: 448.0, 460.0: 448.0, 1e4: 448.0, -1e4: -448.0, 2.0 ** -9: 2.0 ** -9,
             2.0 ** -10: 0.0, 3 * 2.0 ** -10: 2.0 ** -8, 17.0: 16.0, 19.0: 20.0, 1.0625: 1.0, 1.1875: 1.25,
             0.015: 2.0 ** -6, 0.3: 0.3125}
    for x, want in cases.items():
        assert e4m3_round(np.float32(x)) == np.float32(want), x
    # every value is one of the 253 finite e4m3 values
    grid = set()
    for e in range(1, 16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            grid.add((1 + m / 8) * 2.0 ** (e - 7))
    grid |= {m * 2.0 ** -9 for m in range(8)}
    r = np.random.default_rng(1).normal(scale=50.0, size=5000).astype(np.float32)
    assert all(abs(float(v)) in grid for v in e4m3_round(r))
