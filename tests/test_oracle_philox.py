"""Pins for the oracle's Philox4x32-10 (counter-based generator of the sampler)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_known_answers_c_and_python():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(oracle.philox4x32_10(ctr, key)) == want
        assert oracle.philox_py(ctr, key) == want


def test_c_equals_python_on_random_blocks():
    rng = np.random.default_rng(7)
    for _ in range(500):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64)
        assert list(oracle.philox4x32_10(ctr, key)) == oracle.philox_py(ctr, key)


def test_stream_counter_layout_and_carry():
    seed = (0x1234ABCD << 32) | 0x0BADF00D
    first = 2 ** 32 - 3                       # low word wraps inside the stream
    out = oracle.philox_stream(first, 6, 5, 0, seed)
    for i in range(6):
        j = first + i
        want = oracle.philox_py([j & 0xFFFFFFFF, j >> 32, 5, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert list(out[i]) == want


def test_output_uniformity_chi_square():
    out = oracle.philox_stream(0, 40000, 0, 0, 0).reshape(-1)
    bins = np.bincount((out >> 28).astype(np.int64), minlength=16)
    exp = len(out) / 16
    chi2 = ((bins - exp) ** 2 / exp).sum()
    assert chi2 < 45.0                     # 15 dof, p ~ 1e-4
    bits = np.unpackbits(out.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.002
