"""Pin the oracle's Philox4x32-10 to an independent implementation.

The independent implementation is PyTorch's header-only ``at::philox_engine``
(ATen/core/PhiloxRNGEngine.h), compiled here with g++ for the host.  Its
state maps to ours as key = (seed lo, seed hi), counter = (offset lo,
offset hi, subsequence lo, subsequence hi); its first four outputs are the
four words of one Philox4x32-10 block.
"""
import numpy as np
import pytest

import oracle

def test_philox_matches_torch_engine(torch_philox):
    rng = np.random.default_rng(12345)
    rows = rng.integers(0, 2 ** 32, size=(400, 6), dtype=np.uint64)
    # edge words: zero, all-ones and the counter layouts the sweep uses
    rows[0] = [0, 0, 0, 0, 0, 0]
    rows[1] = [2 ** 32 - 1] * 6
    rows[2] = [1, 0, 5, 0, 2 * 17 + 1, 0]
    rows[3] = [7, 0, 123, 0, 44, 1 | (3 << 8)]
    ref = torch_philox(rows.tolist())
    for row, want in zip(rows, ref):
        key = [int(row[0]), int(row[1])]
        ctr = [int(row[2]), int(row[3]), int(row[4]), int(row[5])]
        got = oracle.philox4x32_10(ctr, key)
        assert got.astype(np.uint64).tolist() == want.tolist(), (key, ctr)


def test_philox_output_bits_are_balanced():
    # 4096 blocks -> 524288 bits; each output word bit should be ~1/2.
    ones = np.zeros(32)
    n = 0
    for i in range(1024):
        out = oracle.philox4x32_10([i, 0, 0, 0], [1, 0])
        for w in out:
            ones += (int(w) >> np.arange(32)) & 1
            n += 1
    frac = ones / n
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
