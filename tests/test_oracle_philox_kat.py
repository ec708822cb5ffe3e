"""The oracle's Philox4x32-10 against the generator's published known-answer
vectors (tests/golden/philox4x32_10_kat.txt, Salmon et al. 2011): all four
output words of each block bit for bit.  A wrong rotation constant, round
count, key schedule or multiplier changes every word."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_vectors():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            assert len(w) == 10
            rows.append((w[0:4], w[4] | (w[5] << 32), w[6:10]))
    return rows


def test_kat_file_has_the_three_vectors():
    assert len(kat_vectors()) == 3


def test_oracle_philox_known_answers(orc):
    for ctr, seed, want in kat_vectors():
        got = orc.philox4x32_10(np.array(ctr, dtype=np.uint32), seed)
        assert [int(x) for x in got] == want, (ctr, hex(seed))
