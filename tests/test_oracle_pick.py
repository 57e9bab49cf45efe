"""Pin the uniform pick (Lemire's method on 16-bit words) used for the choice
among the m free candidates of a step (Eq. 3 requires each free candidate to
be chosen with probability 1/m)."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("m", list(range(1, 65)))
def test_lemire16_exactly_uniform_by_brute_force(m):
    """Over all 65536 words, every index in [0, m) is accepted equally often
    and the rejected words number exactly 2^16 mod m."""
    counts = np.zeros(m, dtype=np.int64)
    rejected = 0
    for x in range(65536):
        r = oracle.lemire16(x, m)
        if r is None:
            rejected += 1
        else:
            assert 0 <= r < m
            counts[r] += 1
    assert rejected == 65536 % m
    assert np.all(counts == (65536 - rejected) // m)


def _find_redraw(m, seed=1, max_chains=4000):
    for c in range(max_chains):
        for step in range(1, 64):
            idx, rej = oracle.pick(seed, c, step, m)
            if rej > 0:
                return c, step, idx, rej
    return None


@pytest.mark.parametrize("m", [3, 6])
def test_redraw_path(m):
    """The rejected primary word is replaced by the redraw stream of the same
    step: the result equals the first accepted half-word of (step, 0xFFFE, 0)."""
    hit = _find_redraw(m)
    assert hit is not None
    c, step, idx, rej = hit
    blk = oracle.philox([c, 0, step, 0xFFFE << 16], 1)
    halves = [int(blk[h >> 1]) >> (16 * (h & 1)) & 0xFFFF for h in range(8)]
    first = next(oracle.lemire16(h, m) for h in halves if oracle.lemire16(h, m) is not None)
    assert idx == first
