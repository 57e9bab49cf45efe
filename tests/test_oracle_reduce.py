"""Pin the oracle's ensemble reductions (paper Eq. 2 weighted average, Eq. 6
mean weight) against correctly rounded sums (math.fsum), exact rational
arithmetic (fractions) and hand-computed special cases."""
import math
from fractions import Fraction

import numpy as np

import oracle


def _rand_inputs(M, seed, dead_frac=0.1):
    rng = np.random.default_rng(seed)
    log_w = rng.normal(50.0, 3.0, M)
    log_w[rng.random(M) < dead_frac] = -np.inf
    r2 = rng.integers(0, 63 * 63 + 1, M).astype(np.float64)
    rg2 = rng.random(M) * 40
    ng = np.full(M, 64, np.int32)
    ng[np.isneginf(log_w)] = rng.integers(5, 64, int(np.isneginf(log_w).sum()))
    return log_w, r2, rg2, ng


def test_sums_against_fsum():
    M = 20000
    log_w, r2, rg2, ng = _rand_inputs(M, 1)
    red = oracle.reduce(64, log_w, r2, rg2, ng, bins=256)
    alive = np.isfinite(log_w)
    L = log_w[alive].max()
    assert red["log_w_max"] == L and red["alive"] == alive.sum() and red["M"] == M
    w = np.exp(log_w[alive] - L)
    a, g = r2[alive], rg2[alive]
    exact = dict(sum_w=math.fsum(w), sum_w2=math.fsum(w * w),
                 sum_w_r2=math.fsum(w * a), sum_w2_r2=math.fsum(w * w * a),
                 sum_w2_r2sq=math.fsum(w * w * a * a), sum_w_rg2=math.fsum(w * g),
                 sum_w2_rg2=math.fsum(w * w * g), sum_w2_rg2sq=math.fsum(w * w * g * g))
    for k, v in exact.items():
        assert abs(red[k] - v) <= 2e-16 * abs(v), k
    S0, S2 = exact["sum_w"], exact["sum_w2"]
    assert math.isclose(red["log_c_est"], L + math.log(S0 / M), rel_tol=1e-15)
    assert math.isclose(red["ess"], S0 * S0 / S2, rel_tol=1e-14)
    mr = exact["sum_w_r2"] / S0
    assert math.isclose(red["r2_mean"], mr, rel_tol=1e-15)
    # ratio-estimator error: sqrt(sum w^2 (A - mean)^2) / sum w
    se = math.sqrt(math.fsum((w * (a - mr)) ** 2)) / S0
    assert math.isclose(red["r2_err"], se, rel_tol=1e-8)
    c_err = math.sqrt((M * S2 / S0**2 - 1) / (M - 1))
    assert math.isclose(red["c_rel_err"], c_err, rel_tol=1e-12)
    assert red["steps"] == float((ng - 1).sum())


def test_histogram_bins_exact():
    M = 5000
    log_w, r2, rg2, ng = _rand_inputs(M, 2)
    N, B = 64, 256
    red = oracle.reduce(N, log_w, r2, rg2, ng, bins=B)
    alive = np.isfinite(log_w)
    L = log_w[alive].max()
    n2 = (N - 1) ** 2
    hw = [[] for _ in range(B)]
    hn = [0] * B
    for lw, a in zip(log_w[alive], r2[alive]):
        b = int(Fraction(int(a) * B, n2 + 1))  # floor of the exact ratio
        hw[b].append(math.exp(lw - L))
        hn[b] += 1
    assert list(red["hist_n"]) == hn
    for b in range(B):
        v = math.fsum(hw[b])
        assert abs(red["hist_w"][b] - v) <= 2e-16 * max(v, 1e-300) * 4
    assert math.isclose(red["hist_w"].sum(), red["sum_w"], rel_tol=1e-13)


def test_special_cases():
    # equal weights: weighted averages are plain means, ESS = alive, c = e^L
    lw = np.full(10, 3.0)
    r2 = np.arange(10.0)
    red = oracle.reduce(5, lw, r2, r2 / 2, np.full(10, 5, np.int32))
    assert red["r2_mean"] == 4.5 and red["rg2_mean"] == 2.25
    assert red["ess"] == 10.0 and red["log_c_est"] == 3.0
    # all dead: no estimate
    red = oracle.reduce(5, np.full(4, -np.inf), np.ones(4), np.ones(4), np.full(4, 3, np.int32))
    assert red["alive"] == 0 and red["log_c_est"] == -np.inf and math.isnan(red["r2_mean"])
    # one live chain among M: c estimate = W / M
    lw = np.array([-np.inf, math.log(600.0), -np.inf, -np.inf])
    red = oracle.reduce(5, lw, np.ones(4), np.ones(4), np.array([3, 5, 4, 2], np.int32))
    assert math.isclose(math.exp(red["log_c_est"]), 150.0, rel_tol=1e-15)


def test_exact_integer_sums():
    rng = np.random.default_rng(4)
    w = rng.integers(0, 2**63, 3000, dtype=np.uint64)
    r2 = rng.integers(0, 2**20, 3000).astype(np.int64)
    nn = rng.integers(0, 2**40, 3000).astype(np.int64)
    got = oracle.reduce_exact(w, r2, nn)
    W = [int(x) for x in w]
    assert got["sum_w"] == sum(W)
    assert got["sum_w_r2"] == sum(a * int(b) for a, b in zip(W, r2))
    assert got["sum_w_n2rg2"] == sum(a * int(b) for a, b in zip(W, nn))
