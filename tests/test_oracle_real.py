"""Pin the oracle's hard-sphere growth (paper Sec. 3.3.3, Algorithm 2, Eq. 3)
against things that do not come from the oracle:

* the Marsaglia unit vectors: |e| = 1 to rounding, e_z uniform on (-1, 1),
  isotropy, acceptance rate pi/4;
* closed forms: N = 2 (W = k), N = 3 (m_2 ~ Binomial(k, 3/4), weighted
  <R2> = 5/2, <Rg2> = 1/2, P(dead) = 4^-k), sigma = 0 (freely jointed chain:
  W = k^n, <R2> = n b^2, <Rg2> = b^2 (N^2 - 1) / (6 N));
* brute force: ideal chains from numpy's own generator (Gaussian directions),
  kept when no two non-bonded beads overlap, give the hard-sphere average of
  R^2 and the survival probability E[W] / k^n directly;
* the overlap boundary: touching spheres (d = sigma) do not overlap.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def test_unit_vectors():
    es, atts = [], []
    for c in range(400):
        for t in range(50):
            e, a = oracle.unit_vector(5, c, 1 + (t % 7), t)
            es.append(e); atts.append(a)
    E = np.array(es)
    n2 = (E * E).sum(axis=1)
    assert np.all(np.abs(n2 - 1.0) <= 8 * 2.0**-53)
    # Archimedes: each coordinate of a uniform point on the sphere is uniform on (-1, 1)
    for a in range(3):
        assert stats.kstest(E[:, a], "uniform", args=(-1, 2)).pvalue > 1e-4
    # isotropy of the second moments
    cov = E.T @ E / len(E)
    assert np.allclose(cov, np.eye(3) / 3, atol=0.01)
    # acceptance of the disc step is pi / 4: attempts are geometric
    atts = np.array(atts)
    p_hat = 1.0 / atts.mean()
    se = math.sqrt(p_hat * (1 - p_hat) / len(atts)) * 1.2
    assert abs(p_hat - math.pi / 4) < 5 * se


def test_overlap_boundary():
    s2 = 1.0
    assert not oracle.overlaps([0, 0, 0], [1, 0, 0], s2)       # touching
    assert not oracle.overlaps([0, 0, 0], [0, 0, -1], s2)
    assert oracle.overlaps([0, 0, 0], [1 - 2**-52, 0, 0], s2)   # just inside
    assert oracle.overlaps([0, 0, 0], [0.6, 0.6, 0.0], s2)      # d^2 = 0.72
    assert not oracle.overlaps([0, 0, 0], [0.6, 0.8, 0.1], s2)  # d^2 = 1.01


@pytest.mark.parametrize("k", [1, 8, 16])
def test_two_beads(k):
    o = oracle.gen_real(1, 2, k, 3000)
    assert np.all(o["n_grown"] == 2)
    assert np.all(o["log_w"] == math.log(k))
    assert np.all(np.abs(o["r2"] - 1.0) < 1e-15)


@pytest.mark.parametrize("k,seed", [(1, 31), (2, 32), (8, 33)])
def test_three_beads_closed_form(k, seed):
    M = 120_000
    o = oracle.gen_real(seed, 3, k, M)
    alive = o["n_grown"] == 3
    m2 = np.where(alive, np.rint(np.exp(o["log_w"]) / k), 0).astype(int)
    # m_2 is Binomial(k, 3/4): a trial is free iff e1.e2 >= -1/2
    obs = np.bincount(m2, minlength=k + 1)
    exp = stats.binom.pmf(np.arange(k + 1), k, 0.75) * M
    keep = exp >= 5
    assert stats.chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum()).pvalue > 1e-4
    if k <= 2:
        p_dead = 4.0**-k
        assert abs((~alive).mean() - p_dead) < 5 * math.sqrt(p_dead * (1 - p_dead) / M)
    W = np.where(alive, np.exp(o["log_w"]), 0.0)
    # E[W] = 3 k^2 / 4
    se = W.std() / math.sqrt(M)
    assert abs(W.mean() - 0.75 * k * k) < 5 * se
    for A, exact in ((o["r2"], 2.5), (o["rg2"], 0.5)):
        est = (W * A).sum() / W.sum()
        s = math.sqrt(((W * (A - est)) ** 2).sum()) / W.sum()
        assert abs(est - exact) < 5 * s, (est, exact, s)


@pytest.mark.parametrize("N,k,b", [(8, 4, 1.0), (24, 8, 1.5)])
def test_ideal_chain_sigma_zero(N, k, b):
    M = 40_000
    o = oracle.gen_real(17, N, k, M, b=b, sigma=0.0)
    n = N - 1
    assert np.all(o["n_grown"] == N)
    # log W = n_k log k: one product, rounded once (the count-based rule)
    assert np.all(o["log_w"] == float(n) * math.log(k))
    for A, exact in ((o["r2"], n * b * b), (o["rg2"], b * b * (N * N - 1) / (6 * N))):
        se = A.std() / math.sqrt(M)
        assert abs(A.mean() - exact) < 5 * se, (A.mean(), exact, se)


def _brute_force_hard_sphere(N, M, seed, sigma=1.0, b=1.0):
    """Ideal chains with Gaussian-normalised directions, kept if no
    non-bonded pair is closer than sigma."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((M, N - 1, 3))
    d *= b / np.linalg.norm(d, axis=2, keepdims=True)
    pos = np.concatenate([np.zeros((M, 1, 3)), np.cumsum(d, axis=1)], axis=1)
    ok = np.ones(M, bool)
    for i in range(N):
        for j in range(i + 2, N):
            dd = ((pos[:, i] - pos[:, j]) ** 2).sum(axis=1)
            ok &= dd >= sigma * sigma
    end = pos[:, -1]
    return ok, (end ** 2).sum(axis=1)


def test_hard_sphere_against_brute_force():
    N, k = 7, 8
    ok, r2 = _brute_force_hard_sphere(N, 400_000, 123)
    acc = ok.mean()
    r2_bf = r2[ok].mean()
    r2_bf_se = r2[ok].std() / math.sqrt(ok.sum())
    M = 150_000
    o = oracle.gen_real(77, N, k, M)
    W = np.where(o["n_grown"] == N, np.exp(o["log_w"]), 0.0)
    # E[W / k^n] is the probability that an ideal chain is self-avoiding
    surv = W / k ** (N - 1)
    se = math.hypot(surv.std() / math.sqrt(M), math.sqrt(acc * (1 - acc) / len(ok)))
    assert abs(surv.mean() - acc) < 5 * se, (surv.mean(), acc, se)
    est = (W * o["r2"]).sum() / W.sum()
    s = math.sqrt(((W * (o["r2"] - est)) ** 2).sum()) / W.sum()
    assert abs(est - r2_bf) < 5 * math.hypot(s, r2_bf_se), (est, r2_bf)


def test_chain_invariants_and_rg2():
    N, k = 32, 8
    for c in range(200):
        ch = oracle.real_chain(9, c, N, k)
        x = ch["xyz"]
        g = ch["n_grown"]
        assert np.all(x[0] == 0)
        bonds = np.linalg.norm(np.diff(x, axis=0), axis=1)
        assert np.all(np.abs(bonds - 1.0) < 1e-14)
        for i in range(g):
            for j in range(i + 2, g):
                dx = x[i] - x[j]
                d2 = dx[0] * dx[0] + dx[1] * dx[1]
                d2 = d2 + dx[2] * dx[2]
                assert d2 >= 1.0
        cm = x.mean(axis=0)
        rg2 = ((x - cm) ** 2).sum(axis=1).mean()
        assert abs(ch["rg2"] - rg2) < 1e-12 * rg2
        pair = sum(((x[i] - x[j]) ** 2).sum() for i in range(g) for j in range(i + 1, g))
        assert abs(ch["rg2"] - pair / g / g) < 1e-12 * rg2
        assert abs(ch["r2"] - (x[-1] ** 2).sum()) < 1e-13 * ch["r2"]
        assert np.all(ch["end"] == x[-1])
        assert 1 <= ch["m"][1] == k
        if g == N:
            assert abs(ch["log_w"] - sum(math.log(m) for m in ch["m"][1:])) < 1e-13 * N


def test_log_m_is_correctly_rounded():
    """log W sums log(m_i); each term must be ln(m) correctly rounded to
    binary64 (checked with 60-digit decimal arithmetic) so that any
    implementation using correctly rounded logarithms reproduces the bits."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    for k in range(1, 65):
        o = oracle.gen_real(1, 2, k, 1)
        assert o["log_w"][0] == float(Decimal(k).ln()), k
