"""Pin the oracle's lattice growth (paper Sec. 3.3.2, Algorithm 1, Eq. 3)
against things that do not come from the oracle:

* exact enumeration of all self-avoiding walks (brute force, tests/pins):
  the law of the Rosenbluth weight W, E[W] = c_n (Eq. 6), and the exact
  W-weighted <R^2> and <Rg^2> (the uniform averages over SAWs);
* closed forms for short chains (W is constant for n <= 3);
* geometric invariants recomputed from the coordinates (unit bonds, no site
  visited twice, m_i equal to the free neighbours of the tip, the end-to-end
  parity, g^2 Rg^2 equal to the pair sum), and uniformity of the pick.
"""
import math
from collections import Counter

import numpy as np
import pytest
from scipy import stats

import oracle

NEIGH = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def _chi2_pvalue(observed, expected_p, n):
    """Chi-square goodness of fit, bins with expectation < 5 merged."""
    keys = sorted(expected_p, key=lambda k: expected_p[k])
    obs, exp, acc_o, acc_e = [], [], 0, 0.0
    for k in keys:
        acc_o += observed.get(k, 0)
        acc_e += expected_p[k] * n
        if acc_e >= 5:
            obs.append(acc_o); exp.append(acc_e); acc_o, acc_e = 0, 0.0
    if acc_e > 0:
        obs[-1] += acc_o; exp[-1] += acc_e
    extra = sum(v for k, v in observed.items() if k not in expected_p)
    assert extra == 0, "weights outside the exact support"
    stat = sum((o - e) ** 2 / e for o, e in zip(obs, exp))
    return stats.chi2.sf(stat, len(obs) - 1)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_constant_weight_short_chains(N):
    """For n <= 3 steps no walk can block its own tip: W = 6 * 5^(n-1)."""
    n = N - 1
    o = oracle.gen_lattice(7, N, 5000)
    want = 1 if n == 0 else 6 * 5 ** (n - 1)
    assert np.all(o["w_exact"] == want)
    assert np.all(o["n_grown"] == N)
    assert np.allclose(o["log_w"], math.log(want), rtol=0, atol=4e-15 * max(1, n))


@pytest.mark.parametrize("n,seed", [(4, 11), (5, 12), (6, 13), (8, 14), (10, 15)])
def test_weight_law_matches_enumeration(saw_enum, n, seed):
    """Sampled W follows the exact law P(W = w) = #{SAW with weight w} / w."""
    ex = saw_enum(n)
    M = 200_000
    o = oracle.gen_lattice(seed, n + 1, M)
    p = {w: cnt / w for w, cnt in ex["w_hist"].items()}
    attr = 1.0 - sum(p.values())
    assert abs(attr) < 1e-12  # no trapped walk exists for these n
    assert not ex["traps"]
    obs = Counter(int(w) for w in o["w_exact"])
    assert _chi2_pvalue(obs, p, M) > 1e-4


@pytest.mark.parametrize("n,seed", [(6, 21), (9, 22), (11, 23)])
def test_estimators_match_enumeration(saw_enum, n, seed):
    """Eq. (6): mean W estimates c_n; Eq. (2): W-weighted <R2>, <Rg2> are the
    plain averages over all self-avoiding walks."""
    ex = saw_enum(n)
    N = n + 1
    M = 300_000
    o = oracle.gen_lattice(seed, N, M)
    W = o["w_exact"].astype(np.float64)
    ew2 = sum(cnt * w for w, cnt in ex["w_hist"].items())  # E[W^2] = sum_SAW W
    c = ex["c"]
    z = (W.mean() - c) / math.sqrt((ew2 - c * c) / M)
    assert abs(z) < 4.5, z
    for A, exact in ((o["r2"].astype(np.float64), ex["sum_r2"] / c),
                     (o["n2rg2"].astype(np.float64) / N**2, ex["sum_n2rg2"] / c / N**2)):
        est = (W * A).sum() / W.sum()
        se = math.sqrt(((W * (A - est)) ** 2).sum()) / W.sum()
        assert abs(est - exact) < 4.5 * se, (est, exact, se)
    # the oracle's own reduction agrees with the direct sums
    red = oracle.reduce(N, o["log_w"], o["r2"], o["rg2"], o["n_grown"])
    assert math.isclose(math.exp(red["log_c_est"]), W.mean(), rel_tol=1e-12)
    ex_sums = oracle.reduce_exact(o["w_exact"], o["r2"], o["n2rg2"])
    assert ex_sums["sum_w"] == int(o["w_exact"].astype(object).sum())


def _neighbours(p):
    return [(p[0] + d[0], p[1] + d[1], p[2] + d[2]) for d in NEIGH]


@pytest.mark.parametrize("N,seed,count", [(16, 1, 1500), (64, 5, 1200)])
def test_chain_invariants(N, seed, count):
    picks = Counter()
    dead = 0
    for c in range(count):
        ch = oracle.lattice_chain(seed, c, N)
        xyz = [tuple(int(v) for v in r) for r in ch["xyz"]]
        g = ch["n_grown"]
        assert len(xyz) == g and xyz[0] == (0, 0, 0)
        assert len(set(xyz)) == g, "site visited twice"
        occupied = {xyz[0]}
        w = 1
        for i in range(1, g):
            assert sum(abs(a - b) for a, b in zip(xyz[i], xyz[i - 1])) == 1
            free = [q for q in _neighbours(xyz[i - 1]) if q not in occupied]
            assert ch["m"][i] == len(free)
            assert xyz[i] in free
            picks[(len(free), free.index(xyz[i]))] += 1
            w *= len(free)
            occupied.add(xyz[i])
        if g < N:
            dead += 1
            assert ch["m"][g] == 0
            assert all(q in occupied for q in _neighbours(xyz[-1]))
            assert ch["log_w"] == -math.inf and ch["w_exact"] == 0
        else:
            if N <= 28:
                assert ch["w_exact_ok"] and ch["w_exact"] == w
            # log W against the exact integer W (Python computes log of the big int)
            assert abs(ch["log_w"] - math.log(w)) <= 1e-15 * N * math.log(w)
            r2 = sum(v * v for v in xyz[-1])
            assert r2 % 2 == (N - 1) % 2  # cubic lattice is bipartite
        assert ch["r2"] == sum(v * v for v in xyz[-1])
        assert tuple(ch["end"]) == xyz[-1]
        pair = sum(sum((a - b) ** 2 for a, b in zip(xyz[i], xyz[j]))
                   for i in range(g) for j in range(i + 1, g))
        assert ch["n2rg2"] == pair
        assert ch["rg2"] == pair / (g * g)
    # the pick among the m free candidates is uniform, for every m
    assert all(r == 0 for (m, r) in picks if m == 1)
    for m in range(2, 7):
        obs = [picks[(m, r)] for r in range(m)]
        if sum(obs) < 50 * m:
            continue
        assert stats.chisquare(obs).pvalue > 1e-4, (m, obs)


def test_batch_matches_single_chain_and_offsets():
    o = oracle.gen_lattice(99, 40, 300, chain_offset=1000)
    for c in (0, 17, 299):
        ch = oracle.lattice_chain(99, 1000 + c, 40)
        assert o["log_w"][c] == ch["log_w"]
        assert o["n_grown"][c] == ch["n_grown"]
        assert tuple(o["r_end"][:, c]) == tuple(ch["end"])
        assert o["n2rg2"][c] == ch["n2rg2"]
    a = oracle.gen_lattice(99, 40, 200, chain_offset=1000)
    b = oracle.gen_lattice(99, 40, 100, chain_offset=1200)
    assert np.array_equal(np.concatenate([a["log_w"], b["log_w"]]), o["log_w"])


def test_dead_chains_exist_and_are_attrited():
    """Long chains get trapped; a trapped chain keeps weight 0 and counts in M."""
    o = oracle.gen_lattice(3, 128, 3000)
    dead = o["n_grown"] < 128
    assert dead.sum() > 0
    assert np.all(np.isneginf(o["log_w"][dead]))
    assert np.all(o["w_exact"][dead] == 0)
    assert np.all(np.isfinite(o["log_w"][~dead]))
    red = oracle.reduce(128, o["log_w"], o["r2"], o["rg2"], o["n_grown"])
    assert red["alive"] == int((~dead).sum()) and red["M"] == 3000


def test_cubic_symmetry_of_end_vector():
    o = oracle.gen_lattice(8, 32, 60_000)
    w = np.exp(o["log_w"] - o["log_w"].max())
    comps = [(w * o["r_end"][a].astype(float) ** 2).sum() / w.sum() for a in range(3)]
    means = [(w * o["r_end"][a]).sum() / w.sum() for a in range(3)]
    tot = sum(comps)
    for c in comps:
        assert abs(c - tot / 3) < 0.03 * tot / 3
    for m in means:
        assert abs(m) < 0.15
