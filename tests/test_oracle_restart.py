"""Restart on a dead end (the paper's rule: the whole sequence is discarded
and growth starts again from the first step, Sec. 3.3.2 and 3.3.3).

Pins: attempt 0 is the attrition stream itself; a retried chain is a valid
complete walk whose m_i are the true free-neighbour counts; for hard spheres
at N = 3 the mean weight of restarted chains is E[W | alive] =
(3 k^2 / 4) / (1 - 4^-k)."""
from __future__ import annotations

import math

import numpy as np

import oracle

NEI = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_surviving_chains_are_the_attrition_chains():
    for c in range(400):
        a = oracle.lattice_chain(3, c, 64)
        b = oracle.lattice_chain(3, c, 64, restart=True)
        if a["n_grown"] == 64:
            assert b["rounds"] == 1
            assert b["log_w"] == a["log_w"] and b["n2rg2"] == a["n2rg2"]
            np.testing.assert_array_equal(a["xyz"], b["xyz"])


def test_retried_lattice_chains_are_valid_complete_walks():
    retried = 0
    for c in range(3000):
        a = oracle.lattice_chain(4, c, 64)
        if a["n_grown"] == 64:
            continue
        b = oracle.lattice_chain(4, c, 64, restart=True)
        retried += 1
        assert b["rounds"] >= 2 and b["n_grown"] == 64
        xyz = [tuple(int(v) for v in r) for r in b["xyz"]]
        assert len(set(xyz)) == 64
        lw = 0.0
        counts = [0] * 7
        for i in range(1, 64):
            d = np.abs(np.array(xyz[i]) - np.array(xyz[i - 1])).sum()
            assert d == 1
            occ = set(xyz[:i])
            m = sum((xyz[i - 1][0] + dx, xyz[i - 1][1] + dy, xyz[i - 1][2] + dz) not in occ
                    for dx, dy, dz in NEI)
            assert m == b["m"][i]
            counts[m] += 1
        for m in range(1, 7):
            lw = lw + counts[m] * math.log(m)
        assert abs(lw - b["log_w"]) <= 1e-12 * lw
    assert retried >= 3


def test_hard_sphere_restart_mean_weight_at_n3():
    k, M = 2, 200_000
    out = oracle.gen_real(5, 3, k, M, b=1.0, sigma=1.0, restart=True)
    assert np.all(out["n_grown"] == 3)
    w = np.exp(out["log_w"])
    exact = (3.0 * k * k / 4.0) / (1.0 - 4.0 ** -k)
    assert abs(w.mean() - exact) < 4.0 * w.std() / math.sqrt(M)
    # attrition keeps the dead chains at W = 0: mean 3 k^2 / 4
    att = oracle.gen_real(5, 3, k, M, b=1.0, sigma=1.0)
    wa = np.where(np.isfinite(att["log_w"]), np.exp(att["log_w"]), 0.0)
    assert abs(wa.mean() - 3.0 * k * k / 4.0) < 4.0 * wa.std() / math.sqrt(M)
