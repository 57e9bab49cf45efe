"""26-neighbour lattice variant (the "z = 26" lattice space of Sec. 3.3.2):
candidates are all displacements in {-1, 0, 1}^3 but zero.

Pins: W = 26 * 25 exactly at n = 2; m_i recounted by brute force along
sampled chains; the mean Rosenbluth weight and the weighted R^2 and N^2 Rg^2
against a brute-force enumeration of all walks with n <= 4 (the Rosenbluth
identities E[W] = c_n and E[W A] = sum over walks of A)."""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import oracle

STEPS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def _enumerate(n):
    """c_n, sum of R^2 and sum of N^2 Rg^2 over all 26-neighbour SAWs of n steps."""
    c = s_r2 = s_nn = 0

    def rec(path, occ):
        nonlocal c, s_r2, s_nn
        if len(path) == n + 1:
            c += 1
            e = path[-1]
            s_r2 += e[0] ** 2 + e[1] ** 2 + e[2] ** 2
            g = len(path)
            sx = sum(p[0] for p in path); sy = sum(p[1] for p in path); sz = sum(p[2] for p in path)
            s2 = sum(p[0] ** 2 + p[1] ** 2 + p[2] ** 2 for p in path)
            s_nn += g * s2 - (sx * sx + sy * sy + sz * sz)
            return
        t = path[-1]
        for d in STEPS:
            q = (t[0] + d[0], t[1] + d[1], t[2] + d[2])
            if q not in occ:
                occ.add(q)
                path.append(q)
                rec(path, occ)
                path.pop()
                occ.remove(q)

    rec([(0, 0, 0)], {(0, 0, 0)})
    return c, s_r2, s_nn


def test_weight_is_constant_for_two_steps():
    out = oracle.gen_lattice(3, 3, 2_000, z26=True)
    assert np.all(out["w_exact"] == 26 * 25)
    assert np.all(out["log_w"] == math.log(25) + math.log(26))


def test_m_sequence_is_the_free_neighbour_count():
    for c in range(60):
        ch = oracle.lattice_chain(5, c, 40, z26=True)
        xyz = [tuple(int(v) for v in r) for r in ch["xyz"]]
        assert len(set(xyz)) == len(xyz)
        for i in range(1, ch["n_grown"]):
            t = xyz[i - 1]
            assert max(abs(xyz[i][a] - t[a]) for a in range(3)) == 1
            occ = set(xyz[:i])
            m = sum((t[0] + d[0], t[1] + d[1], t[2] + d[2]) not in occ for d in STEPS)
            assert m == ch["m"][i]


@pytest.mark.parametrize("n", [3, 4])
def test_rosenbluth_identities_against_enumeration(n):
    c, s_r2, s_nn = _enumerate(n)
    M = 200_000
    out = oracle.gen_lattice(7, n + 1, M, z26=True)
    w = out["w_exact"].astype(np.float64)
    assert np.all(out["w_exact_ok"] == 1)
    for est, vals, exact in ((w, w, c), (w * out["r2"], w * out["r2"], s_r2),
                             (w * out["n2rg2"], w * out["n2rg2"], s_nn)):
        assert abs(est.mean() - exact) < 4.5 * vals.std() / math.sqrt(M) + 1e-9 * exact, (n, exact)
