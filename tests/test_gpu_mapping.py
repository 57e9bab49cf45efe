"""Lane mappings of the group kernels and the autotuner (rsaw_mapping_set,
rsaw_autotune): every legal mapping must give per-chain outputs and
summaries bit-identical to the built-in rule's, and to the oracle's.

GPU tests; they call the HIP library through its C ABI (ctypes binding).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu

LANES = (2, 4, 8, 16, 32, 64)
THREADS = (64, 256)


@pytest.fixture(autouse=True)
def _clean_table():
    rs.mapping_clear()
    yield
    rs.mapping_clear()


def _run(geo, N, k, M, seed, **kw):
    out, s = rs.gen_chains(geo, N, k, M, seed, per_chain=True, **kw)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}, s


def _same(a, b, what):
    (oa, sa), (ob, sb) = a, b
    assert oa.keys() == ob.keys()
    for key in oa:
        np.testing.assert_array_equal(oa[key], ob[key], err_msg=f"{what} {key}")
    for key in sa:
        x, y = sa[key], sb[key]
        if isinstance(x, float) and math.isnan(x):
            assert math.isnan(y), (what, key)
        else:
            assert x == y, (what, key, x, y)


CASES = [
    ("lattice", 6, 65, 3_000, dict(coord="i16", hist_bins=64)),
    ("lattice", 6, 128, 2_000, dict(coord="i32")),
    ("lattice", 6, 129, 2_000, dict(coord="i16")),
    ("lattice", 6, 700, 600, dict(coord="i32", hist_bins=256)),
    ("real", 8, 3, 2_000, {}),
    ("real", 8, 64, 2_000, dict(hist_bins=32)),
    ("real", 8, 250, 400, {}),
    ("real", 16, 100, 500, dict(bead_diameter=0.9)),
    ("real", 5, 40, 700, {}),
    ("lattice26", 26, 65, 2_000, dict(coord="i16")),
    ("lattice26", 26, 256, 600, dict(coord="i32")),
    ("lattice26", 26, 400, 300, dict(coord="i16")),
    # 8 lanes hold at most N = 512 in registers: LDS byte words beside
    # register words of 16 to 64 lanes
    ("lattice26", 26, 600, 120, dict(coord="i32")),
]


@pytest.mark.parametrize("geo,k,N,M,kw", CASES, ids=[f"{c[0]}-k{c[1]}-N{c[2]}" for c in CASES])
def test_every_legal_mapping_is_bit_identical(geo, k, N, M, kw):
    seed = 1000 + N + k
    print(f"[gpu] mappings {geo} k={k} N={N} M={M}", flush=True)
    ref = _run(geo, N, k, M, seed, **kw)
    tried = 0
    for lanes in LANES:
        for threads in THREADS:
            try:
                rs.mapping_set(geo, k, N, N, lanes, threads)
            except rs.RsawError:
                continue
            m = rs.mapping_query(rs.make_config(geo, N, k, M, seed, **kw))
            assert (m["lanes"], m["threads"]) == (lanes, threads)
            _same(_run(geo, N, k, M, seed, **kw), ref, f"lanes {lanes} threads {threads}")
            rs.mapping_clear()
            tried += 1
    assert tried >= 3


def test_forced_mappings_match_the_oracle():
    rs.mapping_set("lattice", 6, 65, 200, 64, 64)
    out, _ = _run("lattice", 100, 6, 400, 21, coord="i32")
    ref = oracle.gen_lattice(21, 100, 400)
    for key in ("log_w", "r2", "n2rg2", "n_grown"):
        np.testing.assert_array_equal(out[key], ref[key], err_msg=key)
    rs.mapping_set("real", 8, 2, 200, 64, 64)
    out, _ = _run("real", 64, 8, 300, 22)
    ref = oracle.gen_real(22, 64, 8, 300)
    for key in ("log_w", "r2", "rg2", "n_grown"):
        np.testing.assert_array_equal(out[key], ref[key], err_msg=key)
    rs.mapping_set("lattice26", 26, 65, 200, 32, 256)
    out, _ = _run("lattice26", 150, 26, 300, 23, coord="i32")
    ref = oracle.gen_lattice(23, 150, 300, z26=True)
    for key in ("log_w", "r2", "n2rg2", "n_grown"):
        np.testing.assert_array_equal(out[key], ref[key], err_msg=key)


def test_batch_and_server_use_the_table():
    specs = [
        dict(geometry="lattice", N=100, k=6, n_chains=1_000, seed=31, coord="i16"),
        dict(geometry="real", N=64, k=8, n_chains=500, seed=32),
        dict(geometry="lattice26", N=200, k=26, n_chains=400, seed=33, coord="i32"),
        dict(geometry="lattice", N=40, k=6, n_chains=900, seed=34, coord="i16"),
    ]
    ref = rs.gen_batch(specs)
    torch.cuda.synchronize()
    ref = [({k: v.cpu().numpy() for k, v in o.items()}, s) for o, s in ref]
    rs.mapping_set("lattice", 6, 65, 128, 16, 64)
    rs.mapping_set("real", 8, 2, 100, 32, 256)
    rs.mapping_set("lattice26", 26, 161, 256, 64, 64)
    got = rs.gen_batch(specs)
    torch.cuda.synchronize()
    for i, ((o, s), r) in enumerate(zip(got, ref)):
        _same(({k: v.cpu().numpy() for k, v in o.items()}, s), r, f"ensemble {i}")
    with rs.Server(max_batch=4, streams=2) as srv:
        tickets = [srv.submit(**sp) for sp in specs]
        for t, (_, s) in zip(tickets, ref):
            r = srv.wait(t)
            for key in ("n_alive", "log_c_est", "r2_mean", "rg2_mean", "ess"):
                assert r[key] == s[key], key


@pytest.mark.parametrize("geo,k", [("lattice", 6), ("real", 8), ("lattice26", 26)])
def test_autotune_installs_legal_winners(geo, k):
    edges = [32, 128, 256] if geo != "real" else [16, 64, 200]
    M = 2_000
    before = [_run(geo, n, k, 500, 41) for n in (edges[0], edges[1] - 7, edges[2])]
    print(f"[gpu] autotune {geo} k={k} edges={edges}", flush=True)
    res = rs.autotune(geo, k, edges, M, reps=2)
    assert len(res) == 3
    lo = 1
    for b, r in enumerate(res):
        assert (r["n_lo"], r["n_hi"]) == (lo, edges[b])
        assert r["ms"] > 0.0
        lo = edges[b] + 1
        m = rs.mapping_query(rs.make_config(geo, edges[b], k, M, 1))
        assert (m["lanes"], m["threads"], m["lds_bytes"]) == (r["lanes"], r["threads"], r["lds_bytes"])
        if m["lanes"] > 1:
            assert r["lanes"] in LANES and r["threads"] in THREADS and r["lds_bytes"] <= 160 * 1024
    # results do not depend on the mapping
    after = [_run(geo, n, k, 500, 41) for n in (edges[0], edges[1] - 7, edges[2])]
    for a, b_ in zip(after, before):
        _same(a, b_, "after autotune")


def test_autotune_argument_errors():
    for edges, reps in (([64, 64], 1), ([0], 1), ([64], 0), ([64], 101)):
        with pytest.raises(rs.RsawError):
            rs.autotune("lattice", 6, edges, 100, reps=reps)
    assert rs.mapping_query(rs.make_config("lattice", 100, 6, 100, 1))["lanes"] == 2  # nothing installed


def test_hard_sphere_rule_window_matches_the_oracle():
    # k = 8, 144 <= N <= 213: the built-in rule takes 32 lanes in one-wave blocks
    # k = 16, 285 <= N <= 426: 64 lanes in one-wave blocks
    for N, k, M, seed, lanes in ((150, 8, 300, 51, 32), (213, 8, 200, 52, 32), (300, 16, 60, 53, 64)):
        m = rs.mapping_query(rs.make_config("real", N, k, M, seed))
        assert (m["lanes"], m["threads"]) == (lanes, 64)
        print(f"[gpu] hard-sphere rule window N={N} k={k}", flush=True)
        out, _ = _run("real", N, k, M, seed)
        ref = oracle.gen_real(seed, N, k, M)
        for key in ("log_w", "r2", "rg2", "n_grown"):
            np.testing.assert_array_equal(out[key], ref[key], err_msg=f"N={N} {key}")
