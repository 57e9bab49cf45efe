"""Batched generation (rsaw_gen_batch): every ensemble of a batch must give
exactly what a separate rsaw_gen_chains call gives, and what the oracle gives.

GPU tests; they call the HIP library through its C ABI (ctypes binding).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs
from paper_1704_04381_amd.workloads import mixed_ensembles

pytestmark = pytest.mark.gpu


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same_summary(a, b):
    for key in a:
        x, y = a[key], b[key]
        if isinstance(x, float) and math.isnan(x):
            assert math.isnan(y), key
        else:
            assert x == y, (key, x, y)


def _check_against_single(specs, per_chain=True):
    print(f"[gpu] batch of {len(specs)} ensembles", flush=True)
    res = rs.gen_batch(specs, per_chain=per_chain)
    torch.cuda.synchronize()
    for i, (sp, (out, s)) in enumerate(zip(specs, res)):
        sp = dict(sp)
        one_out, one_s = rs.gen_chains(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                                       sp.pop("seed"), per_chain=per_chain, **sp)
        torch.cuda.synchronize()
        a, b = _host(out), _host(one_out)
        assert a.keys() == b.keys()
        for key in a:
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"ensemble {i} {key}")
        _same_summary(s, one_s)
    return res


def test_mixed_batch_equals_single_calls_and_oracle():
    specs = [
        dict(geometry="lattice", N=16, k=6, n_chains=3_001, seed=5, coord="i32", exact_w=True),
        dict(geometry="lattice", N=64, k=6, n_chains=20_000, seed=6, coord="i16", hist_bins=256),
        dict(geometry="real", N=64, k=8, n_chains=2_000, seed=7, hist_bins=64),
        dict(geometry="lattice", N=5, k=6, n_chains=999, seed=8, coord="i16"),
        dict(geometry="lattice", N=100, k=6, n_chains=1_500, seed=9, coord="i32", hist_bins=32),
        dict(geometry="real", N=40, k=16, n_chains=700, seed=10),
        dict(geometry="lattice", N=1, k=6, n_chains=50, seed=11, coord="i32"),
        dict(geometry="lattice", N=33, k=6, n_chains=0, seed=12, coord="i32", hist_bins=8),
        dict(geometry="lattice", N=300, k=6, n_chains=300, seed=13, coord="i16"),
        dict(geometry="real", N=700, k=8, n_chains=20, seed=14, bead_diameter=0.8),
        dict(geometry="lattice", N=64, k=6, n_chains=777, seed=15, coord="i32"),
        dict(geometry="lattice", N=2_049, k=6, n_chains=40, seed=16, coord="i16"),
        dict(geometry="real", N=3, k=8, n_chains=64, seed=17),
    ]
    res = _check_against_single(specs)
    # oracle spot checks on a lattice and a hard-sphere ensemble of the batch
    out, s = res[4]
    ref = oracle.gen_lattice(9, 100, 1_500)
    np.testing.assert_array_equal(out["log_w"].cpu().numpy(), ref["log_w"])
    np.testing.assert_array_equal(out["n2rg2"].cpu().numpy(), ref["n2rg2"])
    out, s = res[2]
    ref = oracle.gen_real(7, 64, 8, 2_000)
    np.testing.assert_array_equal(out["r2"].cpu().numpy(), ref["r2"])
    np.testing.assert_array_equal(out["log_w"].cpu().numpy(), ref["log_w"])
    # the empty ensemble
    assert res[7][1]["n_chains"] == 0 and res[7][1]["n_alive"] == 0


def test_batch_of_the_mixed_workload_small():
    specs = mixed_ensembles(n=256, m_lo=2.0, m_span=1.5)
    _check_against_single(specs, per_chain=True)


def test_batch_without_per_chain_outputs_or_summaries():
    specs = mixed_ensembles(n=40, m_lo=2.0, m_span=2.0)
    _check_against_single(specs, per_chain=False)
    # no summaries at all: growth only, outputs still written
    cfgs = [rs.make_config(sp["geometry"], sp["N"], sp["k"], sp["n_chains"], sp["seed"],
                           coord=sp["coord"]) for sp in specs]
    outs, allocs = [], []
    for c in cfgs:
        out, o = rs._alloc_outputs(c, torch.device("cuda", 0), True, 0)
        outs.append(o)
        allocs.append(out)
    rs.gen_batch_raw(cfgs, outs, 0, None, None, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    res = rs.gen_batch(specs)
    for a, (b, _) in zip(allocs, res):
        np.testing.assert_array_equal(a["log_w"].cpu().numpy(), b["log_w"].cpu().numpy())


def test_consecutive_batches_reuse_the_staging_buffer():
    a = mixed_ensembles(n=64, meta_seed=3, m_lo=2.0, m_span=1.0)
    b = mixed_ensembles(n=200, meta_seed=4, m_lo=2.0, m_span=1.0)
    stream = torch.cuda.current_stream().cuda_stream
    r1 = rs.gen_batch(a, sync=False, stream=stream)
    r2 = rs.gen_batch(b, sync=False, stream=stream)
    r3 = rs.gen_batch(a, sync=False, stream=stream)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r1[1].cpu().numpy(), r3[1].cpu().numpy())
    for x, y in zip(r1[0], r3[0]):
        np.testing.assert_array_equal(x["log_w"].cpu().numpy(), y["log_w"].cpu().numpy())
    _check_against_single(b[:20])
