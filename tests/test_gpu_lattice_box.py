"""Boxed byte words of the long-chain lattice kernels against the oracle.

Beyond N = 128 the simple cubic group kernels keep one byte per coordinate
up to N = 2048, and to N = 4096 in the group's registers (LDS holds them
for mappings whose lanes cannot hold a plane), and regrow, in two-word format in LDS, any chain
whose tip reaches |coordinate| = edge (rsaw_set_byte_box; 127 by default,
when no sampled chain of these sizes gets there).  Lowering the edge sends
many chains of every block through that regrowth, including blocks with
more such chains than fit in one pass of the block's LDS and, at edge 1,
every chain.  Every per-chain output and the summaries must still match
the oracle bit for bit (Sec. 3.3.2; the oracle knows nothing of word
formats).  The 26-neighbour group kernel keeps byte words up to N = 640 in
a box of |coordinate| <= 61 and packed words up to N = 4096 in a box of
253, and regrows the same way.  GPU test; calls the HIP library through
its C ABI.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs
from test_gpu_parity import _check_summary, _lattice_case

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _restore():
    yield
    rs.set_byte_box(0)
    rs.mapping_clear()


@pytest.mark.parametrize("N,M,seed,coord,edge,mapping,offset,restart", [
    # 4 lanes per chain, 256-thread blocks; at edge 20 most chains of N = 200
    # are regrown, more than one pass of the block's LDS holds
    (200, 1_500, 71, "i16", 20, None, 0, False),
    (256, 1_000, 72, "i32", 40, None, 0, False),
    # every chain regrown from step 1
    (129, 800, 75, "i16", 1, None, 0, False),
    # 8 lanes per chain (byte words up to N = 512)
    (300, 600, 73, "i16", 30, None, 0, False),
    (512, 300, 74, "i32", 40, None, 0, False),
    # dead ends restarted, and regrown chains among them
    (400, 500, 76, "i32", 25, None, 0, True),
    # other legal mappings: 8 lanes in one-wave blocks (registers), 4 lanes
    # in one-wave blocks (N > 256: byte words in LDS)
    (200, 700, 77, "i16", 20, (8, 64), 0, False),
    (300, 500, 78, "i32", 30, (4, 64), 0, False),
    # chain offset past 2^32
    (256, 900, 79, "i16", 30, None, (1 << 32) + 5, False),
    # beyond N = 512 the regrowth runs with 32 lanes per chain
    (1_000, 60, 85, "i16", 30, None, 0, False),
    (700, 120, 87, "i32", 1, None, 0, False),
    (2_048, 24, 86, "i32", 40, None, 0, False),
    (1_500, 40, 88, "i16", 35, None, 0, True),
    # 64 lanes per chain (registers up to N = 4096), one chain per wave; at
    # the production edge, chain 5 of seed 1 (N = 4096) reaches x = -134
    (3_000, 12, 110, "i32", 60, None, 0, False),
    (4_096, 8, 1, "i16", 127, None, 0, False),
    # one chain per 64-thread block: byte words with room for one regrown
    # chain up to N = 768, wide words beyond
    (600, 40, 89, "i32", 20, (64, 64), 0, False),
    (1_000, 30, 90, "i16", 30, (64, 64), 0, False),
])
def test_regrown_chains_bit_exact(N, M, seed, coord, edge, mapping, offset, restart):
    rs.set_byte_box(edge)
    if mapping:
        rs.mapping_set("lattice", 6, N, N, *mapping)
        q = rs.mapping_query(rs.make_config("lattice", N, 6, M, seed))
        assert (q["lanes"], q["threads"]) == mapping
    out, _ = _lattice_case(N, M, seed, coord=coord, bins=64, offset=offset, restart=restart)
    # the edge was reached by many chains (end vectors alone show some); at
    # the production edge the case names its chain
    assert edge == 127 or (np.abs(out["r_end"].astype(np.int64)).max(axis=0) >= edge).sum() > 0


def test_regrown_chains_in_a_batch():
    rs.set_byte_box(24)
    specs = [dict(geometry="lattice", N=200, k=6, n_chains=700, seed=81),
             dict(geometry="lattice", N=300, k=6, n_chains=400, seed=82, coord="i16"),
             dict(geometry="lattice", N=600, k=6, n_chains=100, seed=83),
             dict(geometry="lattice", N=129, k=6, n_chains=333, seed=84, restart=True)]
    print("[gpu] boxed batch", flush=True)
    res = rs.gen_batch(specs)
    torch.cuda.synchronize()
    for sp, (out, s) in zip(specs, res):
        ref = oracle.gen_lattice(sp["seed"], sp["N"], sp["n_chains"], restart=sp.get("restart", False))
        np.testing.assert_array_equal(out["n_grown"].cpu().numpy().view(np.uint16), ref["n_grown"])
        np.testing.assert_array_equal(out["log_w"].cpu().numpy(), ref["log_w"])
        np.testing.assert_array_equal(out["r_end"].cpu().numpy().astype(np.int32), ref["r_end"])
        np.testing.assert_array_equal(out["n2rg2"].cpu().numpy(), ref["n2rg2"])
        red = oracle.reduce(sp["N"], ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"])
        _check_summary(s, red, sp["n_chains"])


# 26-neighbour lattice: byte words (x, y, z + 64, plus 128) in the group
# kernel up to N = 640, packed 11/11/10-bit words up to N = 4096 (in the
# group's registers where its lanes hold the chain, else in LDS); a chain
# whose tip reaches |coordinate| = the edge (62 or 254, lowered by the
# knob) is regrown in two-word format by its block.
@pytest.mark.parametrize("N,M,seed,coord,edge,mapping,offset,restart", [
    (200, 800, 91, "i16", 20, None, 0, False),
    # 2 lanes per chain (N <= 128, registers only), with restarts
    (100, 600, 112, "i16", 20, None, 0, True),
    # 4 lanes per chain (8-bit n_m fields), every chain regrown from step 1
    (129, 600, 92, "i32", 1, None, 0, False),
    (300, 300, 93, "i16", 25, None, 0, True),
    (384, 200, 94, "i32", 30, None, 0, False),
    (640, 60, 95, "i16", 40, None, 0, False),
    # the production edge: chain 11031 of seed 1 (N = 256) reaches x = 63
    (256, 300, 1, "i16", 127, None, 11_000, False),
    # four chains per one-wave block; one chain per block
    (200, 300, 96, "i32", 20, (16, 64), 0, False),
    (200, 300, 97, "i16", 20, (64, 64), 0, False),
    # packed 11/11/10-bit words (640 < N <= 4096), regrown with 32 lanes per
    # chain; one chain per 64-thread block
    (700, 80, 102, "i16", 30, None, 0, False),
    (1_000, 40, 103, "i32", 40, None, 0, True),
    (2_048, 16, 104, "i16", 60, None, (1 << 32) + 5, False),
    (4_096, 4, 105, "i32", 100, None, 0, False),
    (1_000, 30, 106, "i32", 40, (64, 64), 0, False),
    (900, 24, 107, "i16", 0, None, 0, False),
    # words in LDS: mappings whose lanes cannot hold the chain (N > 64 G),
    # byte words with 8 lanes, packed words with 16
    (600, 60, 108, "i32", 30, (8, 256), 0, False),
    (1_100, 20, 109, "i16", 40, (16, 256), 0, True),
])
def test_lattice26_regrown_chains_bit_exact(N, M, seed, coord, edge, mapping, offset, restart):
    from test_gpu_lattice26 import _case
    rs.set_byte_box(edge)
    if mapping:
        rs.mapping_set("lattice26", 26, N, N, *mapping)
        q = rs.mapping_query(rs.make_config("lattice26", N, 26, M, seed))
        assert (q["lanes"], q["threads"]) == mapping
    out, _ = _case(N, M, seed, coord=coord, bins=64, offset=offset, restart=restart)
    reach = np.abs(out["r_end"].astype(np.int64)).max(axis=0)
    assert edge in (0, 127) or (reach >= min(edge, 62)).sum() > 0 or offset


def test_lattice26_regrown_chains_in_a_batch():
    rs.set_byte_box(20)
    specs = [dict(geometry="lattice26", N=200, k=26, n_chains=500, seed=98),
             dict(geometry="lattice", N=300, k=6, n_chains=300, seed=99, coord="i16"),
             dict(geometry="lattice26", N=150, k=26, n_chains=300, seed=100, coord="i16")]
    print("[gpu] boxed z26 batch", flush=True)
    res = rs.gen_batch(specs)
    torch.cuda.synchronize()
    for sp, (out, s) in zip(specs, res):
        z26 = sp["geometry"] == "lattice26"
        ref = oracle.gen_lattice(sp["seed"], sp["N"], sp["n_chains"], z26=z26)
        np.testing.assert_array_equal(out["n_grown"].cpu().numpy().view(np.uint16), ref["n_grown"])
        np.testing.assert_array_equal(out["log_w"].cpu().numpy(), ref["log_w"])
        np.testing.assert_array_equal(out["r_end"].cpu().numpy().astype(np.int32), ref["r_end"])
        np.testing.assert_array_equal(out["n2rg2"].cpu().numpy(), ref["n2rg2"])
