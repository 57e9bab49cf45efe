"""Tuning table of the group kernels' lane mapping: the host-only calls
(rsaw_mapping_set / _query / _clear) of the HIP library, no device call.

The mapping only decides how a chain's scan is spread over lanes; which
mappings are legal follows from each group kernel's word formats and its
LDS need (a CU holds 160 KiB).
"""
from __future__ import annotations

import pytest

import paper_1704_04381_amd as rs


@pytest.fixture(autouse=True)
def _clean_table():
    if not __import__("os").path.exists(rs.LIB_PATH):
        pytest.skip("librsaw.so not built")
    rs.mapping_clear()
    yield
    rs.mapping_clear()


def _q(geo, N, k):
    return rs.mapping_query(rs.make_config(geo, N, k, 1000, 1))


def test_builtin_rule():
    # one lane per chain where there is no group kernel
    assert _q("lattice", 64, 6)["lanes"] == 1
    assert _q("lattice26", 64, 26)["lanes"] == 1
    # group widths of the built-in rule
    assert [_q("lattice", n, 6)["lanes"] for n in (65, 128, 129, 256, 257, 512, 513, 1024, 2048, 2049, 3000,
                                                   4096, 4097)] == \
        [2, 2, 4, 4, 8, 8, 16, 16, 32, 64, 64, 64, 64]
    assert [_q("lattice26", n, 26)["lanes"] for n in (65, 128, 129, 256, 257, 512, 513, 1024, 1025, 2048, 2049,
                                                     4096, 4097)] == \
        [2, 2, 4, 4, 8, 8, 16, 16, 32, 32, 64, 64, 64]
    assert _q("real", 64, 8)["lanes"] == 8 and _q("real", 64, 16)["lanes"] == 16
    assert _q("real", 300, 8)["lanes"] == 32  # 0.075 N = 22.5 -> 32
    # k = 8: 16 lanes while a 256-thread block leaves 3 blocks per CU, then
    # 32 lanes in one-wave blocks
    assert (_q("real", 128, 8)["lanes"], _q("real", 128, 8)["threads"]) == (16, 256)
    for n in (144, 192, 213):
        assert (_q("real", n, 8)["lanes"], _q("real", n, 8)["threads"]) == (32, 64), n
    assert (_q("real", 192, 16)["lanes"], _q("real", 192, 16)["threads"]) == (16, 256)
    # k = 16: 32 lanes in 256-thread blocks up to N = 284, then 64 lanes
    # in one-wave blocks while the occupancy term asks for 32
    assert (_q("real", 256, 16)["lanes"], _q("real", 256, 16)["threads"]) == (32, 256)
    for n in (285, 384, 426):
        assert (_q("real", n, 16)["lanes"], _q("real", n, 16)["threads"]) == (64, 64), n
    assert (_q("real", 106, 4)["lanes"], _q("real", 106, 4)["threads"]) == (8, 256)  # k = 4 unchanged
    # beyond N = 1536 hard-sphere planes live in HBM
    m = _q("real", 3000, 8)
    assert m["lanes"] == 64 and m["threads"] == 64 and m["lds_bytes"] == 0
    for geo, k in (("lattice", 6), ("real", 8), ("lattice26", 26)):
        for n in (65, 200, 1000, 1536):
            assert _q(geo, n, k)["lds_bytes"] <= 160 * 1024


def test_set_overrides_inside_its_range_only():
    base = _q("lattice", 100, 6)
    rs.mapping_set("lattice", 6, 65, 128, 32, 64)
    m = _q("lattice", 100, 6)
    assert (m["lanes"], m["threads"]) == (32, 64)
    assert _q("lattice", 129, 6)["lanes"] == 4       # outside the range
    assert _q("lattice", 64, 6)["lanes"] == 1        # register kernel: never tuned
    assert _q("lattice26", 100, 26)["lanes"] == 2    # other geometry
    # a later entry wins where ranges overlap
    rs.mapping_set("lattice", 6, 90, 110, 16, 256)
    assert (_q("lattice", 100, 6)["lanes"], _q("lattice", 100, 6)["threads"]) == (16, 256)
    assert _q("lattice", 80, 6)["lanes"] == 32
    rs.mapping_clear()
    assert _q("lattice", 100, 6) == base


def test_hard_sphere_mapping_is_per_k():
    rs.mapping_set("real", 8, 1, 200, 64, 64)
    assert _q("real", 100, 8)["lanes"] == 64
    assert _q("real", 100, 16)["lanes"] == 16


@pytest.mark.parametrize("args", [
    ("lattice", 6, 65, 2100, 4, 64),     # 4 lanes: byte words, N <= 2048
    ("lattice", 6, 65, 129, 2, 64),      # 2 lanes hold N <= 128 only
    ("real", 8, 65, 100, 2, 256),        # not a hard-sphere group width
    ("lattice26", 26, 65, 129, 2, 256),  # 2 lanes hold N <= 128 only
    ("lattice", 6, 65, 100, 8, 128),     # threads must be 64 or 256
    ("lattice", 6, 10, 64, 8, 64),       # N <= 64: register kernel
    ("real", 16, 10, 100, 8, 256),       # fewer lanes than trials
    ("real", 8, 10, 100, 64, 256),       # 64 lanes only in one-wave blocks
    ("real", 8, 10, 3000, 32, 64),       # beyond the LDS kernel
    ("real", 8, 10, 1536, 8, 64),        # 8 chains' planes exceed 160 KiB
    ("lattice26", 26, 65, 300, 4, 256),  # 8-bit n_m fields need N <= 256
    ("lattice26", 26, 70, 60, 8, 64),    # empty range
    ("lattice", 5, 65, 100, 8, 64),      # lattice k must be 6
])
def test_set_rejects_illegal_mappings(args):
    geo, k = args[0], (args[1] if args[1] in (6, 8, 16, 26) else 6)
    before = _q(geo, 100, k)
    with pytest.raises(rs.RsawError) as e:
        rs.mapping_set(*args)
    assert e.value.status == 1  # RSAW_E_INVALID
    assert _q(geo, 100, k) == before  # nothing installed


def test_legal_mapping_at_n_hi_is_legal_below():
    for geo, k in (("lattice", 6), ("real", 8), ("lattice26", 26)):
        for lanes in (2, 4, 8, 16, 32, 64):
            for threads in (64, 256):
                try:
                    rs.mapping_set(geo, k, 65, 1000, lanes, threads)
                except rs.RsawError:
                    continue
                for n in (65, 300, 999, 1000):
                    m = _q(geo, n, k)
                    assert (m["lanes"], m["threads"]) == (lanes, threads), (geo, n, lanes, threads)
                rs.mapping_clear()


def test_list_save_and_load_round_trip(tmp_path):
    assert rs.mapping_list() == []
    rs.mapping_set("lattice", 6, 65, 128, 32, 64)
    rs.mapping_set("real", 16, 1, 100, 32, 256)
    rs.mapping_set("lattice26", 26, 65, 256, 4, 64)
    rows = rs.mapping_list()
    assert [(m["geometry"], m["lanes"], m["threads"]) for m in rows] == [(0, 32, 64), (1, 32, 256), (2, 4, 64)]
    path = tmp_path / "mappings.json"
    assert rs.save_mappings(path) == 3
    probes = [("lattice", 100, 6), ("real", 50, 16), ("lattice26", 200, 26), ("lattice", 300, 6)]
    before = [_q(*p) for p in probes]
    rs.mapping_clear()
    assert rs.mapping_list() == []
    assert rs.load_mappings(path) == 3
    assert rs.mapping_list() == rows
    assert [_q(*p) for p in probes] == before


def test_byte_box_edge_range():
    # rsaw_set_byte_box: host-only; 0 (each format's own edge) or 1..127,
    # anything else rejected
    for bad in (-1, 128, 1 << 20):
        with pytest.raises(rs.RsawError) as e:
            rs.set_byte_box(bad)
        assert e.value.status == 1  # RSAW_E_INVALID
    rs.set_byte_box(1)
    rs.set_byte_box(127)
    rs.set_byte_box(0)
