"""rsaw_gen_chains_static, the allocation-free variant of rsaw_gen_chains
(workspace in the library's static device scratch), against rsaw_gen_chains
on the same inputs: every per-chain array, the histograms and the summary
bit for bit, on consecutive calls whose second one is smaller, with and
without caller-supplied per-chain outputs.  Also the host-side rejection of
a call that needs more workspace than the scratch holds.

GPU test; calls the HIP library through its C ABI (ctypes binding).
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu

# (geometry, N, k, first M, second M, coord, hist bins, extra)
CASES = [("lattice", 64, 6, 300_000, 70_001, "i16", 64, {}),
         ("lattice", 16, 6, 50_000, 4_097, "i32", 32, dict(exact_w=True)),
         ("lattice", 200, 6, 20_000, 3_001, "i16", 0, {}),
         ("lattice26", 40, 26, 40_000, 9_999, "i32", 16, {}),
         ("real", 64, 8, 30_000, 5_003, None, 16, {}),
         ("real", 300, 5, 3_000, 777, None, 0, {})]


def _run(fn, cfg, dev, per_chain, bins, stream):
    out, o = rs._alloc_outputs(cfg, dev, per_chain, bins)
    for v in out.values():
        v.view(torch.uint8).fill_(0xA5)  # stale bytes must not leak into results
    summ = torch.full((rs.SUMMARY_BYTES,), 0x5A, dtype=torch.uint8, device=dev)
    fn(cfg, o if per_chain else None, summ.data_ptr(), out["hist_w"].data_ptr() if bins else 0,
       out["hist_n"].data_ptr() if bins else 0, stream)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().copy() for k, v in out.items()}, summ.cpu().numpy().copy()


@pytest.mark.parametrize("geometry,N,k,m1,m2,coord,bins,extra", CASES)
@pytest.mark.parametrize("per_chain", [True, False])
def test_static_matches_gen_chains(geometry, N, k, m1, m2, coord, bins, extra, per_chain):
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    for M, seed in ((m1, 11), (m2, 12)):
        print(f"[gpu] static scratch: {geometry} N={N} k={k} M={M} per_chain={per_chain}", flush=True)
        cfg = rs.make_config(geometry, N, k, M, seed, coord=coord, hist_bins=bins, chain_offset=(1 << 32) + 9,
                             **extra)
        ref_out, ref_sum = _run(rs.gen_chains_raw, cfg, dev, per_chain, bins, stream)
        got_out, got_sum = _run(rs.gen_chains_static_raw, cfg, dev, per_chain, bins, stream)
        assert np.array_equal(got_sum, ref_sum), "summary bytes differ"
        s = rs.parse_summary(torch.from_numpy(got_sum))
        assert s["status"] == 0 and s["n_chains"] == M
        assert set(got_out) == set(ref_out)
        for name in ref_out:
            assert np.array_equal(got_out[name].view(np.uint8), ref_out[name].view(np.uint8)), name


def test_static_rejects_a_call_beyond_the_scratch():
    lib = rs.load()
    # 2 million lattice chains with no per-chain outputs: the reduction's
    # per-chain arrays alone need 52 MB
    cfg = rs.make_config("lattice", 64, 6, 2_000_000, 1, coord="i16")
    need = rs.workspace_size(cfg, None, True)
    assert need > rs.STATIC_SCRATCH_BYTES
    dev = torch.device("cuda", 0)
    summ = torch.empty(rs.SUMMARY_BYTES, dtype=torch.uint8, device=dev)
    st = lib.rsaw_gen_chains_static(C.byref(cfg), None, C.c_void_p(summ.data_ptr()), None, None, None)
    assert st == 4, (st, lib.rsaw_last_error())
    assert b"static scratch" in lib.rsaw_last_error()
    # a fitting call on the same device still works afterwards
    cfg = rs.make_config("lattice", 16, 6, 1000, 1, coord="i32")
    _run(rs.gen_chains_static_raw, cfg, dev, False, 0, torch.cuda.current_stream(dev).cuda_stream)
