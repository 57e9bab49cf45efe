"""rsaw_gen_chains under HIP graph capture: once a stream's workspace
exists, a call records only kernel launches (no allocation, no memset), so
a captured sequence replays bit-identically to the eager calls.  Replays
are separated by the program's own eager work (other ensembles on the
default stream, output clearing) and synchronisations, and every replay is
checked against the eager result.

GPU test; calls the HIP library through its C ABI (ctypes binding).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu

SPECS = [dict(geometry="lattice", N=64, k=6, n_chains=200_000, seed=5, coord="i16", hist_bins=64),
         dict(geometry="lattice26", N=40, k=26, n_chains=50_000, seed=6, coord="i32", hist_bins=32),
         dict(geometry="real", N=48, k=8, n_chains=20_000, seed=7, hist_bins=16)]


def _prepare(dev):
    calls = []
    for sp in SPECS:
        sp = dict(sp)
        bins = sp["hist_bins"]
        cfg = rs.make_config(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                             sp.pop("seed"), **sp)
        out, o = rs._alloc_outputs(cfg, dev, True, bins)
        summ = torch.empty(rs.SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        calls.append((cfg, o, out, summ))
    return calls


def _launch(calls, stream):
    for cfg, o, out, summ in calls:
        rs.gen_chains_raw(cfg, o, summ.data_ptr(), out["hist_w"].data_ptr(), out["hist_n"].data_ptr(),
                          stream)


def _snapshot(calls):
    return [({k: v.cpu().numpy().copy() for k, v in out.items()}, summ.cpu().numpy().copy())
            for _, _, out, summ in calls]


def test_captured_calls_replay_bit_identically():
    dev = torch.device("cuda", 0)
    calls = _prepare(dev)
    side = torch.cuda.Stream(device=dev)
    print("[gpu] graph: eager reference on the capture stream", flush=True)
    with torch.cuda.stream(side):
        _launch(calls, side.cuda_stream)  # also sizes this stream's workspace
    torch.cuda.synchronize()
    ref = _snapshot(calls)

    g = torch.cuda.CUDAGraph()
    print("[gpu] graph: capture", flush=True)
    with torch.cuda.graph(g, stream=side):
        _launch(calls, side.cuda_stream)
    torch.cuda.synchronize()

    other = _prepare(dev)
    for rep in range(3):
        for _, _, out, summ in calls:
            for v in out.values():
                v.zero_()
            summ.zero_()
        _launch(other, torch.cuda.current_stream(dev).cuda_stream)  # eager work between replays
        torch.cuda.synchronize()
        print(f"[gpu] graph: replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(calls)
        for i, ((o_ref, s_ref), (o_got, s_got)) in enumerate(zip(ref, got)):
            for k in o_ref:
                np.testing.assert_array_equal(o_got[k], o_ref[k], err_msg=f"replay {rep} call {i} {k}")
            np.testing.assert_array_equal(s_got, s_ref, err_msg=f"replay {rep} call {i} summary")
    del g
