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


# one ensemble per growth-kernel family: lattice in registers (one lane,
# and a group), lattice with its words in LDS (N > 4096), hard spheres with
# LDS and HBM planes, 26-neighbour lattice in registers and in LDS, and an
# empty ensemble
BATCH = [dict(geometry="lattice", N=16, k=6, n_chains=30_000, seed=11, coord="i32", exact_w=True, hist_bins=8),
         dict(geometry="lattice", N=100, k=6, n_chains=20_000, seed=12, coord="i16", hist_bins=64),
         dict(geometry="lattice", N=5_000, k=6, n_chains=12, seed=17, coord="i32"),
         dict(geometry="real", N=64, k=8, n_chains=10_000, seed=13, hist_bins=16),
         dict(geometry="real", N=1800, k=8, n_chains=40, seed=14),
         dict(geometry="lattice26", N=200, k=26, n_chains=5_000, seed=15, coord="i32"),
         dict(geometry="lattice26", N=5_000, k=26, n_chains=6, seed=18, coord="i16"),
         dict(geometry="lattice", N=33, k=6, n_chains=0, seed=16, coord="i32", hist_bins=4)]


def _plan_snapshot(plan):
    return [({k: v.cpu().numpy().copy() for k, v in out.items()}, plan.summaries.cpu().numpy().copy())
            for out in plan.outputs]


def test_batch_plan_equals_gen_batch_and_replays_in_a_graph():
    dev = torch.device("cuda", 0)
    print("[gpu] batch plan: eager gen_batch reference", flush=True)
    ref = rs.gen_batch(BATCH)
    torch.cuda.synchronize()
    ref = [({k: v.cpu().numpy() for k, v in out.items()}, s) for out, s in ref]
    plan = rs.BatchPlan(BATCH)
    side = torch.cuda.Stream(device=dev)

    def check(tag):
        for i, ((o_ref, s_ref), (o_got, s_got)) in enumerate(zip(ref, plan.results())):
            for k in o_ref:
                np.testing.assert_array_equal(o_got[k].cpu().numpy(), o_ref[k], err_msg=f"{tag} ensemble {i} {k}")
            for k, v in s_ref.items():
                w = s_got[k]
                assert w == v or (v != v and w != w), (tag, i, k, v, w)

    print("[gpu] batch plan: eager launches", flush=True)
    for rep in range(2):
        with torch.cuda.stream(side):
            plan.launch(side.cuda_stream)
        torch.cuda.synchronize()
        check(f"eager {rep}")

    g = torch.cuda.CUDAGraph()
    print("[gpu] batch plan: capture", flush=True)
    with torch.cuda.graph(g, stream=side):
        plan.launch(side.cuda_stream)
    torch.cuda.synchronize()
    other = _prepare(dev)
    for rep in range(3):
        for out in plan.outputs:
            for v in out.values():
                v.zero_()
        plan.summaries.zero_()
        _launch(other, torch.cuda.current_stream(dev).cuda_stream)  # eager work between replays
        torch.cuda.synchronize()
        print(f"[gpu] batch plan: replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        check(f"replay {rep}")
    del g
    plan.close()


def test_batch_plan_argument_errors():
    with pytest.raises(rs.RsawError):
        rs.BatchPlan([dict(geometry="lattice", N=70000, k=6, n_chains=10, seed=1)])
    empty = rs.BatchPlan([])
    empty.launch()
    torch.cuda.synchronize()
    empty.close()


def test_caller_workspace_allows_capture_without_warm_up():
    """rsaw_set_workspace: a fresh stream bound to a caller-owned buffer is
    captured into a graph with no earlier call on it; every replay equals the
    eager calls on another stream bit for bit.  A call needing more than the
    buffer fails with RSAW_E_NOMEM and enqueues nothing."""
    dev = torch.device("cuda", 0)
    calls = _prepare(dev)
    print("[gpu] caller workspace: eager reference on the current stream", flush=True)
    _launch(calls, torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    ref = _snapshot(calls)
    need = max(rs.workspace_size(cfg, o) for cfg, o, _, _ in calls)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    fresh = torch.cuda.Stream(device=dev)
    with torch.cuda.device(dev):
        rs.set_workspace(ws.data_ptr(), need, fresh.cuda_stream)
    try:
        g = torch.cuda.CUDAGraph()
        print("[gpu] caller workspace: capture on a fresh stream", flush=True)
        with torch.cuda.graph(g, stream=fresh):
            _launch(calls, fresh.cuda_stream)
        torch.cuda.synchronize()
        other = _prepare(dev)
        for rep in range(3):
            for _, _, out, summ in calls:
                for v in out.values():
                    v.zero_()
                summ.zero_()
            _launch(other, torch.cuda.current_stream(dev).cuda_stream)
            torch.cuda.synchronize()
            print(f"[gpu] caller workspace: replay {rep}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            got = _snapshot(calls)
            for i, ((o_ref, s_ref), (o_got, s_got)) in enumerate(zip(ref, got)):
                for k in o_ref:
                    np.testing.assert_array_equal(o_got[k], o_ref[k], err_msg=f"replay {rep} call {i} {k}")
                np.testing.assert_array_equal(s_got, s_ref, err_msg=f"replay {rep} call {i} summary")
        del g
        # too small for a call without per-chain outputs: refused, nothing enqueued
        big = rs.make_config("lattice", 64, 6, 10 * need, 1, coord="i16")
        summ = torch.zeros(rs.SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        with pytest.raises(rs.RsawError) as e:
            rs.gen_chains_raw(big, None, summ.data_ptr(), 0, 0, fresh.cuda_stream)
        assert e.value.status == 4
        torch.cuda.synchronize()
        assert int(summ.sum()) == 0
    finally:
        with torch.cuda.device(dev):
            rs.set_workspace(0, 0, fresh.cuda_stream)
    # unbound: the stream allocates its own workspace again
    cfg, o, out, summ = calls[0]
    rs.gen_chains_raw(cfg, o, summ.data_ptr(), out["hist_w"].data_ptr(), out["hist_n"].data_ptr(),
                      fresh.cuda_stream)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(summ.cpu().numpy(), ref[0][1])
