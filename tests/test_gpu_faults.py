"""Device allocation failure.  A batch whose workspace exceeds the device's
memory fails with RSAW_E_NOMEM before enqueueing anything, keeps no partial
allocation, and leaves the library usable on the same stream: the next call
there is bit-exact against the oracle.  GPU test; calls the HIP library
through its C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu


def test_workspace_allocation_failure_reports_nomem_and_recovers():
    M = (1 << 32) - 1  # the largest ensemble; summaries only, so the
    cfgs = [rs.make_config("lattice", 64, 6, M, seed) for seed in (1, 2, 3, 4)]  # per-chain arrays in the workspace
    need = sum(rs.workspace_size(c) for c in cfgs)
    summ = torch.zeros(len(cfgs) * rs.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    assert int(summ.count_nonzero()) == 0
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    print(f"[gpu] allocation failure: workspace {need / 2**30:.0f} GiB, device {total / 2**30:.0f} GiB", flush=True)
    assert need > total
    with pytest.raises(rs.RsawError) as e:
        rs.gen_batch_raw(cfgs, None, summ.data_ptr())
    assert e.value.status == 4  # RSAW_E_NOMEM
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # no device allocation kept (the stream's earlier workspace, if any, is
    # released before the failed attempt, so free memory can only grow)
    assert free1 >= free0 - (4 << 20), (free0, free1)
    assert int(summ.count_nonzero()) == 0  # nothing was enqueued
    # the same (current) stream serves the next calls, single and batched
    out, s = rs.gen_chains("lattice", 64, 6, 1_000, 5)
    torch.cuda.synchronize()
    ref = oracle.gen_lattice(5, 64, 1_000)
    np.testing.assert_array_equal(out["log_w"].cpu().numpy(), ref["log_w"])
    np.testing.assert_array_equal(out["n2rg2"].cpu().numpy(), ref["n2rg2"])
    assert s["status"] == 0
    res = rs.gen_batch([dict(geometry="lattice", N=100, k=6, n_chains=500, seed=6)])
    torch.cuda.synchronize()
    ref = oracle.gen_lattice(6, 100, 500)
    np.testing.assert_array_equal(res[0][0]["log_w"].cpu().numpy(), ref["log_w"])
