"""Parity of the 26-neighbour lattice kernel (RSAW_LATTICE_26, the z = 26
lattice space of Sec. 3.3.2) with the oracle, bit for bit: log W, exact W,
end vector, R^2, g^2 Rg^2, Rg^2 and monomers placed per chain, and the
ensemble summary and histogram.  Sizes cover both kernels (one lane per
chain up to N = 64, G = 4, 8, 16, 32 and 64 lanes per chain beyond), one
and several scan passes, the largest N, and ragged chain counts over
256-thread blocks.

Dead ends are too rare on this lattice to appear in any ensemble the
oracle can search: it grows no trapped chain among the first 4 10^6
chains of N = 64, 4 10^5 of N = 256 and 2 10^4 of N = 2048 (seed 1), so
no chain index exists to replay here through chain_offset, and the
dead-end and restart branches are exercised only in their no-dead-end
form.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu

RTOL_SUM = 1e-12


def _case(N, M, seed, coord="i32", exact_w=False, bins=0, offset=0, restart=False):
    print(f"[gpu] lattice26 N={N} M={M} seed={seed} coord={coord} exact={exact_w} "
          f"bins={bins} offset={offset} restart={restart}", flush=True)
    out, s = rs.gen_chains("lattice26", N, 26, M, seed, coord=coord, exact_w=exact_w,
                           hist_bins=bins, chain_offset=offset, restart=restart)
    torch.cuda.synchronize()
    out = {n: t.cpu().numpy() for n, t in out.items()}
    ref = oracle.gen_lattice(seed, N, M, chain_offset=offset, restart=restart, z26=True)
    np.testing.assert_array_equal(out["n_grown"].view(np.uint16), ref["n_grown"])
    np.testing.assert_array_equal(out["log_w"], ref["log_w"])
    np.testing.assert_array_equal(out["r_end"].astype(np.int32), ref["r_end"])
    np.testing.assert_array_equal(out["r2"], ref["r2"].astype(np.float64))
    np.testing.assert_array_equal(out["n2rg2"], ref["n2rg2"])
    np.testing.assert_array_equal(out["rg2"], ref["rg2"])
    if exact_w:
        assert ref["w_exact_ok"].all()
        np.testing.assert_array_equal(out["w_exact"], ref["w_exact"])
    red = oracle.reduce(N, ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"], bins=bins)
    assert s["status"] == 0 and s["n_chains"] == M
    assert s["n_alive"] == red["alive"] and s["steps"] == red["steps"]
    if red["alive"]:
        assert s["log_w_max"] == red["log_w_max"]
        for key in ("sum_w", "sum_w2", "sum_w_r2", "sum_w_rg2", "log_c_est", "r2_mean",
                    "rg2_mean", "ess"):
            assert abs(s[key] - red[key]) <= RTOL_SUM * abs(red[key]), (key, s[key], red[key])
    if exact_w:
        ex = oracle.reduce_exact(ref["w_exact"], ref["r2"], ref["n2rg2"])
        assert s["exact_valid"] == 1
        assert s["sum_w_exact"] == ex["sum_w"]
        assert s["sum_w_r2_exact"] == ex["sum_w_r2"]
        assert s["sum_w_n2rg2_exact"] == ex["sum_w_n2rg2"]
    if bins:
        np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
        np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)
    return out, s


@pytest.mark.parametrize("N,M,seed,coord", [
    (1, 300, 1, "i32"), (2, 257, 2, "i16"), (3, 1_000, 3, "i32"), (5, 999, 4, "i16"),
    (16, 5_000, 5, "i32"), (64, 20_000, 6, "i16"), (100, 3_001, 7, "i32"),
    (129, 1_000, 8, "i16"), (161, 500, 10, "i16"), (256, 1_500, 15, "i16"), (257, 600, 16, "i32"),
    (300, 700, 9, "i32"), (512, 150, 17, "i32"), (513, 120, 18, "i16"), (600, 200, 14, "i16")])
def test_lattice26_bit_exact(N, M, seed, coord):
    _case(N, M, seed, coord=coord, bins=256 if N > 1 else 0)


@pytest.mark.parametrize("N,M,seed", [(14, 20_000, 11), (10, 3_333, 12), (2, 100, 13)])
def test_lattice26_exact_weights(N, M, seed):
    _case(N, M, seed, exact_w=True, bins=64)


@pytest.mark.parametrize("N,M,seed,coord", [
    (1_000, 65, 21, "i16"), (4_096, 5, 22, "i32"), (4_097, 5, 23, "i16"),
    (6_000, 3, 24, "i32"), (16_384, 1, 25, "i16")])
def test_lattice26_long_chains(N, M, seed, coord):
    _case(N, M, seed, coord=coord, bins=256)


def test_lattice26_offset_and_restart():
    _case(64, 2_000, 31, offset=123_456_789, bins=32)
    # the group kernel (G = 8): offset past 2^32 and restart
    _case(200, 800, 34, offset=(1 << 32) + 5, bins=32, restart=True)
    a, sa = _case(40, 3_000, 32, restart=True)
    b, sb = _case(40, 3_000, 32, restart=False)
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])


def test_lattice26_in_mixed_batch_equals_single_calls():
    specs = [dict(geometry="lattice26", N=64, k=26, n_chains=5_000, seed=41, coord="i16", hist_bins=64),
             dict(geometry="lattice", N=64, k=6, n_chains=3_000, seed=42, coord="i16"),
             dict(geometry="lattice26", N=12, k=26, n_chains=777, seed=43, exact_w=True),
             dict(geometry="lattice26", N=200, k=26, n_chains=300, seed=44),
             dict(geometry="real", N=30, k=8, n_chains=500, seed=45),
             dict(geometry="lattice26", N=5_000, k=26, n_chains=2, seed=46)]
    print("[gpu] lattice26 mixed batch", flush=True)
    res = rs.gen_batch(specs)
    torch.cuda.synchronize()
    for i, (sp, (out, s)) in enumerate(zip(specs, res)):
        sp = dict(sp)
        one, one_s = rs.gen_chains(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                                   sp.pop("seed"), **sp)
        torch.cuda.synchronize()
        for key in out:
            np.testing.assert_array_equal(out[key].cpu().numpy(), one[key].cpu().numpy(),
                                          err_msg=f"ensemble {i} {key}")
        for key in s:
            assert s[key] == one_s[key] or (s[key] != s[key] and one_s[key] != one_s[key]), (i, key)


def test_grid_slices_cover_every_chain():
    """A grid above 2^31 work-items is issued in slices: 1.5e8 chains of 32
    lanes each take three launches; every chain must be grown once, with the
    chains at the slice boundaries equal to the oracle's."""
    N, M, seed = 2, 150_000_000, 51
    print(f"[gpu] lattice26 sliced grid N={N} M={M}", flush=True)
    out, s = rs.gen_chains("lattice26", N, 26, M, seed, coord="i16", hist_bins=4)
    torch.cuda.synchronize()
    assert s["status"] == 0 and s["n_alive"] == M and s["steps"] == M
    assert s["sum_w"] == float(M)  # every chain has W = 26 = max W
    hn = out["hist_n"].cpu().numpy()
    assert hn.sum() == M and hn[0] == 0 and hn[1] == 0
    # R^2 in {1, 2, 3} with probabilities 6, 12, 8 over 26
    p1 = hn[2] / M
    assert abs(p1 - 6 / 26) < 6 * (6 / 26 * 20 / 26 / M) ** 0.5
    per_slice = ((1 << 31) // 256) * 8
    for c0 in (0, per_slice - 3, 2 * per_slice - 3, M - 5):
        ref = oracle.gen_lattice(seed, N, 6, chain_offset=c0, z26=True)
        np.testing.assert_array_equal(out["r_end"][:, c0:c0 + 6].cpu().numpy().astype(np.int32),
                                      ref["r_end"][:, :min(6, M - c0)])
        np.testing.assert_array_equal(out["log_w"][c0:c0 + 6].cpu().numpy(), ref["log_w"][:min(6, M - c0)])
    del out
    torch.cuda.empty_cache()


def test_workload_lattice26_n64_sampled():
    """The benchmarked workload (N = 64, 10^7 chains, int16, 256 bins) in the
    launch configuration the benchmark times: sampled chains against the
    oracle one by one, and the full reduction against the oracle's reduction
    of the same per-chain outputs."""
    from paper_1704_04381_amd.workloads import WORKLOADS

    w = WORKLOADS["lattice26_n64"]
    M, N = w["n_chains"], w["N"]
    print(f"[gpu] lattice26 workload N={N} M={M}", flush=True)
    out, s = rs.gen_chains(w["geometry"], N, w["k"], M, w["seed"], coord=w["coord"],
                           hist_bins=w["hist_bins"])
    torch.cuda.synchronize()
    out = {n: t.cpu().numpy() for n, t in out.items()}
    rng = np.random.default_rng(97)
    idx = np.unique(np.concatenate([np.arange(0, M, M // 1000), rng.integers(0, M, 1000), [M - 1]]))
    for c in idx:
        ch = oracle.lattice_chain(w["seed"], int(c), N, z26=True)
        assert out["log_w"][c] == ch["log_w"]
        assert int(out["n_grown"].view(np.uint16)[c]) == ch["n_grown"]
        assert tuple(int(v) for v in out["r_end"][:, c]) == tuple(int(v) for v in ch["end"])
        assert out["n2rg2"][c] == ch["n2rg2"]
        assert out["rg2"][c] == ch["rg2"]
    red = oracle.reduce(N, out["log_w"], out["r2"], out["rg2"],
                        out["n_grown"].view(np.uint16).astype(np.int32), bins=w["hist_bins"])
    assert s["status"] == 0 and s["n_alive"] == red["alive"] and s["steps"] == red["steps"]
    assert s["log_w_max"] == red["log_w_max"]
    for key in ("sum_w", "sum_w2", "sum_w_r2", "sum_w_rg2", "log_c_est", "r2_mean", "rg2_mean", "ess"):
        assert abs(s[key] - red[key]) <= RTOL_SUM * abs(red[key]), (key, s[key], red[key])
    np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
    np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)
