"""Parity of the HIP path (librsaw through its C ABI) with the oracle.

Lattice: every per-chain output (log W, exact W, end vector, R^2, g^2 Rg^2,
Rg^2, monomers placed) must match the oracle bit for bit; the exact 128-bit
ensemble sums too.  Real space: the same per-chain outputs, required within
1e-12 relative (the decisions use correctly rounded sqrt and division and no
contraction, so they come out identical in practice).  Floating-point
ensemble sums: 1e-12 relative; the derivation is in the module constant
below.  Sizes span several 256-chain tiles with a ragged tail; the headline
sizes are checked on sampled chains plus a full re-reduction by the oracle.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1704_04381_amd as rs
from paper_1704_04381_amd.workloads import WORKLOADS

pytestmark = pytest.mark.gpu

# Ensemble sums of positive terms: the GPU sums each thread's chains in order,
# then two fixed trees; the oracle sums sequentially with compensation.  Both
# are within ~log2(M) * 2^-53 ~ 3e-15 of the exact sum for M <= 10^7, and the
# device exp() differs from the host's by at most 1 ulp per term.  1e-12 leaves
# a wide margin while still catching any dropped or double-counted chain
# (a single chain weighs at least 1/ESS of the sum).
RTOL_SUM = 1e-12
RTOL_REAL = 1e-12

SUM_KEYS = ["sum_w", "sum_w2", "sum_w_r2", "sum_w2_r2", "sum_w2_r2sq", "sum_w_rg2",
            "sum_w2_rg2", "sum_w2_rg2sq", "log_c_est", "r2_mean", "rg2_mean", "ess"]


def _np(t):
    return t.cpu().numpy()


def _gpu(geometry, N, k, M, seed, **kw):
    print(f"[gpu] {geometry} N={N} k={k} M={M} seed={seed} {kw}", flush=True)
    out, s = rs.gen_chains(geometry, N, k, M, seed, **kw)
    torch.cuda.synchronize()
    return {n: _np(t) for n, t in out.items()}, s


def _check_summary(s, ref, M, exact_ref=None):
    assert s["status"] == 0
    assert s["n_chains"] == M
    assert s["n_alive"] == ref["alive"]
    assert s["steps"] == ref["steps"]
    if ref["alive"] == 0:
        assert s["log_c_est"] == -math.inf
        return
    assert s["log_w_max"] == ref["log_w_max"]
    for key in SUM_KEYS:
        a, b = s[key], ref[key]
        assert abs(a - b) <= RTOL_SUM * abs(b), (key, a, b)
    b = ref["c_rel_err"]
    if math.isfinite(b):
        assert abs(s["c_rel_err"] - b) <= 1e-6 * abs(b) + 1e-300, ("c_rel_err", s["c_rel_err"], b)
    # std. error of <A> (Eq. 2): sqrt(|S_w2A2 - 2 <A> S_w2A + <A>^2 S2|) / S0
    # on both sides.  The three terms agree to RTOL_SUM, but they cancel when
    # a few chains carry the weight, so the square under the root is
    # compared on the scale of its terms, not relative to itself.
    for key, k4, k3, km in (("r2_err", "sum_w2_r2sq", "sum_w2_r2", "r2_mean"),
                            ("rg2_err", "sum_w2_rg2sq", "sum_w2_rg2", "rg2_mean")):
        a, b = s[key], ref[key]
        if math.isfinite(b):
            S0, m = ref["sum_w"], ref[km]
            scale = ref[k4] + 2.0 * abs(m) * ref[k3] + m * m * ref["sum_w2"]
            assert abs((a * S0) ** 2 - (b * S0) ** 2) <= 1e-10 * scale + 1e-300, (key, a, b)
    if exact_ref is not None:
        assert s["exact_valid"] == 1
        assert s["sum_w_exact"] == exact_ref["sum_w"]
        assert s["sum_w_r2_exact"] == exact_ref["sum_w_r2"]
        assert s["sum_w_n2rg2_exact"] == exact_ref["sum_w_n2rg2"]


def _lattice_case(N, M, seed, coord="i32", exact_w=False, bins=0, offset=0, restart=False):
    out, s = _gpu("lattice", N, 6, M, seed, coord=coord, exact_w=exact_w, hist_bins=bins,
                  chain_offset=offset, restart=restart)
    ref = oracle.gen_lattice(seed, N, M, chain_offset=offset, restart=restart)
    np.testing.assert_array_equal(out["n_grown"].view(np.uint16), ref["n_grown"])
    np.testing.assert_array_equal(out["log_w"], ref["log_w"])
    np.testing.assert_array_equal(out["r_end"].astype(np.int32), ref["r_end"])
    np.testing.assert_array_equal(out["r2"], ref["r2"].astype(np.float64))
    np.testing.assert_array_equal(out["n2rg2"], ref["n2rg2"])
    np.testing.assert_array_equal(out["rg2"], ref["rg2"])
    if exact_w:
        np.testing.assert_array_equal(out["w_exact"], ref["w_exact"])
    red = oracle.reduce(N, ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"], bins=bins)
    ex = oracle.reduce_exact(ref["w_exact"], ref["r2"], ref["n2rg2"]) if exact_w else None
    _check_summary(s, red, M, ex)
    if bins:
        np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
        np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)
    return out, s


@pytest.mark.parametrize("N,M,seed", [(16, 20_000, 1), (16, 777, 5), (28, 3001, 2)])
def test_lattice_exact_weights(N, M, seed):
    _lattice_case(N, M, seed, coord="i32", exact_w=True)


@pytest.mark.parametrize("N,M,seed,coord", [(64, 6_000, 1, "i16"), (64, 2_561, 3, "i32"),
                                            (33, 4_100, 4, "i16"), (17, 1_000, 6, "i32"),
                                            (1, 300, 7, "i32"), (2, 300, 8, "i16"),
                                            (3, 257, 9, "i32"), (5, 10_000, 10, "i16")])
def test_lattice_bit_exact(N, M, seed, coord):
    _lattice_case(N, M, seed, coord=coord, bins=256 if N > 1 else 0)


@pytest.mark.parametrize("N,M,seed,coord", [
    # group kernels: byte words in the group's registers with 2 lanes per
    # chain (N <= 128), 4 (N <= 256; boxed beyond 128), 8 (N <= 512), 16
    # (N <= 1024), 32 (N <= 2048) and 64 (N <= 4096; each lane's last slot at
    # the top of each range), then wide words in LDS with 32 and 64 lanes
    # per chain, up to the largest N
    (65, 3_001, 21, "i16"), (100, 1_500, 22, "i32"), (128, 2_000, 23, "i16"),
    (129, 801, 24, "i32"), (256, 2_000, 41, "i16"), (257, 700, 42, "i32"),
    (300, 333, 25, "i16"), (512, 300, 26, "i32"),
    (513, 200, 27, "i16"), (1_024, 100, 32, "i16"), (1_025, 80, 33, "i32"),
    (2_048, 60, 28, "i32"), (2_049, 40, 29, "i16"), (3_001, 16, 34, "i32"),
    (4_096, 10, 35, "i16"), (4_097, 8, 36, "i32"),
    (5_000, 12, 30, "i32"), (16_384, 3, 31, "i16")])
def test_lattice_long_chains_bit_exact(N, M, seed, coord):
    _lattice_case(N, M, seed, coord=coord, bins=256)


def test_lattice_long_offset_and_dead_chains():
    # the LDS kernel with a chain offset past 2^32; N = 400 chains meet dead
    # ends often enough to cover that branch
    out, _ = _lattice_case(400, 2_000, 43, coord="i32", bins=64, offset=(1 << 32) + 5)
    assert (out["n_grown"].view(np.uint16) < 400).sum() > 10


def test_lattice_dead_chains_bit_exact():
    # N = 64 chains get trapped often enough to exercise the dead-end path
    out, _ = _lattice_case(64, 40_000, 11, coord="i16", bins=256)
    assert (out["n_grown"].view(np.uint16) < 64).sum() > 10


def _real_case(N, k, M, seed, b=1.0, sigma=1.0, bins=0, offset=0, restart=False):
    out, s = _gpu("real", N, k, M, seed, bond_length=b, bead_diameter=sigma, hist_bins=bins,
                  chain_offset=offset, restart=restart)
    ref = oracle.gen_real(seed, N, k, M, b=b, sigma=sigma, chain_offset=offset, restart=restart)
    np.testing.assert_array_equal(out["n_grown"].view(np.uint16), ref["n_grown"])
    alive = np.isfinite(ref["log_w"])
    np.testing.assert_array_equal(np.isfinite(out["log_w"]), alive)
    np.testing.assert_allclose(out["log_w"][alive], ref["log_w"][alive], rtol=RTOL_REAL, atol=0)
    for key in ("r2", "rg2"):
        np.testing.assert_allclose(out[key], ref[key], rtol=RTOL_REAL, atol=1e-300)
    scale = np.maximum(np.abs(ref["r_end"]).max(), 1.0)
    np.testing.assert_allclose(out["r_end"], ref["r_end"], rtol=0, atol=RTOL_REAL * scale)
    red = oracle.reduce(N, ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"], bins=bins)
    _check_summary(s, red, M)
    if bins:
        np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
        np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)
    exact = all(np.array_equal(out[kk], ref[kk]) for kk in ("log_w", "r2", "rg2", "r_end"))
    print(f"[gpu] real N={N} k={k}: per-chain outputs bit-identical: {exact}", flush=True)
    return out, s, exact


@pytest.mark.parametrize("N,k,M,seed", [(64, 8, 1_500, 1), (17, 8, 2_003, 2), (3, 8, 999, 3),
                                        (2, 8, 100, 4), (1, 8, 64, 5), (24, 1, 700, 6),
                                        (24, 5, 700, 7), (20, 16, 600, 8), (12, 33, 300, 9),
                                        (10, 64, 200, 10),
                                        # one-wave blocks (bead planes above 64 KiB at
                                        # 256 threads) up to the largest N
                                        (100, 8, 403, 11), (256, 8, 77, 12), (200, 16, 101, 13),
                                        (150, 33, 65, 14), (256, 64, 21, 15),
                                        # round-1 draws spread over spare lanes
                                        # (G >= 4k), k not dividing G
                                        (300, 5, 90, 16), (600, 7, 30, 17), (480, 3, 40, 18)])
def test_real_parity(N, k, M, seed):
    _, _, exact = _real_case(N, k, M, seed, bins=128)
    assert exact


@pytest.mark.parametrize("N,k,M,seed,sigma", [
    # LDS planes: 32 lanes per chain in 256-thread blocks (N = 300), one
    # wave per chain in one-wave blocks from N = 427 to the LDS limit 1536
    (300, 8, 64, 41, 1.0), (460, 8, 40, 49, 1.0), (512, 16, 20, 50, 0.8),
    (700, 8, 24, 42, 1.0), (700, 16, 12, 43, 0.8), (1_536, 8, 6, 51, 0.5),
    # HBM-resident planes beyond the LDS limit (persistent grid)
    (2_048, 8, 6, 44, 0.5), (6_144, 8, 3, 45, 0.5), (6_145, 8, 3, 46, 0.5), (10_000, 8, 3, 47, 0.4), (16_384, 16, 2, 48, 0.4)])
def test_real_long_chains(N, k, M, seed, sigma):
    _, _, exact = _real_case(N, k, M, seed, sigma=sigma, bins=64)
    assert exact


@pytest.mark.parametrize("N,k,M,seed,offset,sigma", [
    # chain index g = offset + c keys every Philox counter (Sec. 3.2: one
    # independent stream per chain).  G = 8 lanes for k = 8: the wave-wide
    # helper round of the Marsaglia draws (lanes serving other chains'
    # failed trials) runs at most steps and recomputes the owner's g
    (64, 8, 1_500, 61, (1 << 32) + 5, 1.0), (64, 8, 700, 62, 4_321, 1.0),
    (33, 16, 400, 63, (1 << 40) + 3, 1.0),
    # G = 32 with round-1 attempts spread over spare lanes (k = 5)
    (300, 5, 90, 64, (1 << 32) + 5, 1.0), (300, 5, 90, 65, 4_321, 1.0),
    # one chain per wave (G = 64), and HBM-resident bead planes
    (700, 8, 20, 66, (1 << 32) + 5, 1.0), (2_048, 8, 5, 67, (1 << 32) + 5, 0.5)])
def test_real_chain_offset_bit_exact(N, k, M, seed, offset, sigma):
    _, _, exact = _real_case(N, k, M, seed, sigma=sigma, bins=32, offset=offset)
    assert exact


def test_real_split_ranges_equal_one_launch():
    """Hard spheres: two calls over [0, a) and [a, M) (chain_offset = a)
    give the chains of one call over [0, M), bit for bit."""
    M, a = 3_000, 1_234
    full, _ = _gpu("real", 64, 8, M, 23)
    x, _ = _gpu("real", 64, 8, a, 23)
    y, _ = _gpu("real", 64, 8, M - a, 23, chain_offset=a)
    for key in ("log_w", "r2", "rg2", "n_grown"):
        np.testing.assert_array_equal(np.concatenate([x[key], y[key]]), full[key])
    np.testing.assert_array_equal(np.concatenate([x["r_end"], y["r_end"]], axis=1), full["r_end"])


@pytest.mark.parametrize("N,M,seed,coord,exact", [(64, 20_000, 31, "i16", False), (28, 5_000, 32, "i32", True),
                                                  (200, 500, 33, "i32", False), (2_049, 40, 34, "i16", False)])
def test_lattice_restart_bit_exact(N, M, seed, coord, exact):
    out, s = _lattice_case(N, M, seed, coord=coord, exact_w=exact, bins=64, restart=True)
    assert s["n_alive"] == M


@pytest.mark.parametrize("N,k,M,seed,sigma", [(64, 8, 2_000, 31, 1.0), (40, 4, 300, 32, 1.4),
                                              (300, 8, 30, 33, 1.0)])
def test_real_restart_bit_exact(N, k, M, seed, sigma):
    out, s, exact = _real_case(N, k, M, seed, sigma=sigma, bins=32, restart=True)
    assert exact and s["n_alive"] == M


def test_real_ideal_chain_and_bond_length():
    out, s, exact = _real_case(30, 8, 1_000, 12, b=1.5, sigma=0.0)
    assert exact
    assert np.all(out["log_w"] == out["log_w"][0])


def test_real_dense_spheres_with_dead_chains():
    # sigma > b makes dead ends frequent
    out, s, exact = _real_case(40, 4, 3_000, 13, b=1.0, sigma=1.4)
    assert (out["n_grown"].view(np.uint16) < 40).sum() > 10
    assert exact


def test_empty_ensemble():
    out, s = _gpu("lattice", 16, 6, 0, 1, hist_bins=16)
    assert s["n_chains"] == 0 and s["n_alive"] == 0 and s["log_c_est"] == -math.inf
    assert out["hist_n"].sum() == 0


def test_split_ranges_equal_one_launch_and_determinism():
    M = 10_000
    full, s_full = _gpu("lattice", 64, 6, M, 21, coord="i16", hist_bins=64)
    again, s_again = _gpu("lattice", 64, 6, M, 21, coord="i16", hist_bins=64)
    for key in full:
        np.testing.assert_array_equal(full[key], again[key])
    assert s_full == s_again
    a, _ = _gpu("lattice", 64, 6, 4_321, 21, coord="i16")
    b, _ = _gpu("lattice", 64, 6, M - 4_321, 21, coord="i16", chain_offset=4_321)
    for key in ("log_w", "r2", "rg2", "n2rg2", "n_grown"):
        np.testing.assert_array_equal(np.concatenate([a[key], b[key]]), full[key])
    np.testing.assert_array_equal(np.concatenate([a["r_end"], b["r_end"]], axis=1), full["r_end"])
    ra, _ = _gpu("real", 40, 8, 3_000, 22)
    rb, _ = _gpu("real", 40, 8, 3_000, 22)
    for key in ra:
        np.testing.assert_array_equal(ra[key], rb[key])


def test_kernel_timing_counts_growth_launches():
    rs.kernel_time()
    rs.kernel_timing(True)
    try:
        _gpu("lattice", 64, 6, 50_000, 3, coord="i16")
        _gpu("real", 24, 8, 2_000, 3)
        _gpu("lattice", 16, 6, 0, 3)  # empty: no growth launch, no pair
    finally:
        rs.kernel_timing(False)
    ms, n = rs.kernel_time()
    assert n == 2 and 0.0 < ms < 10_000.0
    _gpu("lattice", 16, 6, 1_000, 3)  # timing off: nothing recorded
    assert rs.kernel_time() == (0.0, 0)


def _sampled_indices(M, n, seed):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([np.arange(0, M, max(1, M // n)), rng.integers(0, M, n),
                                    [0, M - 1]]))
    return idx


def test_headline_lattice_n64_sampled():
    """Full-size lattice workload: sampled chains against the oracle chain by
    chain, and the full reduction against the oracle's reduction of the same
    per-chain outputs."""
    w = WORKLOADS["lattice_n64"]
    out, s = _gpu(w["geometry"], w["N"], w["k"], w["n_chains"], w["seed"], coord=w["coord"],
                  hist_bins=w["hist_bins"])
    M, N = w["n_chains"], w["N"]
    idx = _sampled_indices(M, 1500, 99)
    for c in idx:
        ch = oracle.lattice_chain(w["seed"], int(c), N)
        assert out["log_w"][c] == ch["log_w"]
        assert int(out["n_grown"].view(np.uint16)[c]) == ch["n_grown"]
        assert tuple(int(v) for v in out["r_end"][:, c]) == tuple(int(v) for v in ch["end"])
        assert out["n2rg2"][c] == ch["n2rg2"]
        assert out["rg2"][c] == ch["rg2"]
    red = oracle.reduce(N, out["log_w"], out["r2"], out["rg2"],
                        out["n_grown"].view(np.uint16).astype(np.int32), bins=w["hist_bins"])
    _check_summary(s, red, M)
    np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
    np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)
    assert s["n_alive"] > 0.9 * M


def test_headline_real_n64_sampled():
    """Full-size hard-sphere workload: sampled chains against the oracle
    chain by chain, bit for bit (log W, R^2, Rg^2, end vector, monomers
    placed), and the full reduction against the oracle's reduction of the
    same per-chain outputs."""
    w = WORKLOADS["real_n64"]
    out, s = _gpu(w["geometry"], w["N"], w["k"], w["n_chains"], w["seed"],
                  bond_length=w["bond_length"], bead_diameter=w["bead_diameter"],
                  hist_bins=w["hist_bins"])
    M, N, k = w["n_chains"], w["N"], w["k"]
    idx = _sampled_indices(M, 400, 98)
    for c in idx:
        ch = oracle.real_chain(w["seed"], int(c), N, k)
        assert int(out["n_grown"].view(np.uint16)[c]) == ch["n_grown"], c
        assert out["log_w"][c] == ch["log_w"], c
        assert out["r2"][c] == ch["r2"], c
        assert out["rg2"][c] == ch["rg2"], c
        assert tuple(float(v) for v in out["r_end"][:, c]) == tuple(float(v) for v in ch["end"]), c
    red = oracle.reduce(N, out["log_w"], out["r2"], out["rg2"],
                        out["n_grown"].view(np.uint16).astype(np.int32), bins=w["hist_bins"])
    _check_summary(s, red, M)
    np.testing.assert_array_equal(out["hist_n"], red["hist_n"])
    np.testing.assert_allclose(out["hist_w"], red["hist_w"], rtol=RTOL_SUM, atol=0)


def test_headline_lattice_n16_full():
    w = WORKLOADS["lattice_n16"]
    _lattice_case(w["N"], w["n_chains"], w["seed"], coord=w["coord"], exact_w=True)


def _within_3_sigma(g, r, keys=("r2", "rg2")):
    for key in keys:
        d = g[f"{key}_mean"] - r[f"{key}_mean"]
        se = math.hypot(g[f"{key}_err"], r[f"{key}_err"])
        assert abs(d) < 3 * se, (key, d, se)
    d = g["log_c_est"] - r["log_c_est"]
    assert abs(d) < 3 * math.hypot(g["c_rel_err"], r["c_rel_err"]), ("log_c_est", d)


def test_ensemble_averages_agree_within_3_sigma():
    """Independent seeds: GPU and oracle ensembles are statistically equal
    (weighted <R^2>, <Rg^2> of Eq. 2 and the c estimate of Eq. 6), at the
    headline shapes: hard spheres N = 64, k = 8 and the lattice N = 64."""
    w = WORKLOADS["real_n64"]
    _, g = _gpu("real", w["N"], w["k"], w["n_chains"], 31)
    ref = oracle.gen_real(32, w["N"], w["k"], 60_000)
    r = oracle.reduce(w["N"], ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"])
    _within_3_sigma(g, r)
    _, g = _gpu("lattice", 64, 6, 1_000_000, 33, coord="i16")
    ref = oracle.gen_lattice(34, 64, 100_000)
    r = oracle.reduce(64, ref["log_w"], ref["r2"], ref["rg2"], ref["n_grown"])
    _within_3_sigma(g, r)
