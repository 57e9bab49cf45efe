"""Device binary64 square root and division against the host.

The hard-sphere kernels reproduce the oracle bit for bit only if the device
sqrt (Marsaglia's q = 2 sqrt(1 - s), Sec. 3.3.3, with the kernels' own
routine on [2^-60, 1]) and division (centre of mass, Rg^2) are correctly
rounded, as the host's are (IEEE 754).  This runs
rsaw_fp64_check, compiled with the growth kernels' settings, on 2^21
inputs of each kind: the Marsaglia domain 1 - s for s in (0, 1) drawn as
the kernels draw it, uniform mantissas over many binades, the subnormal
range and edge values.  GPU test; calls the HIP library through its C ABI.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_04381_amd as rs

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    g = np.random.Generator(np.random.Philox(key=seed))
    # 1 - s with s = v1^2 + v2^2, v uniform 53-bit multiples of 2^-52 in [-1, 1)
    v = (g.integers(0, 1 << 53, size=(n, 2), dtype=np.int64) - (1 << 52)).astype(np.float64) * 2.0**-52
    s = v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]
    s = s[(s < 1.0) & (s > 0.0)]
    dom = 1.0 - s
    # random bit patterns of positive normal doubles over many binades
    e = g.integers(1023 - 200, 1023 + 200, size=n, dtype=np.uint64)
    m = g.integers(0, 1 << 52, size=n, dtype=np.uint64)
    wide = ((e << np.uint64(52)) | m).view(np.float64)
    sub = (g.integers(1, 1 << 52, size=n // 8, dtype=np.uint64)).view(np.float64)
    edge = np.array([0.0, 1.0, 2.0, 0.25, 1.0 - 2.0**-53, 1.0 + 2.0**-52, np.finfo(np.float64).tiny,
                     np.finfo(np.float64).max, 5e-324, 4.0, 9.0, 1e300, 1e-300])
    # the domain [2^-60, 1] of the hard-sphere kernels' own square root,
    # uniform mantissas in every binade, and its end points
    e2 = g.integers(1023 - 60, 1023, size=n // 4, dtype=np.uint64)
    m2 = g.integers(0, 1 << 52, size=n // 4, dtype=np.uint64)
    unit = np.concatenate([((e2 << np.uint64(52)) | m2).view(np.float64),
                           np.array([2.0**-60, 2.0**-53, 0.5, 1.0 - 2.0**-53])])
    a = np.concatenate([dom, wide, sub, edge, unit])
    # divisors: sums of bead counts as the kernels divide by (1..16384), and
    # random doubles
    b = np.concatenate([g.integers(1, 16385, size=len(dom)).astype(np.float64),
                        wide[::-1].copy(), g.integers(1, 1 << 20, size=len(sub)).astype(np.float64),
                        np.array([1.0, 3.0, 7.0, 3.0, 3.0, 3.0, 3.0, 2.0, 3.0, 3.0, 3.0, 7.0, 7.0]),
                        g.integers(1, 16385, size=len(unit)).astype(np.float64)])
    return a, b


def test_device_sqrt_and_division_are_correctly_rounded():
    n = 1 << 21
    a, b = _inputs(n, 5)
    assert len(a) >= 10**6
    print(f"[gpu] fp64 check: {len(a)} inputs", flush=True)
    da = torch.from_numpy(a).cuda()
    db = torch.from_numpy(b).cuda()
    sq, dv = rs.fp64_check(da, db)
    torch.cuda.synchronize()
    sq, dv = sq.cpu().numpy(), dv.cpu().numpy()
    # host IEEE 754: sqrt and division are correctly rounded (numpy uses the
    # SSE2 instructions sqrtsd / divsd)
    want_sq = np.sqrt(a)
    want_dv = a / b
    bad_sq = np.flatnonzero(sq.view(np.uint64) != want_sq.view(np.uint64))
    bad_dv = np.flatnonzero(dv.view(np.uint64) != want_dv.view(np.uint64))
    assert bad_sq.size == 0, (a[bad_sq[:5]], sq[bad_sq[:5]], want_sq[bad_sq[:5]])
    assert bad_dv.size == 0, (a[bad_dv[:5]], b[bad_dv[:5]], dv[bad_dv[:5]], want_dv[bad_dv[:5]])
