"""Plain CPU oracle for Rosenbluth chain growth (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
it; the oracle shares no code with the HIP library.

The C source (``rsaw_oracle.c``) follows the paper's growth rules
(Sec. 3.3.2 / Algorithm 1 for the cubic lattice, Sec. 3.3.3 / Algorithm 2 for
hard spheres in continuous space), the Rosenbluth weight of Eq. (3) and the
weighted averages of Eqs. (2) and (6).  This module only marshals numpy
arrays in and out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsaw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "librsaw_oracle.so")
_lib = None
_lock = threading.Lock()

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-msse2", "-mfpmath=sse", "-Wall"]

REDUCE_FIELDS = [
    "M", "alive", "log_w_max", "sum_w", "sum_w2",
    "sum_w_r2", "sum_w2_r2", "sum_w2_r2sq",
    "sum_w_rg2", "sum_w2_rg2", "sum_w2_rg2sq",
    "log_c_est", "c_rel_err", "r2_mean", "r2_err", "rg2_mean", "rg2_err",
    "ess", "steps",
]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/librsaw_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = C.CDLL(_LIB_PATH)
        u64, i32, dbl, vp = C.c_uint64, C.c_int32, C.c_double, C.c_void_p
        lib.oro_philox4x32_10.argtypes = [vp, u64, vp]
        lib.oro_philox4x32_10.restype = None
        lib.oro_lattice_chain.argtypes = [u64, u64, i32] + [vp] * 10 + [i32, vp]
        lib.oro_lattice_chain.restype = C.c_int
        lib.oro_real_chain.argtypes = [u64, u64, i32, i32, dbl, dbl] + [vp] * 7 + [i32, vp]
        lib.oro_real_chain.restype = C.c_int
        lib.oro_unit_vector.argtypes = [u64, u64, C.c_uint32, C.c_uint32, vp, vp]
        lib.oro_unit_vector.restype = C.c_int
        lib.oro_overlaps.argtypes = [vp, vp, dbl]
        lib.oro_overlaps.restype = C.c_int
        lib.oro_gen_lattice.argtypes = [u64, u64, u64, i32] + [vp] * 8 + [i32]
        lib.oro_gen_lattice.restype = C.c_int
        lib.oro_gen_real.argtypes = [u64, u64, u64, i32, i32, dbl, dbl] + [vp] * 5 + [i32]
        lib.oro_gen_real.restype = C.c_int
        lib.oro_reduce.argtypes = [u64, i32, vp, vp, vp, vp, i32, vp, vp, vp]
        lib.oro_reduce.restype = None
        lib.oro_reduce_exact.argtypes = [u64, vp, vp, vp, vp]
        lib.oro_reduce_exact.restype = None
        lib.oro_lemire16.argtypes = [C.c_uint32, C.c_uint32, vp]
        lib.oro_lemire16.restype = C.c_int
        lib.oro_pick.argtypes = [u64, u64, C.c_uint32, C.c_uint32, vp, vp]
        lib.oro_pick.restype = C.c_int
        _lib = lib
        return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(status, what):
    if status != 0:
        raise OracleError(f"{what} failed with status {status}")


def philox(counter, seed):
    """Philox4x32-10 of one 4x32-bit counter under the 64-bit key ``seed``."""
    lib = _load()
    ctr = np.asarray(counter, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib.oro_philox4x32_10(_p(ctr), C.c_uint64(seed), _p(out))
    return out


def lemire16(x, m):
    """Lemire acceptance of one 16-bit word for [0, m): index or None."""
    lib = _load()
    idx = np.zeros(1, dtype=np.uint32)
    return int(idx[0]) if lib.oro_lemire16(x, m, _p(idx)) else None


def pick(seed, chain, step, m):
    """(index, rejected half-words) of the uniform pick of step ``step``."""
    lib = _load()
    idx = np.zeros(1, dtype=np.uint32)
    rej = np.zeros(1, dtype=np.uint32)
    _check(lib.oro_pick(seed, chain, step, m, _p(idx), _p(rej)), "pick")
    return int(idx[0]), int(rej[0])


def unit_vector(seed, chain, step, trial):
    """Marsaglia unit vector of trial ``trial`` at step ``step``; (e, attempts)."""
    lib = _load()
    e = np.zeros(3)
    att = np.zeros(1, dtype=np.uint32)
    _check(lib.oro_unit_vector(seed, chain, step, trial, _p(e), _p(att)), "unit_vector")
    return e, int(att[0])


def overlaps(c, r, sigma2):
    lib = _load()
    c = np.ascontiguousarray(c, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return bool(lib.oro_overlaps(_p(c), _p(r), sigma2))


RESTART = 2  # flag: a dead end restarts the chain with the next round of random numbers
Z26 = 4      # flag: lattice with the 26 neighbours of the tip as candidates


def lattice_chain(seed, chain, N, restart=False, z26=False):
    """One lattice chain with its coordinates and the m_i sequence (of the
    final growth attempt); ``rounds`` counts the attempts."""
    lib = _load()
    xyz = np.zeros((N, 3), dtype=np.int32)
    mseq = np.zeros(N, dtype=np.int32)
    lw = np.zeros(1); we = np.zeros(1, np.uint64); ok = np.zeros(1, np.int32)
    flags = (RESTART if restart else 0) | (Z26 if z26 else 0)
    g = np.zeros(1, np.int32); e = np.zeros(3, np.int32)
    r2 = np.zeros(1, np.int64); nn = np.zeros(1, np.int64); rg = np.zeros(1)
    rounds = np.zeros(1, np.int32)
    _check(lib.oro_lattice_chain(seed, chain, N, _p(xyz), _p(mseq), _p(lw), _p(we),
                                 _p(ok), _p(g), _p(e), _p(r2), _p(nn), _p(rg),
                                 flags, _p(rounds)),
           "lattice_chain")
    n = int(g[0])
    return dict(xyz=xyz[:n], m=mseq, log_w=float(lw[0]), w_exact=int(we[0]),
                w_exact_ok=bool(ok[0]), n_grown=n, end=e, r2=int(r2[0]),
                n2rg2=int(nn[0]), rg2=float(rg[0]), rounds=int(rounds[0]))


def real_chain(seed, chain, N, k, b=1.0, sigma=1.0, restart=False):
    """One hard-sphere chain with its coordinates and the m_i sequence (of the
    final growth attempt); ``rounds`` counts the attempts."""
    lib = _load()
    xyz = np.zeros((N, 3))
    mseq = np.zeros(N, dtype=np.int32)
    lw = np.zeros(1); g = np.zeros(1, np.int32); e = np.zeros(3)
    r2 = np.zeros(1); rg = np.zeros(1)
    rounds = np.zeros(1, np.int32)
    _check(lib.oro_real_chain(seed, chain, N, k, b, sigma, _p(xyz), _p(mseq), _p(lw),
                              _p(g), _p(e), _p(r2), _p(rg), RESTART if restart else 0,
                              _p(rounds)), "real_chain")
    n = int(g[0])
    return dict(xyz=xyz[:n], m=mseq, log_w=float(lw[0]), n_grown=n, end=e,
                r2=float(r2[0]), rg2=float(rg[0]), rounds=int(rounds[0]))


def gen_lattice(seed, N, n_chains, chain_offset=0, restart=False, z26=False):
    """Per-chain lattice outputs for chains chain_offset .. +n_chains-1."""
    lib = _load()
    n = int(n_chains)
    out = dict(log_w=np.zeros(n), w_exact=np.zeros(n, np.uint64),
               w_exact_ok=np.zeros(n, np.int32), r_end=np.zeros((3, n), np.int32),
               r2=np.zeros(n, np.int64), n2rg2=np.zeros(n, np.int64),
               rg2=np.zeros(n), n_grown=np.zeros(n, np.int32))
    _check(lib.oro_gen_lattice(seed, chain_offset, n, N, _p(out["log_w"]),
                               _p(out["w_exact"]), _p(out["w_exact_ok"]),
                               _p(out["r_end"]), _p(out["r2"]), _p(out["n2rg2"]),
                               _p(out["rg2"]), _p(out["n_grown"]),
                               (RESTART if restart else 0) | (Z26 if z26 else 0)),
           "gen_lattice")
    return out


def gen_real(seed, N, k, n_chains, b=1.0, sigma=1.0, chain_offset=0, restart=False):
    """Per-chain hard-sphere outputs for chains chain_offset .. +n_chains-1."""
    lib = _load()
    n = int(n_chains)
    out = dict(log_w=np.zeros(n), r_end=np.zeros((3, n)), r2=np.zeros(n),
               rg2=np.zeros(n), n_grown=np.zeros(n, np.int32))
    _check(lib.oro_gen_real(seed, chain_offset, n, N, k, b, sigma, _p(out["log_w"]),
                            _p(out["r_end"]), _p(out["r2"]), _p(out["rg2"]),
                            _p(out["n_grown"]), RESTART if restart else 0), "gen_real")
    return out


def reduce(N, log_w, r2, rg2, n_grown, bins=0):
    """Weighted ensemble averages (Eqs. 2 and 6) of per-chain outputs."""
    lib = _load()
    M = len(log_w)
    lw = np.ascontiguousarray(log_w, dtype=np.float64)
    a = np.ascontiguousarray(r2, dtype=np.float64)
    g = np.ascontiguousarray(rg2, dtype=np.float64)
    ng = np.ascontiguousarray(n_grown, dtype=np.int32)
    out = np.zeros(len(REDUCE_FIELDS))
    hw = np.zeros(bins) if bins > 0 else None
    hn = np.zeros(bins, np.uint64) if bins > 0 else None
    lib.oro_reduce(M, N, _p(lw), _p(a), _p(g), _p(ng), bins, _p(out), _p(hw), _p(hn))
    res = dict(zip(REDUCE_FIELDS, out.tolist()))
    res["M"] = int(res["M"]); res["alive"] = int(res["alive"])
    if bins > 0:
        res["hist_w"] = hw
        res["hist_n"] = hn
    return res


def reduce_exact(w_exact, r2, n2rg2):
    """Exact integer sums (sum W, sum W R2, sum W g^2 Rg2) as Python ints."""
    lib = _load()
    w = np.ascontiguousarray(w_exact, dtype=np.uint64)
    a = np.ascontiguousarray(r2, dtype=np.int64)
    g = np.ascontiguousarray(n2rg2, dtype=np.int64)
    out = np.zeros(6, np.uint64)
    lib.oro_reduce_exact(len(w), _p(w), _p(a), _p(g), _p(out))
    v = [int(x) for x in out]
    return dict(sum_w=v[0] | (v[1] << 64), sum_w_r2=v[2] | (v[3] << 64),
                sum_w_n2rg2=v[4] | (v[5] << 64))
