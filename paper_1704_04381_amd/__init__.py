"""Python binding of librsaw: Rosenbluth chain growth on MI355X.

Argument marshalling only.  Every step of the method runs in the HIP kernels
of ``librsaw.so`` behind the C ABI in ``include/rsaw.h``; PyTorch provides
device memory and the stream.  There is no CPU fallback: without the built
library (``python -m paper_1704_04381_amd.build``) or without a GPU, the calls
raise.

    out, summary = gen_chains("lattice", N=64, k=6, n_chains=10**7, seed=1,
                              coord="i16", hist_bins=256)
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsaw.so")

RSAW_LATTICE_SC = 0
RSAW_REAL_HS = 1
RSAW_LATTICE_26 = 2
GEOMETRIES = {"lattice": RSAW_LATTICE_SC, "real": RSAW_REAL_HS, "lattice26": RSAW_LATTICE_26}
RSAW_I16, RSAW_I32, RSAW_F64 = 0, 1, 2
RSAW_EXACT_W = 1
RSAW_RESTART = 2

STATUS = {0: "RSAW_OK", 1: "RSAW_E_INVALID", 2: "RSAW_E_UNSUPPORTED", 3: "RSAW_E_OVERFLOW",
          4: "RSAW_E_NOMEM", 5: "RSAW_E_DEVICE", 6: "RSAW_E_RNG"}


class rsaw_config(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("n_monomers", C.c_int32), ("k_trials", C.c_int32),
                ("coord_type", C.c_int32), ("n_chains", C.c_uint64), ("seed", C.c_uint64),
                ("chain_offset", C.c_uint64), ("bond_length", C.c_double),
                ("bead_diameter", C.c_double), ("hist_bins", C.c_int32), ("flags", C.c_uint32)]


class rsaw_chain_out(C.Structure):
    _fields_ = [("log_w", C.c_void_p), ("w_exact", C.c_void_p), ("r_end", C.c_void_p),
                ("r2", C.c_void_p), ("rg2", C.c_void_p), ("n2rg2", C.c_void_p),
                ("n_grown", C.c_void_p)]


class rsaw_summary(C.Structure):
    _fields_ = [("n_chains", C.c_uint64), ("n_alive", C.c_uint64), ("log_w_max", C.c_double),
                ("sum_w", C.c_double), ("sum_w2", C.c_double), ("sum_w_r2", C.c_double),
                ("sum_w2_r2", C.c_double), ("sum_w2_r2sq", C.c_double), ("sum_w_rg2", C.c_double),
                ("sum_w2_rg2", C.c_double), ("sum_w2_rg2sq", C.c_double),
                ("log_c_est", C.c_double), ("c_rel_err", C.c_double), ("r2_mean", C.c_double),
                ("r2_err", C.c_double), ("rg2_mean", C.c_double), ("rg2_err", C.c_double),
                ("ess", C.c_double), ("steps", C.c_double),
                ("sum_w_exact", C.c_uint64 * 2), ("sum_w_r2_exact", C.c_uint64 * 2),
                ("sum_w_n2rg2_exact", C.c_uint64 * 2), ("exact_valid", C.c_int32),
                ("status", C.c_int32)]


SUMMARY_BYTES = C.sizeof(rsaw_summary)


class rsaw_server_params(C.Structure):
    _fields_ = [("bytes_per_stream", C.c_uint64), ("max_batch", C.c_int32), ("streams", C.c_int32),
                ("large_ms", C.c_double)]

class rsaw_mapping(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("k_trials", C.c_int32), ("n_lo", C.c_int32), ("n_hi", C.c_int32),
                ("lanes", C.c_int32), ("threads", C.c_int32), ("lds_bytes", C.c_uint64)]


# Every symbol include/rsaw.h declares.
EXPORTS = ["rsaw_gen_chains", "rsaw_gen_chains_sync", "rsaw_gen_batch", "rsaw_server_create",
           "rsaw_server_submit", "rsaw_server_poll", "rsaw_server_wait", "rsaw_server_destroy",
           "rsaw_status_string",
           "rsaw_last_error", "rsaw_version", "rsaw_kernel_timing", "rsaw_kernel_time",
           "rsaw_workspace_size", "rsaw_mapping_set", "rsaw_mapping_clear", "rsaw_mapping_list", "rsaw_mapping_query",
           "rsaw_autotune", "rsaw_batch_plan_create", "rsaw_batch_plan_launch", "rsaw_batch_plan_destroy",
           "rsaw_set_workspace", "rsaw_fp64_check", "rsaw_gen_chains_static", "rsaw_shutdown",
           "rsaw_set_byte_box"]

_lib = None
_lock = threading.Lock()


class RsawError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load librsaw.so and declare the C ABI; raises if it was not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RsawError(5, f"{path} is missing: build it with "
                               "`python -m paper_1704_04381_amd.build`")
        lib = C.CDLL(path)
        vp = C.c_void_p
        lib.rsaw_gen_chains.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out),
                                        vp, vp, vp, vp]
        lib.rsaw_gen_chains.restype = C.c_int
        lib.rsaw_gen_chains_static.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out),
                                               vp, vp, vp, vp]
        lib.rsaw_gen_chains_static.restype = C.c_int
        lib.rsaw_gen_chains_sync.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out),
                                             C.POINTER(rsaw_summary), vp, vp, vp]
        lib.rsaw_gen_chains_sync.restype = C.c_int
        lib.rsaw_gen_batch.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out), C.c_int32,
                                       vp, C.POINTER(vp), C.POINTER(vp), vp]
        lib.rsaw_gen_batch.restype = C.c_int
        lib.rsaw_server_create.argtypes = [C.POINTER(rsaw_server_params), C.c_int32, C.POINTER(vp)]
        lib.rsaw_server_create.restype = C.c_int
        lib.rsaw_server_submit.argtypes = [vp, C.POINTER(rsaw_config), C.POINTER(C.c_uint64)]
        lib.rsaw_server_submit.restype = C.c_int
        lib.rsaw_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(rsaw_summary),
                                         C.POINTER(C.c_double)]
        lib.rsaw_server_poll.restype = C.c_int
        lib.rsaw_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(rsaw_summary), C.POINTER(C.c_double)]
        lib.rsaw_server_wait.restype = C.c_int
        lib.rsaw_server_destroy.argtypes = [vp]
        lib.rsaw_server_destroy.restype = None
        lib.rsaw_status_string.argtypes = [C.c_int]
        lib.rsaw_status_string.restype = C.c_char_p
        lib.rsaw_last_error.argtypes = []
        lib.rsaw_last_error.restype = C.c_char_p
        lib.rsaw_version.argtypes = []
        lib.rsaw_version.restype = C.c_int32
        lib.rsaw_kernel_timing.argtypes = [C.c_int32]
        lib.rsaw_kernel_timing.restype = C.c_int
        lib.rsaw_kernel_time.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        lib.rsaw_kernel_time.restype = C.c_int
        lib.rsaw_shutdown.argtypes = []
        lib.rsaw_shutdown.restype = None
        lib.rsaw_workspace_size.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out), C.c_int32,
                                            C.POINTER(C.c_size_t)]
        lib.rsaw_workspace_size.restype = C.c_int
        lib.rsaw_mapping_set.argtypes = [C.POINTER(rsaw_mapping)]
        lib.rsaw_mapping_set.restype = C.c_int
        lib.rsaw_mapping_clear.argtypes = []
        lib.rsaw_mapping_clear.restype = None
        lib.rsaw_set_byte_box.argtypes = [C.c_int32]
        lib.rsaw_set_byte_box.restype = C.c_int
        lib.rsaw_mapping_list.argtypes = [C.POINTER(rsaw_mapping), C.c_int32, C.POINTER(C.c_int32)]
        lib.rsaw_mapping_list.restype = C.c_int
        lib.rsaw_mapping_query.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_mapping)]
        lib.rsaw_mapping_query.restype = C.c_int
        lib.rsaw_autotune.argtypes = [C.POINTER(rsaw_config), C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                      C.POINTER(rsaw_mapping), C.POINTER(C.c_double), vp]
        lib.rsaw_autotune.restype = C.c_int
        lib.rsaw_batch_plan_create.argtypes = [C.POINTER(rsaw_config), C.POINTER(rsaw_chain_out), C.c_int32,
                                               vp, vp, vp, C.POINTER(vp)]
        lib.rsaw_batch_plan_create.restype = C.c_int
        lib.rsaw_batch_plan_launch.argtypes = [vp, vp]
        lib.rsaw_batch_plan_launch.restype = C.c_int
        lib.rsaw_batch_plan_destroy.argtypes = [vp]
        lib.rsaw_batch_plan_destroy.restype = None
        lib.rsaw_set_workspace.argtypes = [vp, C.c_size_t, vp]
        lib.rsaw_set_workspace.restype = C.c_int
        lib.rsaw_fp64_check.argtypes = [vp, vp, vp, vp, C.c_uint64, vp]
        lib.rsaw_fp64_check.restype = C.c_int
        _lib = lib
        return lib


def _check(status):
    if status != 0:
        raise RsawError(status, load().rsaw_last_error().decode())


def make_config(geometry, N, k, n_chains, seed, *, coord=None, chain_offset=0,
                bond_length=1.0, bead_diameter=1.0, hist_bins=0, exact_w=False, restart=False):
    geo = GEOMETRIES[geometry] if isinstance(geometry, str) else int(geometry)
    if coord is None:
        coord = "f64" if geo == RSAW_REAL_HS else "i32"
    ct = {"i16": RSAW_I16, "i32": RSAW_I32, "f64": RSAW_F64}[coord]
    return rsaw_config(geo, int(N), int(k), ct, int(n_chains), int(seed), int(chain_offset),
                       float(bond_length), float(bead_diameter), int(hist_bins),
                       (RSAW_EXACT_W if exact_w else 0) | (RSAW_RESTART if restart else 0))


def summary_to_dict(s: rsaw_summary) -> dict:
    d = {}
    for name, _ in rsaw_summary._fields_:
        v = getattr(s, name)
        if name.endswith("_exact"):
            v = int(v[0]) | (int(v[1]) << 64)
        d[name] = v
    return d


def parse_summary(buf) -> dict:
    """Summary dict from a device or host uint8 tensor of SUMMARY_BYTES."""
    raw = bytes(buf.cpu().numpy().tobytes())
    return summary_to_dict(rsaw_summary.from_buffer_copy(raw))


def gen_chains_raw(cfg: rsaw_config, out: rsaw_chain_out | None, d_summary: int,
                   d_hist_w: int, d_hist_n: int, stream: int):
    """Direct call of rsaw_gen_chains with raw device addresses (0 = NULL)."""
    lib = load()
    _check(lib.rsaw_gen_chains(C.byref(cfg), C.byref(out) if out is not None else None,
                               d_summary or None, d_hist_w or None, d_hist_n or None,
                               stream or None))


STATIC_SCRATCH_BYTES = 32 << 20


def gen_chains_static_raw(cfg: rsaw_config, out: rsaw_chain_out | None, d_summary: int,
                          d_hist_w: int, d_hist_n: int, stream: int):
    """Direct call of rsaw_gen_chains_static (the allocation-free variant of
    rsaw_gen_chains, workspace in the library's static device scratch) with
    raw device addresses (0 = NULL)."""
    lib = load()
    _check(lib.rsaw_gen_chains_static(C.byref(cfg), C.byref(out) if out is not None else None,
                                      d_summary or None, d_hist_w or None, d_hist_n or None,
                                      stream or None))


def _alloc_outputs(cfg: rsaw_config, dev, per_chain: bool, hist_bins: int):
    """Device tensors for one ensemble's per-chain outputs and histogram, and
    the rsaw_chain_out that points at them."""
    import torch

    M = int(cfg.n_chains)
    lattice = cfg.geometry != RSAW_REAL_HS
    out = {}
    o = rsaw_chain_out()
    if per_chain:
        ctype = {RSAW_I16: torch.int16, RSAW_I32: torch.int32, RSAW_F64: torch.float64}[cfg.coord_type]
        out["log_w"] = torch.empty(M, dtype=torch.float64, device=dev)
        out["r_end"] = torch.empty((3, M), dtype=ctype, device=dev)
        out["r2"] = torch.empty(M, dtype=torch.float64, device=dev)
        out["rg2"] = torch.empty(M, dtype=torch.float64, device=dev)
        out["n_grown"] = torch.empty(M, dtype=torch.int16, device=dev)  # uint16 bits
        o.log_w, o.r_end, o.r2, o.rg2, o.n_grown = (out[n].data_ptr() for n in
                                                      ("log_w", "r_end", "r2", "rg2", "n_grown"))
        if lattice:
            out["n2rg2"] = torch.empty(M, dtype=torch.int64, device=dev)
            o.n2rg2 = out["n2rg2"].data_ptr()
            if cfg.flags & RSAW_EXACT_W:
                out["w_exact"] = torch.empty(M, dtype=torch.uint64, device=dev)
                o.w_exact = out["w_exact"].data_ptr()
    if hist_bins:
        out["hist_w"] = torch.empty(hist_bins, dtype=torch.float64, device=dev)
        out["hist_n"] = torch.empty(hist_bins, dtype=torch.uint64, device=dev)
    return out, o


def _device(device):
    import torch

    if not torch.cuda.is_available():
        raise RsawError(5, "no GPU: librsaw runs on MI355X only (no CPU fallback)")
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


def gen_chains(geometry, N, k, n_chains, seed, *, coord=None, chain_offset=0,
               bond_length=1.0, bead_diameter=1.0, hist_bins=0, exact_w=False, restart=False,
               per_chain=True, device=None, stream=None, sync=True):
    """Grow ``n_chains`` chains on the GPU and reduce them.

    Returns ``(out, summary)``: ``out`` is a dict of device tensors (log_w,
    r_end [3, M], r2, rg2, n_grown, and n2rg2 / w_exact on the lattice), empty
    when ``per_chain`` is false; ``summary`` is a dict (host) when ``sync`` is
    true, else the raw device uint8 tensor (parse with ``parse_summary``).
    """
    import torch

    dev = _device(device)
    cfg = make_config(geometry, N, k, n_chains, seed, coord=coord, chain_offset=chain_offset,
                      bond_length=bond_length, bead_diameter=bead_diameter,
                      hist_bins=hist_bins, exact_w=exact_w, restart=restart)
    out, o = _alloc_outputs(cfg, dev, per_chain, hist_bins)
    summ = torch.empty(SUMMARY_BYTES, dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        gen_chains_raw(cfg, o, summ.data_ptr(), out["hist_w"].data_ptr() if hist_bins else 0,
                       out["hist_n"].data_ptr() if hist_bins else 0, stream)
    if not sync:
        return out, summ
    s = parse_summary(summ)
    if s["status"] != 0:
        raise RsawError(s["status"], "device reported a rejection-cap hit")
    return out, s


def gen_batch_raw(cfgs, outs, d_summaries: int, hist_w=None, hist_n=None, stream: int = 0):
    """Direct call of rsaw_gen_batch: lists of configs and chain-out structs,
    a device address of len(cfgs) summaries (0 = none), and optional lists of
    per-ensemble histogram device addresses (0 = NULL)."""
    lib = load()
    n = len(cfgs)
    carr = (rsaw_config * max(n, 1))(*cfgs)
    oarr = (rsaw_chain_out * max(n, 1))(*outs) if outs is not None else None
    hw = (C.c_void_p * max(n, 1))(*[p or None for p in hist_w]) if hist_w is not None else None
    hn = (C.c_void_p * max(n, 1))(*[p or None for p in hist_n]) if hist_n is not None else None
    _check(lib.rsaw_gen_batch(carr, oarr, n, d_summaries or None, hw, hn, stream or None))


def gen_batch(specs, *, per_chain=True, device=None, stream=None, sync=True):
    """Grow and reduce several ensembles with one rsaw_gen_batch call.

    ``specs`` is a list of dicts with the arguments of ``gen_chains``
    (geometry, N, k, n_chains, seed and the optional keywords).  Returns a
    list of ``(out, summary)`` pairs as ``gen_chains`` does; with ``sync``
    false the summaries are the raw device tensor of all of them.
    """
    import torch

    dev = _device(device)
    cfgs, outs, allocs = [], [], []
    for sp in specs:
        sp = dict(sp)
        bins = int(sp.get("hist_bins", 0))
        cfg = make_config(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                          sp.pop("seed"), **sp)
        out, o = _alloc_outputs(cfg, dev, per_chain, bins)
        cfgs.append(cfg)
        outs.append(o)
        allocs.append(out)
    n = len(cfgs)
    summ = torch.empty(max(n, 1) * SUMMARY_BYTES, dtype=torch.uint8, device=dev)
    hist_w = [a["hist_w"].data_ptr() if "hist_w" in a else 0 for a in allocs]
    hist_n = [a["hist_n"].data_ptr() if "hist_n" in a else 0 for a in allocs]
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        gen_batch_raw(cfgs, outs, summ.data_ptr(), hist_w, hist_n, stream)
    if not sync:
        return allocs, summ
    res = []
    for i, out in enumerate(allocs):
        s = parse_summary(summ[i * SUMMARY_BYTES:(i + 1) * SUMMARY_BYTES])
        if s["status"] != 0:
            raise RsawError(s["status"], f"ensemble {i}: device reported a rejection-cap hit")
        res.append((out, s))
    return res


class BatchPlan:
    """A batch prepared once (rsaw_batch_plan_create) and launched any number
    of times with kernel launches only (rsaw_batch_plan_launch), e.g. inside
    a torch.cuda.graph capture.  ``specs`` as for ``gen_batch``; the outputs
    are allocated here and rewritten by every launch."""

    def __init__(self, specs, *, per_chain=True, device=None):
        import torch

        dev = _device(device)
        self._lib = load()
        cfgs, outs, self.outputs = [], [], []
        for sp in specs:
            sp = dict(sp)
            bins = int(sp.get("hist_bins", 0))
            cfg = make_config(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                              sp.pop("seed"), **sp)
            out, o = _alloc_outputs(cfg, dev, per_chain, bins)
            cfgs.append(cfg)
            outs.append(o)
            self.outputs.append(out)
        n = len(cfgs)
        self.n = n
        self.summaries = torch.empty(max(n, 1) * SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        carr = (rsaw_config * max(n, 1))(*cfgs)
        oarr = (rsaw_chain_out * max(n, 1))(*outs)
        hw = (C.c_void_p * max(n, 1))(*[a["hist_w"].data_ptr() if "hist_w" in a else None for a in self.outputs])
        hn = (C.c_void_p * max(n, 1))(*[a["hist_n"].data_ptr() if "hist_n" in a else None for a in self.outputs])
        self._h = C.c_void_p()
        with torch.cuda.device(dev):
            _check(self._lib.rsaw_batch_plan_create(carr, oarr, n, C.c_void_p(self.summaries.data_ptr()),
                                                    C.cast(hw, C.c_void_p), C.cast(hn, C.c_void_p),
                                                    C.byref(self._h)))
        self.device = dev

    def launch(self, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(self._lib.rsaw_batch_plan_launch(self._h, C.c_void_p(stream)))

    def results(self):
        """(out, summary) per ensemble, after the last launch has finished."""
        res = []
        for i, out in enumerate(self.outputs):
            res.append((out, parse_summary(self.summaries[i * SUMMARY_BYTES:(i + 1) * SUMMARY_BYTES])))
        return res

    def close(self):
        if self._h:
            self._lib.rsaw_batch_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop of librsaw (rsaw_server_*): submit ensembles, take their
    summaries.  Each result equals a stand-alone gen_chains call."""

    def __init__(self, bytes_per_stream=2 << 30, max_batch=256, streams=2, device=0, large_ms=0.0):
        lib = load()
        self._lib = lib
        p = rsaw_server_params(int(bytes_per_stream), int(max_batch), int(streams), float(large_ms))
        h = C.c_void_p()
        _check(lib.rsaw_server_create(C.byref(p), int(device), C.byref(h)))
        self._h = h

    def submit(self, geometry, N, k, n_chains, seed, **kw) -> int:
        cfg = make_config(geometry, N, k, n_chains, seed, **kw)
        t = C.c_uint64()
        _check(self._lib.rsaw_server_submit(self._h, C.byref(cfg), C.byref(t)))
        return t.value

    def _result(self, st, summ, times):
        if st != 0:
            raise RsawError(st, self._lib.rsaw_last_error().decode())
        d = summary_to_dict(summ)
        d["queue_us"], d["latency_us"] = times[0], times[1]
        return d

    def poll(self, ticket):
        """Summary dict (with queue_us and latency_us) or None while running."""
        done = C.c_int32()
        summ = rsaw_summary()
        times = (C.c_double * 2)()
        st = self._lib.rsaw_server_poll(self._h, ticket, C.byref(done), C.byref(summ), times)
        if not done.value:
            _check(st)
            return None
        return self._result(st, summ, times)

    def wait(self, ticket):
        summ = rsaw_summary()
        times = (C.c_double * 2)()
        st = self._lib.rsaw_server_wait(self._h, ticket, C.byref(summ), times)
        return self._result(st, summ, times)

    def close(self):
        if self._h:
            self._lib.rsaw_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def version() -> int:
    return int(load().rsaw_version())


def kernel_timing(enable: bool) -> None:
    """Switch growth-kernel event timing on or off (rsaw_kernel_timing)."""
    _check(load().rsaw_kernel_timing(1 if enable else 0))


def kernel_time() -> tuple[float, int]:
    """(summed ms, launches) of the growth kernels timed since the last read."""
    ms = C.c_double(0.0)
    n = C.c_uint64(0)
    _check(load().rsaw_kernel_time(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def shutdown():
    load().rsaw_shutdown()


def workspace_size(cfg: rsaw_config, out: rsaw_chain_out | None = None, reduce: bool = True) -> int:
    """Device workspace bytes an rsaw_gen_chains call with these arguments
    needs (rsaw_workspace_size; a host-only query)."""
    n = C.c_size_t(0)
    _check(load().rsaw_workspace_size(C.byref(cfg), C.byref(out) if out is not None else None,
                                      1 if reduce else 0, C.byref(n)))
    return n.value


def set_workspace(ptr: int, nbytes: int, stream: int = 0) -> None:
    """Bind caller-owned device memory (address ``ptr``, ``nbytes``; 0
    unbinds) as the workspace of (current device, stream)
    (rsaw_set_workspace)."""
    _check(load().rsaw_set_workspace(ptr or None, int(nbytes), stream or None))


def fp64_check(a, b, stream=None):
    """Device sqrt(a) and a / b (rsaw_fp64_check) for float64 device tensors
    of equal length; returns (sqrt, quotient) tensors."""
    import torch

    a = a.contiguous()
    b = b.contiguous()
    if a.dtype != torch.float64 or b.dtype != torch.float64 or a.numel() != b.numel():
        raise RsawError(1, "fp64_check needs two float64 tensors of equal length")
    sq = torch.empty_like(a)
    dv = torch.empty_like(a)
    if stream is None:
        stream = torch.cuda.current_stream(a.device).cuda_stream
    with torch.cuda.device(a.device):
        _check(load().rsaw_fp64_check(a.data_ptr(), b.data_ptr(), sq.data_ptr(), dv.data_ptr(),
                                      a.numel(), stream or None))
    return sq, dv


def _mapping_dict(m: rsaw_mapping) -> dict:
    return {name: getattr(m, name) for name, _ in rsaw_mapping._fields_}


def mapping_set(geometry, k, n_lo, n_hi, lanes, threads) -> None:
    """Install a lane mapping for (geometry, k, N in [n_lo, n_hi])
    (rsaw_mapping_set; host-only)."""
    geo = GEOMETRIES[geometry] if isinstance(geometry, str) else int(geometry)
    m = rsaw_mapping(geo, int(k), int(n_lo), int(n_hi), int(lanes), int(threads), 0)
    _check(load().rsaw_mapping_set(C.byref(m)))


def mapping_clear() -> None:
    """Empty the tuning table (rsaw_mapping_clear)."""
    load().rsaw_mapping_clear()


def set_byte_box(edge: int) -> None:
    """|coordinate| at which the one-word lattice kernels regrow a chain in
    two-word format (rsaw_set_byte_box; 1..127 lowers every format's edge,
    0 restores each format's own).  Results do not depend on it."""
    _check(load().rsaw_set_byte_box(int(edge)))


def mapping_list() -> list[dict]:
    """The tuning table, oldest entry first (rsaw_mapping_list)."""
    lib = load()
    n = C.c_int32(0)
    _check(lib.rsaw_mapping_list(None, 0, C.byref(n)))
    arr = (rsaw_mapping * max(n.value, 1))()
    _check(lib.rsaw_mapping_list(arr, n.value, C.byref(n)))
    return [_mapping_dict(arr[i]) for i in range(min(n.value, len(arr)))]


def save_mappings(path) -> int:
    """Write the tuning table to a JSON autotune cache; returns the number
    of entries."""
    import json

    rows = [{k: v for k, v in m.items() if k != "lds_bytes"} for m in mapping_list()]
    with open(path, "w") as f:
        json.dump({"rsaw_mappings": rows, "version": version()}, f, indent=1)
    return len(rows)


def load_mappings(path) -> int:
    """Add the entries of a JSON autotune cache to the tuning table, in their
    saved order (each validated by rsaw_mapping_set); returns their number."""
    import json

    with open(path) as f:
        rows = json.load(f)["rsaw_mappings"]
    for r in rows:
        mapping_set(r["geometry"], r["k_trials"], r["n_lo"], r["n_hi"], r["lanes"], r["threads"])
    return len(rows)


def mapping_query(cfg: rsaw_config) -> dict:
    """The mapping a call with cfg would launch with (rsaw_mapping_query;
    host-only)."""
    m = rsaw_mapping()
    _check(load().rsaw_mapping_query(C.byref(cfg), C.byref(m)))
    return _mapping_dict(m)


def autotune(geometry, k, n_edges, n_chains, *, seed=1, reps=3, stream=None, **cfg_kw) -> list[dict]:
    """Time every legal lane mapping at each bucket edge and install the
    fastest (rsaw_autotune).  Returns one dict per bucket: the chosen
    mapping plus its mean time per call, `ms`."""
    import torch

    edges = [int(n) for n in n_edges]
    cfg = make_config(geometry, edges[-1], k, n_chains, seed, **cfg_kw)
    arr = (C.c_int32 * len(edges))(*edges)
    chosen = (rsaw_mapping * len(edges))()
    ms = (C.c_double * len(edges))()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(load().rsaw_autotune(C.byref(cfg), arr, len(edges), int(reps), chosen, ms, C.c_void_p(stream)))
    return [dict(_mapping_dict(chosen[i]), ms=ms[i]) for i in range(len(edges))]
