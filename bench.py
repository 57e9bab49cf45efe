"""Benchmark of the Rosenbluth chain-growth hot path on one MI355X.

A step is one pass of the whole path over one ensemble: grow every chain
(draw, test, count, pick, weight, observables) and reduce the ensemble
(weighted averages, c_n estimate, R^2 histogram).  The headline workload is
the simple cubic lattice at N = 64 monomers, 10^7 chains, int16 coordinates,
FP64 log-weights and a 256-bin histogram; the hard-sphere N = 64, k = 8,
10^6-chain workload is reported beside it under "secondary", the
26-neighbour lattice at N = 64 and 10^7 chains under "variant", and a mixed
batch of 256 ensembles (one batched call against per-ensemble calls) under
"batch".

Prints one JSON line.  value = monomer-steps/s = M (N - 1) K / T with the
inputs (seed, configuration) resident before the timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

# VALU peaks from the unit counts and clock (256 CUs, 2.4 GHz) and the
# published vector rates: 32-bit operations at the fp32 vector rate
# (157.3 TFLOP/s counts an FMA as 2, so 128 lanes per CU per clock:
# 7.86e13 lane-operations/s), binary64 at the fp64 rate (64 lanes per CU per
# clock: 3.93e13).  The integer instructions that carry the lattice pair tests
# (v_msad_u8, clamped v_sub_u32, v_lshl_or_b32, v_dot4c/v_dot2c, v_sad_u16)
# were measured to issue at about 61 lanes per CU per clock, i.e. at the
# 64-lane rate, so the lattice kernels also report that attainable figure.
VALU_PEAK_INT32_TOPS = 256 * 128 * 2.4e9 / 1e12
VALU_PEAK_FP64_TOPS = 256 * 64 * 2.4e9 / 1e12
ATTAINABLE_INT_PATH_TOPS = VALU_PEAK_FP64_TOPS
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(REPO, "profiles", "grow_traffic.json")
CSRC = os.path.join(REPO, "paper_1704_04381_amd", "csrc")


def kernel_source_hash(kernel_file: str) -> str:
    """SHA-256 of one kernel source plus the shared device header."""
    import hashlib
    h = hashlib.sha256()
    for f in (kernel_file, "rsaw_device.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, kernel_file: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel
    calibration; None when no summary exists or the kernel source changed
    since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)[workload]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_sha256") != kernel_source_hash(kernel_file):
        return None
    return rec["bytes_per_launch"]


def lattice_alg_ops_per_chain(N: int) -> int:
    """Algorithmic VALU lane-operations to grow one lattice chain of N monomers.

    Per step i: the pair tests against the monomers that can neighbour the
    tip (floor(i/2) of them on the bipartite cubic lattice), 4 operations
    each (L1 distance, neighbour flag, direction code, mask insert); one
    eighth of a Philox4x32-10 block, the 16 bits the pick consumes (10
    rounds x 6 operations / 8, rounded up to 8); and 10 operations to
    count, pick and apply the move and tally m_i for log W.
    """
    return sum(4 * (i // 2) + 8 + 10 for i in range(1, N))


# LDS bandwidth of the chip: 128 bytes per clock per CU, 256 CUs, 2.4 GHz.
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12


def real_lds_bytes_per_chain(N: int) -> int:
    """Algorithmic LDS bytes of one hard-sphere chain (beads as three
    binary64 planes).  Per step i the culling pass reads beads 0..i-4 once
    (24 B each), the two beads next to the tip are read once (their loads
    are broadcast to the trial lanes) and the new bead is written (24 B)."""
    return sum(24 * max(i - 3, 0) + 24 * min(max(i - 1, 0), 2) + 24 for i in range(1, N))


def lattice26_lds_bytes_per_chain(N: int) -> int:
    """Algorithmic LDS bytes of one 26-neighbour chain (one 4-byte word per
    monomer): per step i every earlier monomer but the predecessor is read
    once and the new monomer is written."""
    return sum(4 * max(i - 1, 0) + 4 for i in range(1, N))


def lds_object(bytes_per_launch: float, kernel_ms: float, note: str) -> dict:
    ach = bytes_per_launch / (kernel_ms / 1e3) / 1e12
    return {"bytes_per_launch": bytes_per_launch, "achieved": ach, "peak": LDS_PEAK_TBS, "unit": "TB/s",
            "frac": ach / LDS_PEAK_TBS, "model": note}


def real_alg_ops_per_chain(N: int, k: int) -> float:
    """Algorithmic VALU lane-operations to grow one hard-sphere chain.

    Per step i: k candidates, each tested against beads 0..i-2 at 9
    binary64 operations (3 sub, 3 mul, 2 add, 1 compare); k Marsaglia
    directions at 4/pi Philox blocks each (60 operations per block) plus
    ~20 operations for the disc test, square root and candidate; and
    10 operations to count, pick and add log m_i.
    """
    tot = 0.0
    for i in range(1, N):
        tot += k * 9 * max(i - 1, 0) + k * (60 * 4 / math.pi + 20) + 10
    return tot


def lattice26_alg_ops_per_chain(N: int) -> int:
    """Algorithmic VALU lane-operations to grow one 26-neighbour lattice chain.

    Per step i: the pair tests against monomers 0..i-2 (no parity pruning:
    a diagonal step keeps the parity), 6 operations each (byte differences,
    their shifted copy, the range test of every coordinate, the neighbour
    flag, the direction code, the mask insert); 8 for the step's share of a
    Philox block; and 20 to count the free codes, select the r-th, apply the
    move and tally m_i.
    """
    return sum(6 * max(i - 1, 0) + 8 + 20 for i in range(1, N))


def path_model(w) -> dict:
    """Growth kernel of a workload, its algorithmic VALU lane-operations and
    LDS bytes per launch, and the VALU peak it is priced against."""
    geo, N, M = w["geometry"], w["N"], w["n_chains"]
    if geo == "lattice":
        reg = N <= 64 or w.get("exact_w", False)
        grp = not reg and N <= 4096  # history in the group's VGPRs (built-in lane rule)
        kernel = "grow_lattice_reg" if reg else ("grow_lattice_grp" if grp else "grow_lattice_lds")
        return dict(kernel=kernel, kernel_file="grow_lattice.hip" if reg else "grow_lattice_lds.hip",
                    ops=lattice_alg_ops_per_chain(N) * M, peak=VALU_PEAK_INT32_TOPS, int_path=True,
                    lds_bytes=0.0 if reg or grp else lattice_lds_bytes_per_chain(N) * M,
                    lds_note=("chain history in VGPRs: no LDS traffic" if reg or grp else
                              "parity-plane words of the neighbour candidates read once per step"))
    if geo == "lattice26":
        lane = N <= 64
        grp = not lane and N <= 4096  # one-word formats in the group's VGPRs (built-in lane rule)
        return dict(kernel="grow_lattice26_lane" if lane else ("grow_lattice26_grp" if grp else "grow_lattice26"),
                    kernel_file="grow_lattice26.hip",
                    ops=lattice26_alg_ops_per_chain(N) * M, peak=VALU_PEAK_INT32_TOPS, int_path=True,
                    lds_bytes=0.0 if grp else lattice26_lds_bytes_per_chain(N) * M * (1 if lane else 2),
                    lds_note="chain history in VGPRs: no LDS traffic" if grp else "monomer words read once per step")
    hbm = N > 1536
    return dict(kernel="grow_real_hbm" if hbm else "grow_real_tp", kernel_file="grow_real.hip",
                ops=real_alg_ops_per_chain(N, w["k"]) * M, peak=VALU_PEAK_FP64_TOPS, int_path=False,
                lds_bytes=0.0 if hbm else real_lds_bytes_per_chain(N) * M,
                lds_note="beads in HBM planes" if hbm else "beads read once per step")


def lattice_lds_bytes_per_chain(N: int) -> int:
    """Algorithmic LDS bytes of one long lattice chain in LDS (one 4-byte
    word per monomer up to N = 2048, two beyond): per step i the floor(i/2)
    monomers of the tip's opposite parity are read once, and the new monomer
    is written."""
    w = 4 if N <= 2048 else 8
    return sum(w * (i // 2) + w for i in range(1, N))


def roofline_object(pm: dict, kernel_ms: float, workload: str) -> dict:
    """Roofline of a growth kernel: algorithmic lane-operations per launch
    over the kernel's mean duration, against the VALU peak."""
    ach = pm["ops"] / (kernel_ms / 1e3) / 1e12
    out = {"bound": "alu", "achieved": ach, "peak": pm["peak"], "unit": "Tops/s", "frac": ach / pm["peak"]}
    if pm["int_path"]:
        out.update(attainable_peak=ATTAINABLE_INT_PATH_TOPS, frac_attainable=ach / ATTAINABLE_INT_PATH_TOPS)
    out.update(traffic=measured_traffic(pm["kernel"], pm["kernel_file"], workload), kernel=pm["kernel"],
               kernel_ms=kernel_ms, alg_ops_per_launch=pm["ops"])
    return out


def side_leg(w, name, steps, torch, rs) -> dict:
    """Throughput, latency, roofline and LDS objects of one more workload."""
    r = run_gpu(w, steps, 1, torch, rs)
    T = sum(r["lat"]) / 1e3
    pm = path_model(w)
    return {"workload": name, "value": w["n_chains"] * (w["N"] - 1) * steps / T,
            "unit": "monomer-steps/s", "steps": steps, "ms_per_step": T * 1e3 / steps,
            "p50_ms": _percentile(r["lat"], 0.5), "p99_ms": _percentile(r["lat"], 0.99),
            "roofline": roofline_object(pm, r["grow_ms"], name),
            "lds": lds_object(pm["lds_bytes"], r["grow_ms"], pm["lds_note"]),
            "physics": {k: r["summary"][k] for k in ("n_alive", "log_c_est", "r2_mean",
                                                      "r2_err", "rg2_mean", "rg2_err")}}


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    pos = (len(xs) - 1) * q
    lo = int(math.floor(pos))
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


def run_gpu(w, steps, warmup, torch, rs):
    dev = torch.device("cuda", 0)
    M, N = w["n_chains"], w["N"]
    cfg = rs.make_config(w["geometry"], N, w["k"], M, w["seed"], coord=w["coord"],
                         bond_length=w.get("bond_length", 1.0),
                         bead_diameter=w.get("bead_diameter", 1.0),
                         hist_bins=w["hist_bins"], exact_w=w.get("exact_w", False))
    ctype = {rs.RSAW_I16: torch.int16, rs.RSAW_I32: torch.int32, rs.RSAW_F64: torch.float64}[cfg.coord_type]
    bufs = dict(log_w=torch.empty(M, dtype=torch.float64, device=dev),
                r_end=torch.empty((3, M), dtype=ctype, device=dev),
                r2=torch.empty(M, dtype=torch.float64, device=dev),
                rg2=torch.empty(M, dtype=torch.float64, device=dev),
                n_grown=torch.empty(M, dtype=torch.int16, device=dev))
    o = rs.rsaw_chain_out()
    o.log_w, o.r_end, o.r2, o.rg2, o.n_grown = (bufs[k].data_ptr() for k in
                                                  ("log_w", "r_end", "r2", "rg2", "n_grown"))
    if w["geometry"] != "real":
        bufs["n2rg2"] = torch.empty(M, dtype=torch.int64, device=dev)
        o.n2rg2 = bufs["n2rg2"].data_ptr()
    summ = torch.empty(rs.SUMMARY_BYTES, dtype=torch.uint8, device=dev)
    hw = torch.empty(max(w["hist_bins"], 1), dtype=torch.float64, device=dev)
    hn = torch.empty(max(w["hist_bins"], 1), dtype=torch.uint64, device=dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream

    def step():
        rs.gen_chains_raw(cfg, o, summ.data_ptr(), hw.data_ptr() if w["hist_bins"] else 0,
                          hn.data_ptr() if w["hist_bins"] else 0, sh)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    # The library brackets each growth-kernel launch with HIP events on the
    # stream it launches on; read back after the timed region.
    rs.kernel_time()
    rs.kernel_timing(True)
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rs.kernel_timing(False)
    k_ms, k_n = rs.kernel_time()
    if k_n != steps:
        raise RuntimeError(f"timed {k_n} growth launches, expected {steps}")
    lat = [a.elapsed_time(b) for a, b in ev]
    summary = rs.parse_summary(summ)
    if summary["status"] != 0:
        raise RuntimeError(f"device status {summary['status']}")
    # end to end on the host clock: enqueue, then the summary's copy to the
    # host and the wait for it (outside the timed region above)
    e2e = []
    for _ in range(3):
        t1 = time.perf_counter()
        step()
        summ.cpu()
        e2e.append((time.perf_counter() - t1) * 1e3)

    return dict(wall=wall, lat=lat, summary=summary, grow_ms=k_ms / k_n, e2e_ms=_percentile(e2e, 0.5))


def device_info(torch) -> dict:
    """Name, architecture, CU count and memory of device 0 as HIP reports
    them."""
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "cus": p.multi_processor_count,
            "hbm_bytes": p.total_memory, "l2_bytes": getattr(p, "L2_cache_size", None)}


def run_batch(torch, rs, reps, m_lo=3.0, m_span=3.0):
    """Mixed workload of 256 ensembles of 10^m_lo .. 10^(m_lo + m_span)
    chains: one rsaw_gen_batch call against 256 rsaw_gen_chains calls on the
    same stream (per-chain outputs and summaries in both), events around the
    whole and around each plain call."""
    from paper_1704_04381_amd.workloads import mixed_ensembles

    dev = torch.device("cuda", 0)
    specs = mixed_ensembles(m_lo=m_lo, m_span=m_span)
    cfgs, outs, keep = [], [], []
    for sp in specs:
        sp = dict(sp)
        cfg = rs.make_config(sp.pop("geometry"), sp.pop("N"), sp.pop("k"), sp.pop("n_chains"),
                             sp.pop("seed"), **sp)
        out, o = rs._alloc_outputs(cfg, dev, True, 0)
        cfgs.append(cfg)
        outs.append(o)
        keep.append(out)
    n = len(cfgs)
    summ = torch.empty(n * rs.SUMMARY_BYTES, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    steps = sum(c.n_chains * (c.n_monomers - 1) for c in cfgs)

    def batched():
        rs.gen_batch_raw(cfgs, outs, summ.data_ptr(), None, None, sh)

    def plain(evs=None):
        for i, (c, o) in enumerate(zip(cfgs, outs)):
            if evs is not None:
                evs[i][0].record(stream)
            rs.gen_chains_raw(c, o, summ.data_ptr() + i * rs.SUMMARY_BYTES, 0, 0, sh)
            if evs is not None:
                evs[i][1].record(stream)

    batched()
    plain()
    torch.cuda.synchronize()
    t_b, t_p, per, done = [], [], [], []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        batched()
        b.record(stream)
        torch.cuda.synchronize()
        t_b.append(a.elapsed_time(b))
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a2.record(stream)
        plain(evs)
        b2.record(stream)
        torch.cuda.synchronize()
        t_p.append(a2.elapsed_time(b2))
        per.extend(x.elapsed_time(y) for x, y in evs)
        # completion of ensemble i from the common submission at a2: the
        # plain launches finish one after another
        done.extend(a2.elapsed_time(y) for _, y in evs)
    tb, tp = _percentile(t_b, 0.5), _percentile(t_p, 0.5)
    # the same batch after the autotuner has picked the lane mapping of each
    # (geometry, k, N bucket) of the workload
    t0 = time.perf_counter()
    tuning = tune_mixed(rs)
    tune_s = time.perf_counter() - t0
    rows = rs.mapping_list()
    batched()
    torch.cuda.synchronize()

    def timed_batch():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        batched()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    # tuned and built-in batches interleaved, so that both see the same
    # clocks; the built-in figure pools these runs with the ones above.  The
    # autotuner installs an entry only where a mapping beat the rule by 3 %;
    # with none installed the tuned batch is the built-in one, launch for
    # launch, and one pooled figure stands for both.
    t_t = []
    for _ in range(reps):
        rs.mapping_clear()
        t_b.append(timed_batch())
        for m in rows:
            rs.mapping_set(m["geometry"], m["k_trials"], m["n_lo"], m["n_hi"], m["lanes"], m["threads"])
        t_t.append(timed_batch())
    rs.mapping_clear()
    if not rows:
        t_b = t_b + t_t
        t_t = t_b
    tb, tt = _percentile(t_b, 0.5), _percentile(t_t, 0.5)
    return {
        "workload": f"mixed_256 (N = 8..128, lattice k = 6 / hard spheres k = 8, 16, "
                    f"10^{m_lo:g}..10^{m_lo + m_span:g} chains each)",
        "ensembles": n, "chains": sum(c.n_chains for c in cfgs), "monomer_steps": steps,
        "batched_ms": tb, "batched_value": steps / (tb / 1e3),
        "plain_ms": tp, "plain_value": steps / (tp / 1e3),
        "unit": "monomer-steps/s", "speedup": tp / tb, "reps": reps,
        "plain_ensemble_p50_ms": _percentile(per, 0.5), "plain_ensemble_p99_ms": _percentile(per, 0.99),
        # like for like: each ensemble's completion time from the common
        # submission of all of them.  In a batch every summary is written by
        # its last launch, so each ensemble completes when the batch does.
        "completion_ms": {"batched_p50": _percentile(t_b, 0.5), "batched_p99": _percentile(t_b, 0.99),
                          "plain_p50": _percentile(done, 0.5), "plain_p99": _percentile(done, 0.99)},
        "batched_ensemble_latency_ms": tb,
        "tuned_batched_ms": tt, "tuned_batched_value": steps / (tt / 1e3), "tuned_speedup": tp / tt,
        "autotune_s": tune_s, "tuned_mappings": tuning, "tuned_entries_installed": len(rows),
    }


# Buckets of the mixed workload (N = 8..128) that have a group kernel: the
# lattice above N = 64, hard spheres at every N, each k separately.
TUNE_BUCKETS = (("lattice", 6, (96, 128), 1 << 17),
                ("real", 8, (32, 64, 96, 128), 1 << 15),
                ("real", 16, (32, 64, 96, 128), 1 << 15))


def tune_mixed(rs):
    """Autotune the lane mapping for the mixed workload's buckets; returns
    the chosen (geometry, k, N range, lanes, threads, ms) per bucket."""
    out = []
    for geo, k, edges, m in TUNE_BUCKETS:
        lo = 65 if geo == "lattice" else 1
        res = rs.autotune(geo, k, edges, m, reps=3)
        for r in res:
            out.append({"geometry": geo, "k": k, "n_lo": max(lo, r["n_lo"]), "n_hi": r["n_hi"],
                        "lanes": r["lanes"], "threads": r["threads"], "ms": r["ms"]})
    return out


def run_serving(rs, rate, n, warmup, streams=2, max_batch=64, m_lo=4.0, m_span=3.0):
    """Open-loop serving run: requests submitted at their Poisson arrival
    times by one thread, completions taken by another; latency =
    completion - submission (host clock), measured after `warmup` requests."""
    import threading

    from paper_1704_04381_amd.workloads import serving_requests

    reqs = serving_requests(n=n, rate=rate, m_lo=m_lo, m_span=m_span)
    srv = rs.Server(max_batch=max_batch, streams=streams)
    tickets = [None] * n
    ready = [threading.Event() for _ in range(n)]
    t0 = time.perf_counter()

    def submitter():
        for i, (at, sp) in enumerate(reqs):
            d = t0 + at - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets[i] = srv.submit(**sp)
            ready[i].set()

    th = threading.Thread(target=submitter)
    th.start()
    lat, done_t = [], []
    for i in range(n):
        ready[i].wait()
        r = srv.wait(tickets[i])
        if i >= warmup:
            lat.append(r["latency_us"] / 1e3)
        done_t.append(time.perf_counter())
    th.join()
    srv.close()
    work = [sp["n_chains"] * (sp["N"] - 1) for _, sp in reqs]
    t_first = t0 + reqs[warmup][0]
    span = max(done_t[warmup:]) - t_first
    measured = sum(work[warmup:])
    offered = sum(work) / reqs[-1][0]
    achieved = measured / span
    return {
        "rate_per_s": rate, "requests": n, "warmup": warmup, "streams": streams, "max_batch": max_batch,
        "latency_p50_ms": _percentile(lat, 0.5), "latency_p99_ms": _percentile(lat, 0.99),
        "throughput_steps_per_s": achieved, "offered_steps_per_s": offered, "span_s": span,
    }


def serving_leg(rs):
    """Bounded serving measurement for the default run (about a minute): the
    serving workload's request stream at 20/s (300 requests) and 40/s (300),
    and its first 300 requests at 200/s, each served by the server and by
    per-request plain launches (one stream, one request per launch, arrival
    order).  The 200/s run is overloaded, so its throughput is the capacity,
    and rho = offered work / that capacity."""
    runs, plain = [], []
    for rate, n, warm in ((20.0, 300, 30), (40.0, 300, 30), (200.0, 300, 30)):
        print(f"[serve] rate {rate}/s, {n} requests", file=sys.stderr, flush=True)
        runs.append(run_serving(rs, rate, n, warm))
        print(f"[serve] plain launches, rate {rate}/s", file=sys.stderr, flush=True)
        plain.append(run_serving(rs, rate, n, warm, streams=1, max_batch=1))
    cap = runs[-1]["throughput_steps_per_s"]
    for r in runs + plain:
        r["rho"] = r["offered_steps_per_s"] / cap
    return {"workload": "serving_requests (Poisson arrivals; N in {16, 32, 64, 128, 256}; lattice k = 6 or "
                        "hard spheres k = 8; 10^4..10^7 chains each)",
            "unit": "ms / monomer-steps/s", "served": runs, "plain": plain,
            "capacity_steps_per_s": cap, "plain_capacity_steps_per_s": plain[-1]["throughput_steps_per_s"]}


def host_cpu() -> dict:
    """The host's CPU model (/proc/cpuinfo), its logical CPU count (nproc),
    the CPUs this process may run on (affinity) and the thread share the job
    is given (OMP_NUM_THREADS, when set)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS")
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "job_share": int(share) if share and share.isdigit() else None}


def _oracle_rate(w, n, threads):
    """Oracle growth + reduction of the workload's first n chains on
    `threads` threads (chain ranges; the oracle's C calls release the GIL);
    returns (monomer-steps/s, seconds)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    parts = [(i * n // threads, (i + 1) * n // threads) for i in range(threads)]

    def work(rng):
        lo, hi = rng
        if w["geometry"] == "lattice":
            return oracle.gen_lattice(w["seed"], w["N"], hi - lo, chain_offset=lo)
        return oracle.gen_real(w["seed"], w["N"], w["k"], hi - lo, b=w.get("bond_length", 1.0),
                               sigma=w.get("bead_diameter", 1.0), chain_offset=lo)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(work, parts))
    cat = {k: np.concatenate([r[k] for r in res]) for k in ("log_w", "r2", "rg2", "n_grown")}
    oracle.reduce(w["N"], cat["log_w"], cat["r2"], cat["rg2"], cat["n_grown"], bins=w["hist_bins"])
    dt = time.perf_counter() - t0
    return n * (w["N"] - 1) / dt, dt


def cpu_baseline(w, single_chains, all_chains):
    """The oracle, untuned, on the host: a bounded sample of the same
    workload (its first chains, growth and reduction) on one thread and on
    every core the job may use (the affinity set, within the job's thread
    share when one is set).  The oracle's throughput is linear in the chain
    count, so a sample gives the full workload's rate."""
    import oracle

    oracle.build()
    cpu = host_cpu()
    threads = cpu["affinity"]
    if cpu["job_share"]:
        threads = min(threads, cpu["job_share"])
    one, dt1 = _oracle_rate(w, single_chains, 1)
    allc, dta = _oracle_rate(w, all_chains, threads)
    return dict(value=allc, unit="monomer-steps/s", cores=threads, kind="oracle",
                sample=f"first {all_chains} chains of the workload (seed {w['seed']}), growth + reduction, "
                       f"{threads} threads, {dta:.2f} s wall",
                single_thread={"value": one, "cores": 1,
                               "sample": f"first {single_chains} chains, growth + reduction, 1 thread, "
                                         f"{dt1:.2f} s"},
                parallel_efficiency=allc / (one * threads),
                host_cpu=cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lattice_n64")
    ap.add_argument("--secondary", default="real_n64")
    ap.add_argument("--variant", default="lattice26_n64",
                    help="26-neighbour lattice workload reported under \"variant\" ('' to skip)")
    ap.add_argument("--long", default="lattice_n256,lattice26_n256",
                    help="comma-separated long-chain workloads reported under \"long_chains\" ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving benchmark (open-loop Poisson requests; about 2 minutes)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the mixed 256-ensemble batched-launch measurement")
    ap.add_argument("--cpu-scale", type=float, default=1.0,
                    help="scale of the oracle samples of the CPU baseline (1 = about 10 s of CPU "
                         "work per leg)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the bounded serving leg (20/s, 40/s and a shortened 200/s trace, "
                         "served and by plain launches)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (3 times), to scale "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); the chain ranges would shard by chain_offset "
              f"with no data exchange beyond the ensemble partials.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1704_04381_amd as rs
    from paper_1704_04381_amd.workloads import WORKLOADS

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        rs.load()
        out = {"metric": "serving: Poisson requests (N = 16..256, lattice / hard spheres, 10^4..10^7 "
                         "chains each), latency p50/p99 and throughput", "unit": "ms / monomer-steps/s",
               "runs": []}
        rates = ((200.0, 2100, 100), (20.0, 300, 30), (5.0, 150, 15))
        for rate, n, warm in rates:
            print(f"[serve] rate {rate}/s, {n} requests", file=sys.stderr, flush=True)
            out["runs"].append(run_serving(rs, rate, n, warm))
        # the same traces served by per-request plain launches: one stream,
        # one request per launch, in arrival order
        out["plain_runs"] = []
        for rate, n, warm in rates:
            print(f"[serve] plain launches, rate {rate}/s, {n} requests", file=sys.stderr, flush=True)
            out["plain_runs"].append(run_serving(rs, rate, n, warm, streams=1, max_batch=1))
        # the 200/s run is overloaded: its throughput is the capacity, and
        # rho = offered work / capacity for every run
        from paper_1704_04381_amd.workloads import serving_requests

        cap = out["runs"][0]["throughput_steps_per_s"]
        for r in out["runs"] + out["plain_runs"]:
            r["rho"] = r["offered_steps_per_s"] / cap
        out["plain_capacity_steps_per_s"] = out["plain_runs"][0]["throughput_steps_per_s"]
        mean_work = sum(sp["n_chains"] * (sp["N"] - 1) for _, sp in serving_requests()) / 2100
        out["capacity_steps_per_s"] = cap
        out["max_sustainable_rate_per_s"] = cap / mean_work
        print(json.dumps(out), flush=True)
        return
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)
        return
    rs.load()
    w = WORKLOADS[args.workload]
    M, N = w["n_chains"], w["N"]
    r = run_gpu(w, args.steps, args.warmup, torch, rs)
    T = sum(r["lat"]) / 1e3
    value = M * (N - 1) * args.steps / T
    pm = path_model(w)
    line = {
        "metric": "monomer-steps/s at N=64 lattice + hard-sphere; p50/p99 ensemble latency",
        "value": value,
        "unit": "monomer-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3 / args.steps,
        "p50_ms": _percentile(r["lat"], 0.5),
        "p99_ms": _percentile(r["lat"], 0.99),
        "end_to_end_ms": r["e2e_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64" if w["geometry"] != "real" else "f64",
        "data": "synthetic (counter-based Philox draws inside the method)",
        "config": {"workload": args.workload, "geometry": w["geometry"], "N": N, "k": w["k"],
                   "n_chains": M, "seed": w["seed"], "coord": w["coord"],
                   "hist_bins": w["hist_bins"]},
        "roofline": roofline_object(pm, r["grow_ms"], args.workload),
        "lds": lds_object(pm["lds_bytes"], r["grow_ms"], pm["lds_note"]),
        "physics": {k: r["summary"][k] for k in ("n_alive", "log_c_est", "r2_mean", "r2_err",
                                                 "rg2_mean", "rg2_err", "ess")},
        "device": device_info(torch),
    }
    for key, name in (("secondary", args.secondary), ("variant", args.variant)):
        if name:
            line[key] = side_leg(WORKLOADS[name], name, max(3, args.steps // 4), torch, rs)
    if args.long:
        line["long_chains"] = [side_leg(WORKLOADS[n], n, 3, torch, rs) for n in args.long.split(",")]
    if not args.no_batch:
        line["batch"] = {"full": run_batch(torch, rs, 3),
                         "small": run_batch(torch, rs, 5, m_lo=2.0, m_span=2.0)}
    if not args.no_serve:
        print("[bench] serving leg", file=sys.stderr, flush=True)
        line["serving"] = serving_leg(rs)
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        scale = max(args.cpu_scale, 0.01)
        if w["geometry"] == "lattice":
            line["cpu_baseline"] = cpu_baseline(w, int(200_000 * scale), int(1_000_000 * scale))
        else:
            line["cpu_baseline"] = cpu_baseline(w, int(60_000 * scale), int(300_000 * scale))
        if args.secondary and "secondary" in line:
            w2 = WORKLOADS[args.secondary]
            if w2["geometry"] == "lattice":
                line["secondary"]["cpu_baseline"] = cpu_baseline(w2, int(200_000 * scale), int(1_000_000 * scale))
            else:
                line["secondary"]["cpu_baseline"] = cpu_baseline(w2, int(60_000 * scale), int(300_000 * scale))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
