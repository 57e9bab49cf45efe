// C ABI of librsaw (declared in include/rsaw.h): argument validation,
// per-(device, stream) workspace, and the launch sequence
//   reduce_init -> grow_{lattice,real} -> reduce_partials -> reduce_final,
// one ensemble per call or a batch of ensembles sharing the launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <tuple>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "rsaw.h"
#include "rsaw_device.hpp"
#include "rsaw_reduce.hpp"

namespace rsaw {
hipError_t launch_grow_lattice(const GrowArgs &a, bool exact, bool i16, hipStream_t s);
hipError_t launch_grow_real(const GrowArgs &a, hipStream_t s);
int real_max_monomers();
uint32_t real_hbm_slots(int n_monomers, uint64_t n_chains);
int lattice_lds_max_monomers();
void lattice_reg_variant(const GrowArgs &a, bool exact, bool i16, GrowVariant *v);
hipError_t lattice_lds_variant(const GrowArgs &a, bool i16, GrowVariant *v);
hipError_t real_variant(const GrowArgs &a, GrowVariant *v);
hipError_t launch_lattice_reg_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                                    int n, uint64_t blocks, hipStream_t s);
hipError_t launch_lattice_lds_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                                    int n, uint64_t blocks, size_t shmem, hipStream_t s);
hipError_t launch_real_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0, int n,
                             uint64_t blocks, size_t shmem, hipStream_t s);
int lattice26_max_monomers();
hipError_t lattice26_variant(const GrowArgs &a, bool exact, bool i16, GrowVariant *v);
hipError_t launch_grow_lattice26(const GrowArgs &a, bool exact, bool i16, hipStream_t s);
hipError_t launch_lattice26_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0, int n,
                                  uint64_t blocks, size_t shmem, hipStream_t s);
} // namespace rsaw

namespace {

thread_local std::string g_last_error;

rsaw_status fail(rsaw_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

rsaw_status hip_fail(hipError_t e, const char *what)
{
    return fail(RSAW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device buffers reused across calls on one (device, stream).  Grown on
// demand; released by rsaw_shutdown().  A caller-owned buffer bound by
// rsaw_set_workspace replaces the internal one and is never grown or freed.
struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
    bool external = false;      // base is the caller's buffer (rsaw_set_workspace)
    void *stage = nullptr;      // pinned host staging of batch descriptor tables
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr; // recorded after the last copy out of `stage`
};

// Entries are created under g_ws_lock and never move (std::map); an entry is
// then used without the lock by the one host thread that drives its stream
// (the ABI's rule for calls on one stream), so a synchronising call on one
// stream's entry never blocks calls on other streams.
std::mutex g_ws_lock;
std::map<std::pair<int, void *>, Workspace> g_ws;

Workspace &ws_entry(int dev, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_ws_lock);
    return g_ws[{dev, (void *)s}];
}

rsaw_status workspace(int dev, hipStream_t s, size_t need, void **out)
{
    Workspace &w = ws_entry(dev, s);
    if (w.external) {
        if (w.bytes < need)
            return fail(RSAW_E_NOMEM, "the caller's workspace holds " + std::to_string(w.bytes) +
                                          " bytes; this call needs " + std::to_string(need) +
                                          " (rsaw_workspace_size)");
        *out = w.base;
        return RSAW_OK;
    }
    if (w.bytes < need) {
        if (w.base) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            e = hipFree(w.base);
            if (e != hipSuccess) return hip_fail(e, "hipFree");
            w.base = nullptr;
            w.bytes = 0;
        }
        size_t sz = need < ((size_t)1 << 20) ? ((size_t)1 << 20) : need;
        hipError_t e = hipMalloc(&w.base, sz);
        if (e != hipSuccess) {
            w.base = nullptr;
            (void)hipGetLastError(); // a failed allocation must not fail the thread's next launch check
            return fail(RSAW_E_NOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        }
        w.bytes = sz;
    }
    *out = w.base;
    return RSAW_OK;
}

// Pinned host buffer of at least `need` bytes for the batch tables of
// (dev, s), free for writing: waits for the previous copy out of it.
rsaw_status staging(int dev, hipStream_t s, size_t need, void **out, hipEvent_t *done)
{
    Workspace &w = ws_entry(dev, s);
    if (w.stage_done) {
        hipError_t e = hipEventSynchronize(w.stage_done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else {
        hipError_t e = hipEventCreateWithFlags(&w.stage_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (w.stage_bytes < need) {
        if (w.stage) {
            hipError_t e = hipHostFree(w.stage);
            if (e != hipSuccess) return hip_fail(e, "hipHostFree");
            w.stage = nullptr;
            w.stage_bytes = 0;
        }
        size_t sz = need < ((size_t)1 << 16) ? ((size_t)1 << 16) : need;
        hipError_t e = hipHostMalloc(&w.stage, sz, hipHostMallocDefault);
        if (e != hipSuccess) {
            w.stage = nullptr;
            (void)hipGetLastError();
            return fail(RSAW_E_NOMEM, std::string("staging hipHostMalloc: ") + hipGetErrorString(e));
        }
        w.stage_bytes = sz;
    }
    *out = w.stage;
    *done = w.stage_done;
    return RSAW_OK;
}

// Growth-kernel timing: event pairs recorded around launches while enabled.
struct EventPair {
    hipEvent_t start = nullptr, stop = nullptr;
};

std::mutex g_tm_lock;
bool g_tm_enabled = false;
std::vector<EventPair> g_tm_recorded, g_tm_free;

// Record the start event of a timed launch; false (and no pair) when timing is off.
rsaw_status timing_start(hipStream_t s, EventPair *pair, bool *timed)
{
    std::lock_guard<std::mutex> lk(g_tm_lock);
    *timed = false;
    if (!g_tm_enabled) return RSAW_OK;
    EventPair p;
    if (!g_tm_free.empty()) {
        p = g_tm_free.back();
        g_tm_free.pop_back();
    } else {
        hipError_t e = hipEventCreate(&p.start);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        e = hipEventCreate(&p.stop);
        if (e != hipSuccess) {
            (void)hipEventDestroy(p.start);
            return hip_fail(e, "hipEventCreate");
        }
    }
    hipError_t e = hipEventRecord(p.start, s);
    if (e != hipSuccess) {
        g_tm_free.push_back(p);
        return hip_fail(e, "hipEventRecord");
    }
    *pair = p;
    *timed = true;
    return RSAW_OK;
}

rsaw_status timing_stop(hipStream_t s, const EventPair &p)
{
    std::lock_guard<std::mutex> lk(g_tm_lock);
    hipError_t e = hipEventRecord(p.stop, s);
    if (e != hipSuccess) {
        g_tm_free.push_back(p);
        return hip_fail(e, "hipEventRecord");
    }
    g_tm_recorded.push_back(p);
    return RSAW_OK;
}

// ln(m) for m = 0..64, correctly rounded by the host libm (checked by the tests).
const double *logm_table()
{
    static double t[65];
    static std::once_flag once;
    std::call_once(once, [] {
        t[0] = 0.0;
        for (int m = 1; m <= 64; ++m) t[m] = std::log((double)m);
    });
    return t;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t min_workspace_bytes();

rsaw_status validate(const rsaw_config *cfg)
{
    if (!cfg) return fail(RSAW_E_INVALID, "cfg is NULL");
    const int N = cfg->n_monomers;
    if (N < 1 || N > 65535) return fail(RSAW_E_INVALID, "n_monomers must be in 1..65535");
    if (cfg->n_chains >= (1ull << 32)) return fail(RSAW_E_INVALID, "n_chains must be below 2^32");
    if (cfg->hist_bins < 0) return fail(RSAW_E_INVALID, "hist_bins must be >= 0");
    if (cfg->hist_bins > rsaw::kMaxBins) return fail(RSAW_E_UNSUPPORTED, "hist_bins above 256");
    if (cfg->flags & ~(RSAW_EXACT_W | RSAW_RESTART)) return fail(RSAW_E_INVALID, "unknown flag bits");
    if (cfg->geometry == RSAW_LATTICE_SC) {
        if (cfg->k_trials != 6) return fail(RSAW_E_INVALID, "lattice needs k_trials == 6");
        if (cfg->coord_type != RSAW_I16 && cfg->coord_type != RSAW_I32)
            return fail(RSAW_E_INVALID, "lattice coord_type must be RSAW_I16 or RSAW_I32");
        if ((cfg->flags & RSAW_EXACT_W) && N > 28)
            return fail(RSAW_E_OVERFLOW, "RSAW_EXACT_W needs n_monomers <= 28");
        if (N > rsaw::lattice_lds_max_monomers())
            return fail(RSAW_E_UNSUPPORTED, "lattice kernels support n_monomers <= 16384");
    } else if (cfg->geometry == RSAW_LATTICE_26) {
        if (cfg->k_trials != 26) return fail(RSAW_E_INVALID, "26-neighbour lattice needs k_trials == 26");
        if (cfg->coord_type != RSAW_I16 && cfg->coord_type != RSAW_I32)
            return fail(RSAW_E_INVALID, "lattice coord_type must be RSAW_I16 or RSAW_I32");
        if ((cfg->flags & RSAW_EXACT_W) && N > 14)
            return fail(RSAW_E_OVERFLOW, "RSAW_EXACT_W on the 26-neighbour lattice needs n_monomers <= 14");
        if (N > rsaw::lattice26_max_monomers())
            return fail(RSAW_E_UNSUPPORTED, "26-neighbour lattice kernels support n_monomers <= 16384");
    } else if (cfg->geometry == RSAW_REAL_HS) {
        if (cfg->k_trials < 1 || cfg->k_trials > 64)
            return fail(RSAW_E_INVALID, "real-space k_trials must be in 1..64");
        if (cfg->coord_type != RSAW_F64) return fail(RSAW_E_INVALID, "real-space coord_type must be RSAW_F64");
        if (!(cfg->bond_length > 0.0) || !std::isfinite(cfg->bond_length))
            return fail(RSAW_E_INVALID, "bond_length must be finite and > 0");
        if (!(cfg->bead_diameter >= 0.0) || !std::isfinite(cfg->bead_diameter))
            return fail(RSAW_E_INVALID, "bead_diameter must be finite and >= 0");
        if (cfg->flags & RSAW_EXACT_W) return fail(RSAW_E_INVALID, "RSAW_EXACT_W is lattice-only");
        if (N > rsaw::real_max_monomers())
            return fail(RSAW_E_UNSUPPORTED, "real-space kernels support n_monomers <= 16384");
    } else {
        return fail(RSAW_E_INVALID, "unknown geometry");
    }
    return RSAW_OK;
}

// Per-ensemble layout of the workspace: reduction cells, block partials,
// histogram accumulators and the per-chain arrays the reduction needs when
// the caller does not supply them.
struct EnsLayout {
    bool lattice, z26, exact, reduce;
    int bins;
    uint32_t n_blocks; // reduce blocks
    uint64_t chunk;    // chains per reduce block
    size_t off_lmax, off_status, off_summary, off_part, off_hacc;
    size_t off_lw, off_r2, off_rg2, off_ng, off_wx, off_nn;
    size_t off_slots;  // HBM bead planes of the long hard-sphere kernel
    uint32_t n_slots;
    bool need_lw, need_r2, need_rg2, need_ng, need_wx, need_nn;
};

// Appends the ensemble's regions at *off (bytes, 256-aligned).
void layout_ensemble(const rsaw_config *cfg, const rsaw_chain_out &o, bool reduce, size_t *off,
                     EnsLayout *L)
{
    const uint64_t M = cfg->n_chains;
    L->lattice = cfg->geometry != RSAW_REAL_HS;
    L->z26 = cfg->geometry == RSAW_LATTICE_26;
    L->exact = L->lattice && (cfg->flags & RSAW_EXACT_W);
    L->reduce = reduce;
    L->bins = reduce ? cfg->hist_bins : 0;
    // reduce blocks: at most 1024, each a contiguous run of whole 256-chain tiles
    L->n_blocks = 0;
    L->chunk = 256;
    if (M > 0) {
        const uint64_t tiles = (M + 255) / 256;
        const uint64_t nb = tiles < 1024 ? tiles : 1024;
        L->chunk = ((tiles + nb - 1) / nb) * 256;
        L->n_blocks = (uint32_t)((M + L->chunk - 1) / L->chunk);
    }
    size_t x = *off;
    L->off_lmax = x; x = align256(x + sizeof(unsigned long long));
    L->off_status = x; x = align256(x + sizeof(int32_t));
    L->off_summary = x; x = align256(x + sizeof(rsaw_summary));
    L->off_part = x; x = align256(x + (size_t)L->n_blocks * sizeof(rsaw::BlockPartial));
    L->off_hacc = x; x = align256(x + (size_t)4 * L->bins * sizeof(unsigned long long));
    L->need_lw = reduce && !o.log_w;
    L->need_r2 = reduce && !o.r2;
    L->need_rg2 = reduce && !o.rg2;
    L->need_ng = reduce && !o.n_grown;
    L->need_wx = reduce && L->exact && !o.w_exact;
    L->need_nn = reduce && L->exact && !o.n2rg2;
    L->off_lw = x; if (L->need_lw) x = align256(x + M * sizeof(double));
    L->off_r2 = x; if (L->need_r2) x = align256(x + M * sizeof(double));
    L->off_rg2 = x; if (L->need_rg2) x = align256(x + M * sizeof(double));
    L->off_ng = x; if (L->need_ng) x = align256(x + M * sizeof(uint16_t));
    L->off_wx = x; if (L->need_wx) x = align256(x + M * sizeof(uint64_t));
    L->off_nn = x; if (L->need_nn) x = align256(x + M * sizeof(int64_t));
    L->n_slots = L->lattice ? 0u : rsaw::real_hbm_slots(cfg->n_monomers, M);
    L->off_slots = x;
    x = align256(x + (size_t)L->n_slots * 3 * (size_t)cfg->n_monomers * sizeof(double));
    *off = x;
}

// Workspace bytes that every call needs: those of an empty ensemble with a
// reduction (its cells and summary).
size_t min_workspace_bytes()
{
    rsaw_config c;
    std::memset(&c, 0, sizeof(c));
    c.geometry = RSAW_LATTICE_SC;
    c.n_monomers = 1;
    c.k_trials = 6;
    c.coord_type = RSAW_I32;
    rsaw_chain_out none{};
    EnsLayout L;
    size_t off = 0;
    layout_ensemble(&c, none, true, &off, &L);
    return off;
}

// The per-chain arrays the kernels write: the caller's, completed with
// workspace arrays where the reduction needs them.
rsaw_chain_out bind_outputs(const rsaw_chain_out &in, const EnsLayout &L, char *ws)
{
    rsaw_chain_out o = in;
    if (L.need_lw) o.log_w = (double *)(ws + L.off_lw);
    if (L.need_r2) o.r2 = (double *)(ws + L.off_r2);
    if (L.need_rg2) o.rg2 = (double *)(ws + L.off_rg2);
    if (L.need_ng) o.n_grown = (uint16_t *)(ws + L.off_ng);
    if (L.need_wx) o.w_exact = (uint64_t *)(ws + L.off_wx);
    if (L.need_nn) o.n2rg2 = (int64_t *)(ws + L.off_nn);
    if (!L.lattice) o.n2rg2 = nullptr;
    if (!L.exact) o.w_exact = nullptr;
    return o;
}

// |coordinate| at which the boxed lattice kernels regrow a chain in wide
// words, 0 for each format's own edge (rsaw_set_byte_box).
std::atomic<int32_t> g_byte_box{0};

rsaw::GrowArgs grow_args(const rsaw_config *cfg, const rsaw_chain_out &o, const EnsLayout &L, char *ws)
{
    rsaw::GrowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seed = cfg->seed;
    a.chain_offset = cfg->chain_offset;
    a.n_chains = cfg->n_chains;
    a.n_monomers = cfg->n_monomers;
    a.k_trials = cfg->k_trials;
    a.bond_length = cfg->bond_length;
    a.sigma2 = cfg->bead_diameter * cfg->bead_diameter;
    const double bs = cfg->bond_length + cfg->bead_diameter;
    a.cull2 = bs * bs * (1.0 + 0x1p-30);
    a.max_rounds = (cfg->flags & RSAW_RESTART) ? 65536u : 1u;
    a.byte_box = g_byte_box.load(std::memory_order_relaxed);
    a.bead_slots = L.n_slots ? (double *)(ws + L.off_slots) : nullptr;
    a.n_slots = L.n_slots;
    a.log_w = o.log_w;
    a.w_exact = o.w_exact;
    a.r_end = o.r_end;
    a.r2 = o.r2;
    a.rg2 = o.rg2;
    a.n2rg2 = o.n2rg2;
    a.n_grown = o.n_grown;
    a.log_w_max_bits = (unsigned long long *)(ws + L.off_lmax);
    a.status = (int32_t *)(ws + L.off_status);
    std::memcpy(a.logm, logm_table(), sizeof(a.logm));
    return a;
}

rsaw::ReduceArgs reduce_args(const rsaw_config *cfg, const rsaw_chain_out &o, const EnsLayout &L, char *ws)
{
    rsaw::ReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.n_chains = cfg->n_chains;
    r.chunk = L.chunk;
    r.n_monomers = cfg->n_monomers;
    r.bins = L.bins;
    r.exact = L.exact ? 1 : 0;
    r.log_w = o.log_w;
    r.r2 = o.r2;
    r.rg2 = o.rg2;
    r.n_grown = o.n_grown;
    r.w_exact = o.w_exact;
    r.n2rg2 = o.n2rg2;
    r.lmax_bits = (unsigned long long *)(ws + L.off_lmax);
    r.status = (int32_t *)(ws + L.off_status);
    r.partials = (rsaw::BlockPartial *)(ws + L.off_part);
    r.hist_acc = (unsigned long long *)(ws + L.off_hacc);
    return r;
}

// Shared body of the single-ensemble entry points.  With force_reduce the
// summary goes to the workspace when the caller gives no device summary;
// *used_summary receives the device address the summary was written to (or
// NULL).
// With fixed_ws set, the call uses that buffer of fixed_bytes instead of the
// stream's workspace, allocates nothing and records no timing events.
rsaw_status gen_impl(const rsaw_config *cfg, const rsaw_chain_out *out, rsaw_summary *d_summary,
                     double *d_hist_w, uint64_t *d_hist_n, void *stream, bool force_reduce,
                     rsaw_summary **used_summary, void *fixed_ws = nullptr, size_t fixed_bytes = 0)
{
    g_last_error.clear();
    if (used_summary) *used_summary = nullptr;
    rsaw_status st = validate(cfg);
    if (st != RSAW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

    const bool reduce = force_reduce || d_summary != nullptr || d_hist_w != nullptr || d_hist_n != nullptr;
    rsaw_chain_out in{};
    if (out) in = *out;
    EnsLayout L;
    size_t off = 0;
    layout_ensemble(cfg, in, reduce, &off, &L);
    void *wsv = nullptr;
    if (fixed_ws) {
        if (off > fixed_bytes)
            return fail(RSAW_E_NOMEM, "this call needs " + std::to_string(off) +
                                          " bytes of workspace (rsaw_workspace_size); the static scratch holds " +
                                          std::to_string(fixed_bytes));
        wsv = fixed_ws;
    } else {
        st = workspace(dev, s, off, &wsv);
        if (st != RSAW_OK) return st;
    }
    char *ws = (char *)wsv;
    const rsaw_chain_out o = bind_outputs(in, L, ws);

    e = rsaw::launch_reduce_init((unsigned long long *)(ws + L.off_lmax), (int32_t *)(ws + L.off_status),
                                 (unsigned long long *)(ws + L.off_hacc), 4 * L.bins, s);
    if (e != hipSuccess) return hip_fail(e, "reduce_init launch");

    if (cfg->n_chains > 0) {
        const rsaw::GrowArgs a = grow_args(cfg, o, L, ws);
        EventPair tp;
        bool timed = false;
        if (!fixed_ws) {
            st = timing_start(s, &tp, &timed);
            if (st != RSAW_OK) return st;
        }
        const bool i16 = cfg->coord_type == RSAW_I16;
        e = L.z26       ? rsaw::launch_grow_lattice26(a, L.exact, i16, s)
            : L.lattice ? rsaw::launch_grow_lattice(a, L.exact, i16, s)
                        : rsaw::launch_grow_real(a, s);
        if (timed) {
            st = timing_stop(s, tp);
            if (st != RSAW_OK) return st;
        }
        if (e != hipSuccess) return hip_fail(e, "grow kernel launch");
    }

    if (reduce) {
        const rsaw::ReduceArgs r = reduce_args(cfg, o, L, ws);
        rsaw_summary *dsum = d_summary ? d_summary : (rsaw_summary *)(ws + L.off_summary);
        e = rsaw::launch_reduce(r, L.n_blocks, dsum, d_hist_w, d_hist_n, s);
        if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
        if (used_summary) *used_summary = dsum;
    }
    return RSAW_OK;
}

// Growth-kernel variant (kernel family, template parameters, block shape)
// of one ensemble, as its launch would choose it.
hipError_t ensemble_variant(const rsaw_config *cfg, const EnsLayout &L, rsaw::GrowVariant *v)
{
    rsaw::GrowArgs probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.n_monomers = cfg->n_monomers;
    probe.k_trials = cfg->k_trials;
    const bool i16 = cfg->coord_type == RSAW_I16;
    if (!L.lattice) return rsaw::real_variant(probe, v);
    if (L.z26) return rsaw::lattice26_variant(probe, L.exact, i16, v);
    if (L.exact || cfg->n_monomers <= 64) {
        rsaw::lattice_reg_variant(probe, L.exact, i16, v);
        return hipSuccess;
    }
    return rsaw::lattice_lds_variant(probe, i16, v);
}

// Everything the launches of a batch need once its tables are on the device:
// the growth groups and the reduction's segment tables.
struct BatchGroup {
    rsaw::GrowVariant v;
    int32_t first, cnt;
    uint64_t blocks;
    size_t shmem;
    std::vector<rsaw::GrowArgs> hbm; // hard spheres with HBM planes: one grid per ensemble
};
struct BatchLaunch {
    std::vector<BatchGroup> groups;
    const rsaw::GrowEntry *d_gtab = nullptr;
    const uint64_t *d_gb0 = nullptr;
    const rsaw::ReduceEntry *d_rtab = nullptr;
    const uint64_t *d_rb0 = nullptr;
    int32_t n = 0;
    uint64_t rb = 0;
    int max_bins = 0;
    bool reduce = false;
};

// Enqueues the batch's launches on s: zero the accumulators, one growth
// launch per group, the segmented reduction.  Kernel launches only.
rsaw_status run_batch(const BatchLaunch &B, hipStream_t s)
{
    if (B.n == 0) return RSAW_OK;
    hipError_t e = rsaw::launch_reduce_batch(B.d_rtab, B.d_rb0, B.n, 0, 0, s, true);
    if (e != hipSuccess) return hip_fail(e, "batched reduce_init launch");
    for (const BatchGroup &G : B.groups) {
        const rsaw::GrowVariant &v = G.v;
        EventPair tp;
        bool timed = false;
        rsaw_status st = timing_start(s, &tp, &timed);
        if (st != RSAW_OK) return st;
        if (v.family == 2 && v.p1) {
            for (size_t q = 0; q < G.hbm.size() && e == hipSuccess; ++q) e = rsaw::launch_grow_real(G.hbm[q], s);
        } else if (v.family == 0)
            e = rsaw::launch_lattice_reg_batch(v, B.d_gtab + G.first, B.d_gb0 + G.first, G.cnt, G.blocks, s);
        else if (v.family == 1)
            e = rsaw::launch_lattice_lds_batch(v, B.d_gtab + G.first, B.d_gb0 + G.first, G.cnt, G.blocks, G.shmem,
                                               s);
        else if (v.family == 3)
            e = rsaw::launch_lattice26_batch(v, B.d_gtab + G.first, B.d_gb0 + G.first, G.cnt, G.blocks, G.shmem, s);
        else
            e = rsaw::launch_real_batch(v, B.d_gtab + G.first, B.d_gb0 + G.first, G.cnt, G.blocks, G.shmem, s);
        if (timed) {
            st = timing_stop(s, tp);
            if (st != RSAW_OK) return st;
        }
        if (e != hipSuccess) return hip_fail(e, "batched grow kernel launch");
    }
    if (B.reduce) {
        e = rsaw::launch_reduce_batch(B.d_rtab, B.d_rb0, B.n, B.rb, B.max_bins, s, false);
        if (e != hipSuccess) return hip_fail(e, "batched reduce kernel launch");
    }
    return RSAW_OK;
}

// A batch prepared once (own workspace, tables already on the device) and
// launched any number of times, e.g. inside a HIP graph capture.
struct PlannedBatch {
    int dev = 0;
    void *ws = nullptr;
    BatchLaunch B;
};

// Batched body: every ensemble's growth shares one launch per kernel
// variant, and the reductions three launches in all.
// With `plan` set, nothing is enqueued: the workspace is the plan's own
// allocation, the tables are copied synchronously, and the launch
// description goes to *plan.
rsaw_status batch_impl(const rsaw_config *cfgs, const rsaw_chain_out *outs, int32_t n,
                       rsaw_summary *d_summaries, double *const *d_hist_w, uint64_t *const *d_hist_n,
                       void *stream, PlannedBatch *plan = nullptr)
{
    g_last_error.clear();
    if (n < 0) return fail(RSAW_E_INVALID, "n must be >= 0");
    if (n == 0) return RSAW_OK;
    if (!cfgs) return fail(RSAW_E_INVALID, "cfgs is NULL");
    for (int32_t i = 0; i < n; ++i) {
        rsaw_status st = validate(&cfgs[i]);
        if (st != RSAW_OK) return fail(st, "ensemble " + std::to_string(i) + ": " + g_last_error);
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const bool reduce = d_summaries != nullptr;

    // layouts and kernel variants
    std::vector<EnsLayout> L(n);
    std::vector<rsaw_chain_out> in(n);
    std::vector<rsaw::GrowVariant> var(n);
    size_t off = 0;
    int max_bins = 0;
    for (int32_t i = 0; i < n; ++i) {
        in[i] = outs ? outs[i] : rsaw_chain_out{};
        layout_ensemble(&cfgs[i], in[i], reduce, &off, &L[i]);
        max_bins = std::max(max_bins, L[i].bins);
        e = ensemble_variant(&cfgs[i], L[i], &var[i]);
        if (e != hipSuccess) return fail(RSAW_E_UNSUPPORTED, "ensemble " + std::to_string(i) + ": no kernel variant");
    }
    // ensembles with chains, grouped by variant (stable: index order within a
    // group).  A launch gives every block the largest LDS of its ensembles.
    // An ensemble that fills the GPU by itself (at least one block per slot
    // that its own LDS leaves on every CU: 160 KiB / shmem per CU, capped at
    // the 32 waves a CU holds) shares a launch only with ensembles of the
    // same blocks per CU, so it keeps its occupancy instead of running at
    // that of the longest chains in the batch.  Smaller ensembles cannot
    // fill the CUs alone and share one launch per variant, as few launches
    // as possible.
    int n_cu = 256;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        n_cu = 256;
    std::vector<int32_t> order;
    std::vector<uint64_t> per_cu(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (cfgs[i].n_chains == 0) continue;
        order.push_back(i);
        const rsaw::GrowVariant &v = var[i];
        const uint64_t cap = 2048 / (uint64_t)v.threads;
        const uint64_t slots = v.shmem ? std::min((uint64_t)(163840 / v.shmem), cap) : cap;
        const uint64_t blocks = (cfgs[i].n_chains + v.cpb - 1) / v.cpb;
        per_cu[i] = blocks >= slots * (uint64_t)n_cu ? slots : 0;
    }
    auto key = [&](int32_t i) {
        const rsaw::GrowVariant &v = var[i];
        return std::make_tuple(v.family, v.p0, v.p1, v.p2, v.threads, per_cu[i]);
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
    const int32_t ng = (int32_t)order.size();

    // device tables after the ensembles' regions
    const size_t off_gtab = align256(off);
    const size_t off_gb0 = align256(off_gtab + (size_t)ng * sizeof(rsaw::GrowEntry));
    const size_t off_rtab = align256(off_gb0 + (size_t)(ng + 1) * sizeof(uint64_t));
    const size_t off_rb0 = align256(off_rtab + (size_t)n * sizeof(rsaw::ReduceEntry));
    const size_t off_end = align256(off_rb0 + (size_t)(n + 1) * sizeof(uint64_t));
    const size_t tab_bytes = off_end - off_gtab;
    void *wsv = nullptr;
    rsaw_status st = RSAW_OK;
    std::vector<char> plan_stage;
    void *stv = nullptr;
    hipEvent_t stage_done = nullptr;
    if (plan) {
        e = hipMalloc(&wsv, off_end);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(RSAW_E_NOMEM, std::string("plan hipMalloc: ") + hipGetErrorString(e));
        }
        plan->dev = dev;
        plan->ws = wsv;
        plan_stage.resize(tab_bytes);
        stv = plan_stage.data();
    } else {
        st = workspace(dev, s, off_end, &wsv);
        if (st != RSAW_OK) return st;
        st = staging(dev, s, tab_bytes, &stv, &stage_done);
        if (st != RSAW_OK) return st;
    }
    char *ws = (char *)wsv;
    char *stage = (char *)stv;
    rsaw::GrowEntry *gtab = (rsaw::GrowEntry *)(stage + (off_gtab - off_gtab));
    uint64_t *gb0 = (uint64_t *)(stage + (off_gb0 - off_gtab));
    rsaw::ReduceEntry *rtab = (rsaw::ReduceEntry *)(stage + (off_rtab - off_gtab));
    uint64_t *rb0 = (uint64_t *)(stage + (off_rb0 - off_gtab));

    std::vector<rsaw_chain_out> o(n);
    for (int32_t i = 0; i < n; ++i) o[i] = bind_outputs(in[i], L[i], ws);
    // growth groups: [first, last) in `order`, blocks and largest LDS
    struct Group { int32_t first, last; uint64_t blocks; size_t shmem; };
    std::vector<Group> groups;
    uint64_t b = 0;
    for (int32_t q = 0; q < ng; ++q) {
        const int32_t i = order[q];
        if (q == 0 || key(i) != key(order[q - 1])) {
            groups.push_back(Group{q, q, 0, 0});
            b = 0;
        }
        Group &G = groups.back();
        gtab[q].a = grow_args(&cfgs[i], o[i], L[i], ws);
        gtab[q].H = var[i].H;
        gtab[q].S = var[i].S;
        gb0[q] = b;
        b += (cfgs[i].n_chains + var[i].cpb - 1) / var[i].cpb;
        G.last = q + 1;
        G.blocks = b;
        G.shmem = std::max(G.shmem, var[i].shmem);
    }
    gb0[ng] = 0;
    uint64_t rb = 0;
    for (int32_t i = 0; i < n; ++i) {
        rsaw::ReduceEntry &r = rtab[i];
        std::memset(&r, 0, sizeof(r));
        r.r = reduce_args(&cfgs[i], o[i], L[i], ws);
        r.n_blocks = L[i].n_blocks;
        r.lmax = (unsigned long long *)(ws + L[i].off_lmax);
        r.status = (int32_t *)(ws + L[i].off_status);
        r.out = reduce ? d_summaries + i : nullptr;
        r.hist_w = (reduce && d_hist_w) ? d_hist_w[i] : nullptr;
        r.hist_n = (reduce && d_hist_n) ? d_hist_n[i] : nullptr;
        rb0[i] = rb;
        rb += L[i].n_blocks;
    }
    rb0[n] = rb;

    if (plan) {
        e = hipMemcpy(ws + off_gtab, stage, tab_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "plan table copy");
    } else {
        e = hipMemcpyAsync(ws + off_gtab, stage, tab_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "batch table copy");
        e = hipEventRecord(stage_done, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    const rsaw::GrowEntry *d_gtab = (const rsaw::GrowEntry *)(ws + off_gtab);
    const uint64_t *d_gb0 = (const uint64_t *)(ws + off_gb0);
    const rsaw::ReduceEntry *d_rtab = (const rsaw::ReduceEntry *)(ws + off_rtab);
    const uint64_t *d_rb0 = (const uint64_t *)(ws + off_rb0);

    BatchLaunch B;
    B.d_gtab = d_gtab;
    B.d_gb0 = d_gb0;
    B.d_rtab = d_rtab;
    B.d_rb0 = d_rb0;
    B.n = n;
    B.rb = rb;
    B.max_bins = max_bins;
    B.reduce = reduce;
    for (const Group &G : groups) {
        BatchGroup g;
        g.v = var[order[G.first]];
        g.first = G.first;
        g.cnt = G.last - G.first;
        g.blocks = G.blocks;
        g.shmem = G.shmem;
        if (g.v.family == 2 && g.v.p1)
            for (int32_t q = G.first; q < G.last; ++q) g.hbm.push_back(gtab[q].a);
        B.groups.push_back(std::move(g));
    }
    if (plan) {
        plan->B = std::move(B);
        return RSAW_OK;
    }
    return run_batch(B, s);
}

} // namespace

// ---- tuning table of the group kernels' lane mapping --------------------
namespace {
std::mutex g_map_lock;
std::vector<rsaw_mapping> g_map; // newest last
// The autotuner's candidate, forced on its own thread while it is timed.
thread_local bool t_force = false;
thread_local int t_force_lanes = 0, t_force_threads = 0;

struct ForceMapping {
    ForceMapping(int lanes, int threads)
    {
        t_force = true;
        t_force_lanes = lanes;
        t_force_threads = threads;
    }
    ~ForceMapping() { t_force = false; }
};

// Mapping a call with cfg launches its growth kernel with (host-only).
rsaw_status query_mapping(const rsaw_config *cfg, rsaw_mapping *m)
{
    rsaw_chain_out none{};
    EnsLayout L;
    size_t off = 0;
    layout_ensemble(cfg, none, false, &off, &L);
    rsaw::GrowVariant v;
    if (ensemble_variant(cfg, L, &v) != hipSuccess) return fail(RSAW_E_UNSUPPORTED, "no kernel variant");
    m->geometry = cfg->geometry;
    m->k_trials = cfg->k_trials;
    m->n_lo = m->n_hi = cfg->n_monomers;
    // register lattice (family 0) and 26-neighbour lane kernel: one lane per chain
    m->lanes = v.family == 0 || (v.family == 3 && v.p0 == 1) ? 1 : v.p0;
    m->threads = v.threads;
    m->lds_bytes = v.shmem;
    return RSAW_OK;
}

// True when (lanes, threads) is what a group kernel launches for cfg with
// that mapping forced, i.e. the mapping is legal for cfg.
bool mapping_legal(const rsaw_config *cfg, int lanes, int threads, rsaw_mapping *got)
{
    if (lanes < 2) return false; // one-lane kernels have no group mapping
    ForceMapping f(lanes, threads);
    if (query_mapping(cfg, got) != RSAW_OK) return false;
    return got->lanes == lanes && got->threads == threads;
}
} // namespace

namespace rsaw {
bool tuned_mapping(int geometry, int n_monomers, int k_trials, int *lanes, int *threads)
{
    if (t_force) {
        *lanes = t_force_lanes;
        *threads = t_force_threads;
        return true;
    }
    std::lock_guard<std::mutex> lk(g_map_lock);
    for (auto it = g_map.rbegin(); it != g_map.rend(); ++it) {
        if (it->geometry == geometry && it->k_trials == k_trials && it->n_lo <= n_monomers &&
            n_monomers <= it->n_hi) {
            *lanes = it->lanes;
            *threads = it->threads;
            return true;
        }
    }
    return false;
}
} // namespace rsaw

namespace rsaw {
// The argument checks of rsaw_gen_chains, for the serving loop's submit.
rsaw_status check_config(const rsaw_config *cfg)
{
    g_last_error.clear();
    return validate(cfg);
}

// Device workspace bytes one ensemble holds in an rsaw_gen_batch call with no
// per-chain outputs and a reduction: its regions (the layout that
// rsaw_workspace_size reports) and its entries of the descriptor tables.  A
// batch needs at most the sum over its ensembles plus kBatchFixedBytes (the
// alignment of its four tables and their two end entries).
size_t batch_entry_bytes(const rsaw_config *cfg)
{
    rsaw_chain_out none{};
    EnsLayout L;
    size_t off = 0;
    layout_ensemble(cfg, none, true, &off, &L);
    return off + sizeof(GrowEntry) + sizeof(ReduceEntry) + 2 * sizeof(uint64_t);
}

// Pinned staging of the batch tables of (current device, s), grown to at
// least `bytes` now rather than on a later call (which would free and
// reallocate it while batches run).
rsaw_status reserve_staging(hipStream_t s, size_t bytes)
{
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void *stage = nullptr;
    hipEvent_t done = nullptr;
    return staging(dev, s, bytes, &stage, &done);
}

// Forget the (current device, s) entry: free its internal workspace, its
// staging buffer and event (a caller workspace stays the caller's).  For a
// stream about to be destroyed; waits for its queued work first.
rsaw_status release_stream(hipStream_t s)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    Workspace w;
    {
        std::lock_guard<std::mutex> lk(g_ws_lock);
        auto it = g_ws.find({dev, (void *)s});
        if (it == g_ws.end()) return RSAW_OK;
        w = it->second;
        g_ws.erase(it);
    }
    if (w.base && !w.external) (void)hipFree(w.base);
    if (w.stage) (void)hipHostFree(w.stage);
    if (w.stage_done) (void)hipEventDestroy(w.stage_done);
    return RSAW_OK;
}

// Scratch of rsaw_gen_chains_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it is a stand-in, not a device address);
// it uses the address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_lock;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up on the
// first call there.
rsaw_status static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(RSAW_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RSAW_OK;
}

// Staging bytes of the tables of a batch of n ensembles.
size_t batch_stage_bytes(int n)
{
    return (size_t)n * (sizeof(GrowEntry) + sizeof(ReduceEntry) + 2 * sizeof(uint64_t)) + kBatchFixedBytes;
}
} // namespace rsaw

extern "C" {

rsaw_status rsaw_gen_chains(const rsaw_config *cfg, const rsaw_chain_out *out,
                            rsaw_summary *d_summary, double *d_hist_w, uint64_t *d_hist_n,
                            void *stream)
{
    return gen_impl(cfg, out, d_summary, d_hist_w, d_hist_n, stream, false, nullptr);
}

rsaw_status rsaw_gen_chains_static(const rsaw_config *cfg, const rsaw_chain_out *out,
                                   rsaw_summary *d_summary, double *d_hist_w, uint64_t *d_hist_n,
                                   void *stream)
{
    g_last_error.clear();
    rsaw_status st = validate(cfg);
    if (st != RSAW_OK) return st;
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void *ws = nullptr;
    st = rsaw::static_scratch(dev, &ws);
    if (st != RSAW_OK) return st;
    return gen_impl(cfg, out, d_summary, d_hist_w, d_hist_n, stream, false, nullptr, ws, rsaw::kStaticScratchBytes);
}

rsaw_status rsaw_gen_chains_sync(const rsaw_config *cfg, const rsaw_chain_out *out,
                                 rsaw_summary *h_summary, double *d_hist_w, uint64_t *d_hist_n,
                                 void *stream)
{
    g_last_error.clear();
    if (!h_summary) return fail(RSAW_E_INVALID, "h_summary is NULL");
    hipStream_t s = (hipStream_t)stream;
    rsaw_summary *d = nullptr;
    rsaw_status st = gen_impl(cfg, out, nullptr, d_hist_w, d_hist_n, stream, true, &d);
    if (st != RSAW_OK) return st;
    hipError_t e = hipMemcpyAsync(h_summary, d, sizeof(rsaw_summary), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "summary copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (h_summary->status != RSAW_OK) return fail((rsaw_status)h_summary->status, "rejection cap reached");
    return RSAW_OK;
}

rsaw_status rsaw_gen_batch(const rsaw_config *cfgs, const rsaw_chain_out *outs, int32_t n,
                           rsaw_summary *d_summaries, double *const *d_hist_w,
                           uint64_t *const *d_hist_n, void *stream)
{
    return batch_impl(cfgs, outs, n, d_summaries, d_hist_w, d_hist_n, stream);
}

struct rsaw_batch_plan {
    PlannedBatch p;
};

rsaw_status rsaw_batch_plan_create(const rsaw_config *cfgs, const rsaw_chain_out *outs, int32_t n,
                                   rsaw_summary *d_summaries, double *const *d_hist_w,
                                   uint64_t *const *d_hist_n, rsaw_batch_plan **plan)
{
    g_last_error.clear();
    if (!plan) return fail(RSAW_E_INVALID, "plan is NULL");
    *plan = nullptr;
    rsaw_batch_plan *pl = new rsaw_batch_plan();
    const rsaw_status st = batch_impl(cfgs, outs, n, d_summaries, d_hist_w, d_hist_n, nullptr, &pl->p);
    if (st != RSAW_OK) {
        if (pl->p.ws) (void)hipFree(pl->p.ws);
        delete pl;
        return st;
    }
    if (!pl->p.ws) (void)hipGetDevice(&pl->p.dev); // n = 0: nothing to launch
    *plan = pl;
    return RSAW_OK;
}

rsaw_status rsaw_batch_plan_launch(const rsaw_batch_plan *plan, void *stream)
{
    g_last_error.clear();
    if (!plan) return fail(RSAW_E_INVALID, "plan is NULL");
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != plan->p.dev)
        return fail(RSAW_E_INVALID, "the plan was created on device " + std::to_string(plan->p.dev));
    return run_batch(plan->p.B, (hipStream_t)stream);
}

void rsaw_batch_plan_destroy(rsaw_batch_plan *plan)
{
    if (!plan) return;
    if (plan->p.ws) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(plan->p.dev);
        (void)hipFree(plan->p.ws);
        (void)hipSetDevice(cur);
    }
    delete plan;
}

const char *rsaw_status_string(rsaw_status s)
{
    switch (s) {
    case RSAW_OK: return "ok";
    case RSAW_E_INVALID: return "invalid argument";
    case RSAW_E_UNSUPPORTED: return "unsupported configuration";
    case RSAW_E_OVERFLOW: return "exact weight would overflow 64 bits";
    case RSAW_E_NOMEM: return "device allocation failed";
    case RSAW_E_DEVICE: return "HIP runtime error";
    case RSAW_E_RNG: return "rejection loop reached its attempt cap";
    }
    return "unknown status";
}

const char *rsaw_last_error(void) { return g_last_error.c_str(); }

int32_t rsaw_version(void) { return 100; }

rsaw_status rsaw_kernel_timing(int32_t enable)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_tm_lock);
    g_tm_enabled = enable != 0;
    return RSAW_OK;
}

rsaw_status rsaw_kernel_time(double *total_ms, uint64_t *launches)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_tm_lock);
    double sum = 0.0;
    uint64_t n = 0;
    rsaw_status st = RSAW_OK;
    for (const EventPair &p : g_tm_recorded) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e != hipSuccess && st == RSAW_OK) st = hip_fail(e, "kernel timing event");
        sum += ms;
        ++n;
        g_tm_free.push_back(p);
    }
    g_tm_recorded.clear();
    if (total_ms) *total_ms = sum;
    if (launches) *launches = n;
    return st;
}

rsaw_status rsaw_workspace_size(const rsaw_config *cfg, const rsaw_chain_out *out, int32_t reduce,
                                size_t *bytes)
{
    g_last_error.clear();
    if (!bytes) return fail(RSAW_E_INVALID, "bytes is NULL");
    const rsaw_status st = validate(cfg);
    if (st != RSAW_OK) return st;
    rsaw_chain_out in{};
    if (out) in = *out;
    EnsLayout L;
    size_t off = 0;
    layout_ensemble(cfg, in, reduce != 0, &off, &L);
    *bytes = off;
    return RSAW_OK;
}

rsaw_status rsaw_set_workspace(void *d_ws, size_t bytes, void *stream)
{
    g_last_error.clear();
    hipStream_t s = (hipStream_t)stream;
    if (d_ws) {
        if ((uintptr_t)d_ws & 255) return fail(RSAW_E_INVALID, "d_ws must be 256-byte aligned");
        const size_t least = min_workspace_bytes();
        if (bytes < least)
            return fail(RSAW_E_INVALID, "a workspace needs at least " + std::to_string(least) + " bytes");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (d_ws) {
        hipPointerAttribute_t at;
        std::memset(&at, 0, sizeof(at));
        e = hipPointerGetAttributes(&at, d_ws);
        if (e != hipSuccess) {
            (void)hipGetLastError(); // an unknown pointer is an argument error, not a device fault
            return fail(RSAW_E_INVALID, "d_ws is not device memory known to HIP");
        }
        if ((at.type != hipMemoryTypeDevice && !at.isManaged) || at.device != dev)
            return fail(RSAW_E_INVALID, "d_ws must be device memory of the current device " + std::to_string(dev));
    }
    Workspace &w = ws_entry(dev, s);
    if (!w.external && w.base) {
        // the internal buffer may still be in use by work queued on the stream
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipFree(w.base);
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    w.base = d_ws;
    w.bytes = d_ws ? bytes : 0;
    w.external = d_ws != nullptr;
    return RSAW_OK;
}

void rsaw_shutdown(void)
{
    {
        std::lock_guard<std::mutex> lk(g_tm_lock);
        for (auto *v : {&g_tm_recorded, &g_tm_free}) {
            for (const EventPair &p : *v) {
                (void)hipEventSynchronize(p.stop);
                (void)hipEventDestroy(p.start);
                (void)hipEventDestroy(p.stop);
            }
            v->clear();
        }
    }
    std::lock_guard<std::mutex> lk(g_ws_lock);
    for (auto &kv : g_ws) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        if (kv.second.base && !kv.second.external) (void)hipFree(kv.second.base);
        if (kv.second.stage) (void)hipHostFree(kv.second.stage);
        if (kv.second.stage_done) (void)hipEventDestroy(kv.second.stage_done);
        (void)hipSetDevice(cur);
    }
    g_ws.clear();
}

rsaw_status rsaw_mapping_set(const rsaw_mapping *m)
{
    g_last_error.clear();
    if (!m) return fail(RSAW_E_INVALID, "mapping is NULL");
    if (m->n_lo < 1 || m->n_hi < m->n_lo) return fail(RSAW_E_INVALID, "need 1 <= n_lo <= n_hi");
    rsaw_config c;
    std::memset(&c, 0, sizeof(c));
    c.geometry = m->geometry;
    c.n_monomers = m->n_hi;
    c.k_trials = m->k_trials;
    c.coord_type = m->geometry == RSAW_REAL_HS ? RSAW_F64 : RSAW_I32;
    c.n_chains = 1;
    c.bond_length = 1.0;
    c.bead_diameter = 1.0;
    rsaw_status st = validate(&c);
    if (st != RSAW_OK) return st;
    rsaw_mapping got;
    if (!mapping_legal(&c, m->lanes, m->threads, &got))
        return fail(RSAW_E_INVALID, "lanes " + std::to_string(m->lanes) + ", threads " +
                                        std::to_string(m->threads) + " is not a legal mapping at N = " +
                                        std::to_string(m->n_hi));
    rsaw_mapping e = *m;
    e.lds_bytes = 0;
    std::lock_guard<std::mutex> lk(g_map_lock);
    g_map.push_back(e);
    return RSAW_OK;
}

rsaw_status rsaw_set_byte_box(int32_t edge)
{
    if (edge < 0 || edge > 127) return fail(RSAW_E_INVALID, "byte box edge must be in 0..127");
    g_byte_box.store(edge, std::memory_order_relaxed);
    return RSAW_OK;
}

void rsaw_mapping_clear(void)
{
    std::lock_guard<std::mutex> lk(g_map_lock);
    g_map.clear();
}

rsaw_status rsaw_mapping_list(rsaw_mapping *out, int32_t capacity, int32_t *count)
{
    g_last_error.clear();
    if (!count) return fail(RSAW_E_INVALID, "count is NULL");
    if (capacity < 0 || (capacity > 0 && !out)) return fail(RSAW_E_INVALID, "bad output array");
    std::lock_guard<std::mutex> lk(g_map_lock);
    *count = (int32_t)g_map.size();
    const size_t n = std::min(g_map.size(), (size_t)capacity);
    for (size_t i = 0; i < n; ++i) out[i] = g_map[i];
    return RSAW_OK;
}

rsaw_status rsaw_mapping_query(const rsaw_config *cfg, rsaw_mapping *m)
{
    g_last_error.clear();
    if (!m) return fail(RSAW_E_INVALID, "m is NULL");
    const rsaw_status st = validate(cfg);
    if (st != RSAW_OK) return st;
    return query_mapping(cfg, m);
}

// Relative speed-up a tuned mapping needs over the mapping in force.
constexpr double kTuneMargin = 0.03;

rsaw_status rsaw_autotune(const rsaw_config *base, const int32_t *n_edges, int32_t n_buckets,
                          int32_t reps, rsaw_mapping *chosen, double *best_ms, void *stream)
{
    g_last_error.clear();
    if (!base) return fail(RSAW_E_INVALID, "base is NULL");
    if (!n_edges || n_buckets < 1 || n_buckets > 64) return fail(RSAW_E_INVALID, "need 1..64 buckets");
    if (reps < 1 || reps > 100) return fail(RSAW_E_INVALID, "reps must be 1..100");
    for (int32_t b = 0; b < n_buckets; ++b) {
        if (n_edges[b] < 1 || (b > 0 && n_edges[b] <= n_edges[b - 1]))
            return fail(RSAW_E_INVALID, "n_edges must be positive and strictly increasing");
        rsaw_config c = *base;
        c.n_monomers = n_edges[b];
        const rsaw_status st = validate(&c);
        if (st != RSAW_OK) return fail(st, "bucket " + std::to_string(b) + ": " + g_last_error);
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        return hip_fail(e, "hipEventCreate");
    }
    rsaw_status st = RSAW_OK;
    // one untimed call, then reps calls between two events
    auto time_calls = [&](const rsaw_config &c, double *ms) -> rsaw_status {
        rsaw_status r = gen_impl(&c, nullptr, nullptr, nullptr, nullptr, stream, true, nullptr);
        if (r != RSAW_OK) return r;
        hipError_t he = hipEventRecord(ev0, s);
        for (int32_t q = 0; q < reps && he == hipSuccess; ++q) {
            r = gen_impl(&c, nullptr, nullptr, nullptr, nullptr, stream, true, nullptr);
            if (r != RSAW_OK) return r;
        }
        if (he == hipSuccess) he = hipEventRecord(ev1, s);
        if (he == hipSuccess) he = hipEventSynchronize(ev1);
        float t = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&t, ev0, ev1);
        if (he != hipSuccess) return hip_fail(he, "autotune timing");
        *ms = (double)t / reps;
        return RSAW_OK;
    };
    static const int kLanes[] = {2, 4, 8, 16, 32, 64};
    static const int kThreads[] = {64, 256};
    for (int32_t b = 0; b < n_buckets && st == RSAW_OK; ++b) {
        rsaw_config c = *base;
        c.n_monomers = n_edges[b];
        rsaw_mapping win;
        st = query_mapping(&c, &win);
        if (st != RSAW_OK) break;
        // the mapping in force (built-in rule or an earlier entry), timed
        // first: a candidate replaces it only when it is at least
        // kTuneMargin faster, so that timing noise does not move ensembles
        // away from a mapping that also suits co-scheduled launches
        const rsaw_mapping cur = win;
        double cur_ms = -1.0;
        if (cur.lanes >= 2) {
            ForceMapping f(cur.lanes, cur.threads);
            st = time_calls(c, &cur_ms);
            if (st != RSAW_OK) break;
        }
        double win_ms = -1.0;
        bool tuned = false;
        for (int lanes : kLanes) {
            for (int threads : kThreads) {
                rsaw_mapping got;
                if (!mapping_legal(&c, lanes, threads, &got)) continue;
                double ms = 0.0;
                {
                    ForceMapping f(lanes, threads);
                    st = time_calls(c, &ms);
                }
                if (st != RSAW_OK) break;
                if (win_ms < 0.0 || ms < win_ms) {
                    win_ms = ms;
                    win = got;
                }
                tuned = true;
            }
            if (st != RSAW_OK) break;
        }
        if (st != RSAW_OK) break;
        if (!tuned) {
            // no group kernel at this N: the built-in kernel, timed as is
            st = time_calls(c, &win_ms);
            if (st != RSAW_OK) break;
        } else if (cur_ms >= 0.0 && !(win_ms < cur_ms * (1.0 - kTuneMargin))) {
            win = cur; // no candidate clearly faster: keep the mapping in force
            win_ms = cur_ms;
            tuned = false;
        }
        win.n_lo = b == 0 ? 1 : n_edges[b - 1] + 1;
        win.n_hi = n_edges[b];
        if (tuned) {
            std::lock_guard<std::mutex> lk(g_map_lock);
            rsaw_mapping ins = win;
            ins.lds_bytes = 0;
            g_map.push_back(ins);
        }
        if (chosen) chosen[b] = win;
        if (best_ms) best_ms[b] = win_ms;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    return st;
}

} // extern "C"
