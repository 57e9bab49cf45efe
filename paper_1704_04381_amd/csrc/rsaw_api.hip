// C ABI of librsaw (declared in include/rsaw.h): argument validation,
// per-(device, stream) workspace, and the launch sequence
//   reduce_init -> grow_{lattice,real} -> reduce_partials -> reduce_final.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
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
int lattice_lds_max_monomers();
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
// demand; released by rsaw_shutdown().
struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
};

std::mutex g_ws_lock;
std::map<std::pair<int, void *>, Workspace> g_ws;

rsaw_status workspace(int dev, hipStream_t s, size_t need, void **out)
{
    std::lock_guard<std::mutex> lk(g_ws_lock);
    Workspace &w = g_ws[{dev, (void *)s}];
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
            return fail(RSAW_E_NOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        }
        w.bytes = sz;
    }
    *out = w.base;
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

rsaw_status validate(const rsaw_config *cfg)
{
    if (!cfg) return fail(RSAW_E_INVALID, "cfg is NULL");
    const int N = cfg->n_monomers;
    if (N < 1 || N > 65535) return fail(RSAW_E_INVALID, "n_monomers must be in 1..65535");
    if (cfg->n_chains >= (1ull << 32)) return fail(RSAW_E_INVALID, "n_chains must be below 2^32");
    if (cfg->hist_bins < 0) return fail(RSAW_E_INVALID, "hist_bins must be >= 0");
    if (cfg->hist_bins > rsaw::kMaxBins) return fail(RSAW_E_UNSUPPORTED, "hist_bins above 256");
    if (cfg->flags & ~RSAW_EXACT_W) return fail(RSAW_E_INVALID, "unknown flag bits");
    if (cfg->geometry == RSAW_LATTICE_SC) {
        if (cfg->k_trials != 6) return fail(RSAW_E_INVALID, "lattice needs k_trials == 6");
        if (cfg->coord_type != RSAW_I16 && cfg->coord_type != RSAW_I32)
            return fail(RSAW_E_INVALID, "lattice coord_type must be RSAW_I16 or RSAW_I32");
        if ((cfg->flags & RSAW_EXACT_W) && N > 28)
            return fail(RSAW_E_OVERFLOW, "RSAW_EXACT_W needs n_monomers <= 28");
        if (N > rsaw::lattice_lds_max_monomers())
            return fail(RSAW_E_UNSUPPORTED, "lattice kernels support n_monomers <= 16384");
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
            return fail(RSAW_E_UNSUPPORTED, "real-space kernel supports n_monomers <= 6144");
    } else {
        return fail(RSAW_E_INVALID, "unknown geometry");
    }
    return RSAW_OK;
}

// Shared body of the entry points.  With force_reduce the summary goes to the
// workspace when the caller gives no device summary; *used_summary receives
// the device address the summary was written to (or NULL).
rsaw_status gen_impl(const rsaw_config *cfg, const rsaw_chain_out *out, rsaw_summary *d_summary,
                     double *d_hist_w, uint64_t *d_hist_n, void *stream, bool force_reduce,
                     rsaw_summary **used_summary)
{
    g_last_error.clear();
    if (used_summary) *used_summary = nullptr;
    rsaw_status st = validate(cfg);
    if (st != RSAW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

    const uint64_t M = cfg->n_chains;
    const bool lattice = cfg->geometry == RSAW_LATTICE_SC;
    const bool exact = lattice && (cfg->flags & RSAW_EXACT_W);
    const bool reduce = force_reduce || d_summary != nullptr || d_hist_w != nullptr || d_hist_n != nullptr;
    const int bins = reduce ? cfg->hist_bins : 0;
    rsaw_chain_out o{};
    if (out) o = *out;

    // reduce blocks: at most 1024, each a contiguous run of whole 256-chain tiles
    uint32_t n_blocks = 0;
    uint64_t chunk = 256;
    if (M > 0) {
        const uint64_t tiles = (M + 255) / 256;
        const uint64_t nb = tiles < 1024 ? tiles : 1024;
        chunk = ((tiles + nb - 1) / nb) * 256;
        n_blocks = (uint32_t)((M + chunk - 1) / chunk);
    }

    // workspace layout
    size_t off = 0;
    const size_t off_lmax = off; off = align256(off + sizeof(unsigned long long));
    const size_t off_status = off; off = align256(off + sizeof(int32_t));
    const size_t off_summary = off; off = align256(off + sizeof(rsaw_summary));
    const size_t off_part = off; off = align256(off + (size_t)n_blocks * sizeof(rsaw::BlockPartial));
    const size_t off_hacc = off; off = align256(off + (size_t)4 * bins * sizeof(unsigned long long));
    const bool need_lw = reduce && !o.log_w, need_r2 = reduce && !o.r2, need_rg2 = reduce && !o.rg2,
               need_ng = reduce && !o.n_grown, need_wx = reduce && exact && !o.w_exact,
               need_nn = reduce && exact && lattice && !o.n2rg2;
    const size_t off_lw = off; if (need_lw) off = align256(off + M * sizeof(double));
    const size_t off_r2 = off; if (need_r2) off = align256(off + M * sizeof(double));
    const size_t off_rg2 = off; if (need_rg2) off = align256(off + M * sizeof(double));
    const size_t off_ng = off; if (need_ng) off = align256(off + M * sizeof(uint16_t));
    const size_t off_wx = off; if (need_wx) off = align256(off + M * sizeof(uint64_t));
    const size_t off_nn = off; if (need_nn) off = align256(off + M * sizeof(int64_t));

    void *wsv = nullptr;
    st = workspace(dev, s, off, &wsv);
    if (st != RSAW_OK) return st;
    char *ws = (char *)wsv;
    if (need_lw) o.log_w = (double *)(ws + off_lw);
    if (need_r2) o.r2 = (double *)(ws + off_r2);
    if (need_rg2) o.rg2 = (double *)(ws + off_rg2);
    if (need_ng) o.n_grown = (uint16_t *)(ws + off_ng);
    if (need_wx) o.w_exact = (uint64_t *)(ws + off_wx);
    if (need_nn) o.n2rg2 = (int64_t *)(ws + off_nn);
    if (!lattice) o.n2rg2 = nullptr;
    if (!exact) o.w_exact = nullptr;

    unsigned long long *lmax = (unsigned long long *)(ws + off_lmax);
    int32_t *status = (int32_t *)(ws + off_status);

    unsigned long long *hacc = (unsigned long long *)(ws + off_hacc);
    e = rsaw::launch_reduce_init(lmax, status, hacc, 4 * bins, s);
    if (e != hipSuccess) return hip_fail(e, "reduce_init launch");

    if (M > 0) {
        rsaw::GrowArgs a;
        std::memset(&a, 0, sizeof(a));
        a.seed = cfg->seed;
        a.chain_offset = cfg->chain_offset;
        a.n_chains = M;
        a.n_monomers = cfg->n_monomers;
        a.k_trials = cfg->k_trials;
        a.bond_length = cfg->bond_length;
        a.sigma2 = cfg->bead_diameter * cfg->bead_diameter;
        {
            const double bs = cfg->bond_length + cfg->bead_diameter;
            a.cull2 = bs * bs * (1.0 + 0x1p-30);
        }
        a.log_w = o.log_w;
        a.w_exact = o.w_exact;
        a.r_end = o.r_end;
        a.r2 = o.r2;
        a.rg2 = o.rg2;
        a.n2rg2 = o.n2rg2;
        a.n_grown = o.n_grown;
        a.log_w_max_bits = lmax;
        a.status = status;
        std::memcpy(a.logm, logm_table(), sizeof(a.logm));
        EventPair tp;
        bool timed = false;
        st = timing_start(s, &tp, &timed);
        if (st != RSAW_OK) return st;
        e = lattice ? rsaw::launch_grow_lattice(a, exact, cfg->coord_type == RSAW_I16, s)
                    : rsaw::launch_grow_real(a, s);
        if (timed) {
            st = timing_stop(s, tp);
            if (st != RSAW_OK) return st;
        }
        if (e != hipSuccess) return hip_fail(e, "grow kernel launch");
    }

    if (reduce) {
        rsaw::ReduceArgs r;
        std::memset(&r, 0, sizeof(r));
        r.n_chains = M;
        r.chunk = chunk;
        r.n_monomers = cfg->n_monomers;
        r.bins = bins;
        r.exact = exact ? 1 : 0;
        r.log_w = o.log_w;
        r.r2 = o.r2;
        r.rg2 = o.rg2;
        r.n_grown = o.n_grown;
        r.w_exact = o.w_exact;
        r.n2rg2 = o.n2rg2;
        r.lmax_bits = lmax;
        r.status = status;
        r.partials = (rsaw::BlockPartial *)(ws + off_part);
        r.hist_acc = hacc;
        rsaw_summary *dsum = d_summary ? d_summary : (rsaw_summary *)(ws + off_summary);
        e = rsaw::launch_reduce(r, n_blocks, dsum, d_hist_w, d_hist_n, s);
        if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
        if (used_summary) *used_summary = dsum;
    }
    return RSAW_OK;
}

} // namespace

extern "C" {

rsaw_status rsaw_gen_chains(const rsaw_config *cfg, const rsaw_chain_out *out,
                            rsaw_summary *d_summary, double *d_hist_w, uint64_t *d_hist_n,
                            void *stream)
{
    return gen_impl(cfg, out, d_summary, d_hist_w, d_hist_n, stream, false, nullptr);
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
        if (kv.second.base) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(kv.first.first);
            (void)hipDeviceSynchronize();
            (void)hipFree(kv.second.base);
            (void)hipSetDevice(cur);
        }
    }
    g_ws.clear();
}

} // extern "C"
