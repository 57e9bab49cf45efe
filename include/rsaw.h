/*
 * rsaw.h — C ABI of librsaw.so: Rosenbluth chain growth on AMD Instinct
 * MI355X (gfx950).
 *
 * The library grows many independent chains at once, each one monomer per
 * step (Guo & Baulin, Comput. Phys. Commun. 2017):
 *   - on the simple cubic lattice (Sec. 3.3.2, Algorithm 1): the 6
 *     neighbours of the tip are the candidates;
 *   - in continuous space as hard spheres (Sec. 3.3.3, Algorithm 2): k random
 *     directions at bond length b are the candidates, and a candidate closer
 *     than sigma to an earlier, non-bonded bead is blocked.
 * At step i the chain counts the free candidates m_i, picks one uniformly and
 * multiplies its Rosenbluth weight W by m_i (Eq. 3).  A dead end (m_i = 0)
 * leaves the chain at weight zero.  The ensemble is then reduced to weighted
 * averages (Eq. 2) and to the mean weight, the estimate of the number of
 * self-avoiding walks (Eq. 6).
 *
 * Random numbers come from Philox4x32-10 keyed by the seed, with counter
 * (chain, step, slot, attempt); chain index g = chain_offset + c, so results
 * do not depend on how a range of chains is split across calls or devices.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* / device arrays are device memory owned by the
 *     caller; the library never frees them.  Host structs are read or written
 *     before the call returns.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *     in stream order; entry points return once the work is enqueued, except
 *     where stated.
 *   - Errors are returned as rsaw_status; no exception crosses the ABI.  A
 *     human-readable message for the last failure on the calling thread is
 *     available from rsaw_last_error().
 *   - Thread safety: calls on different streams may run concurrently; the
 *     library keeps one workspace per (device, stream) (internal, or the
 *     caller's after rsaw_set_workspace), so calls on the same stream are
 *     ordered by that stream.  Calls on one stream must come from one host
 *     thread at a time (they share that workspace and its staging buffer).
 */
#ifndef RSAW_H
#define RSAW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSAW_OK = 0,
    RSAW_E_INVALID = 1,     /* bad argument (see rsaw_last_error)                 */
    RSAW_E_UNSUPPORTED = 2, /* valid request the library has no kernel for       */
    RSAW_E_OVERFLOW = 3,    /* exact 64-bit weight requested beyond its N limit   */
    RSAW_E_NOMEM = 4,       /* device allocation of the workspace failed          */
    RSAW_E_DEVICE = 5,      /* a HIP runtime call failed                          */
    RSAW_E_RNG = 6          /* a rejection loop reached its 65536-attempt cap     */
} rsaw_status;

/* geometry */
#define RSAW_LATTICE_SC 0 /* simple cubic lattice, k = 6 (Sec. 3.3.2)          */
#define RSAW_REAL_HS 1    /* hard spheres in continuous space (Sec. 3.3.3)    */
/* 26-neighbour lattice (the z = 26 lattice space of Sec. 3.3.2), k = 26: the
 * candidates of a step are the 26 sites within Chebyshev distance 1 of the
 * tip, in the order of the code (dx + 1) + 3 (dy + 1) + 9 (dz + 1). */
#define RSAW_LATTICE_26 2

/* element type of the r_end output planes */
#define RSAW_I16 0 /* lattice only */
#define RSAW_I32 1 /* lattice only */
#define RSAW_F64 2 /* real space only */

/* flags */
#define RSAW_EXACT_W 1u /* lattice: also keep W exactly as uint64 (N <= 28; N <= 14 for k = 26) */
/*
 * RSAW_RESTART: a dead end discards the chain and grows it again from the
 * origin (the rule of Sec. 3.3.2 and 3.3.3), up to 65536 attempts; attempt
 * r draws its random numbers with r in the high 16 bits of the step word of
 * the Philox counter (attempt 0 is the stream used without the flag).  The
 * outputs are those of the first complete attempt (a chain that fails every
 * attempt is dead, as without the flag).  The mean weight then estimates
 * c_n / P(complete) rather than c_n.
 */
#define RSAW_RESTART 2u

typedef struct {
    int32_t geometry;      /* RSAW_LATTICE_SC, RSAW_REAL_HS or RSAW_LATTICE_26        */
    int32_t n_monomers;    /* N >= 1 monomers per chain (N - 1 growth steps)         */
    int32_t k_trials;      /* candidates per step: 6 or 26 (lattices), 1..64 (real)   */
    int32_t coord_type;    /* RSAW_I16 / RSAW_I32 (lattice) or RSAW_F64 (real space)  */
    uint64_t n_chains;     /* M >= 0 chains                                          */
    uint64_t seed;         /* Philox key                                             */
    uint64_t chain_offset; /* global index of the first chain (sharding / resume)    */
    double bond_length;    /* b > 0 (real space; the lattice constant is 1)          */
    double bead_diameter;  /* sigma >= 0 (real space; 0 = ideal chain)               */
    int32_t hist_bins;     /* B >= 0 bins of the R^2 histogram over [0, (N-1)^2]     */
    uint32_t flags;        /* RSAW_EXACT_W | RSAW_RESTART                            */
} rsaw_config;

/*
 * Per-chain outputs, structure of arrays, n_chains entries each, device
 * memory.  Any pointer may be NULL ("do not write").  Chain c of the call is
 * element c.  A dead chain has log_w = -INFINITY, w_exact = 0, n_grown =
 * monomers placed, and the observables of its placed prefix.
 */
typedef struct {
    double *log_w;     /* log W (Eq. 3) grouped by value: sum over m = 1..k, ascending */
                       /* m, of n_m ln m, n_m = steps with m free candidates; each     */
                       /* product and each sum rounded once in binary64, ln m          */
                       /* correctly rounded                                            */
    uint64_t *w_exact; /* lattice with RSAW_EXACT_W: prod_i m_i                       */
    void *r_end;       /* 3 planes (x, y, z) of n_chains, coord_type; r_0 = origin    */
    double *r2;        /* squared end-to-end distance                                */
    double *rg2;       /* squared radius of gyration (1/g) sum |r_i - r_cm|^2         */
    int64_t *n2rg2;    /* lattice: g^2 Rg^2 = g sum |r|^2 - |sum r|^2, exact          */
    uint16_t *n_grown; /* monomers placed, g (N for a complete chain)                 */
} rsaw_chain_out;

/*
 * Ensemble summary (Eq. 2 and Eq. 6), written to device memory by
 * rsaw_gen_chains.  w = exp(log W - log_w_max) for live chains.
 */
typedef struct {
    uint64_t n_chains;     /* M, dead chains included                                */
    uint64_t n_alive;      /* chains that reached N monomers                         */
    double log_w_max;      /* L = max log W over live chains (-inf if none)          */
    double sum_w;          /* S0 = sum w                                             */
    double sum_w2;         /* S2 = sum w^2                                           */
    double sum_w_r2;       /* sum w R^2                                              */
    double sum_w2_r2;      /* sum w^2 R^2                                            */
    double sum_w2_r2sq;    /* sum w^2 R^4                                            */
    double sum_w_rg2;      /* sum w Rg^2                                             */
    double sum_w2_rg2;     /* sum w^2 Rg^2                                           */
    double sum_w2_rg2sq;   /* sum w^2 Rg^4                                           */
    double log_c_est;      /* L + log(S0 / M): log of the mean weight (Eq. 6)        */
    double c_rel_err;      /* sqrt((M S2 / S0^2 - 1) / (M - 1))                      */
    double r2_mean;        /* <R^2> = sum w R^2 / S0 (Eq. 2)                          */
    double r2_err;         /* sqrt(sum w^2 (R^2 - <R^2>)^2) / S0                      */
    double rg2_mean;       /* <Rg^2>                                                 */
    double rg2_err;        /* its standard error                                     */
    double ess;            /* S0^2 / S2                                              */
    double steps;          /* growth steps executed, sum (n_grown - 1)               */
    uint64_t sum_w_exact[2];       /* lattice + RSAW_EXACT_W: sum W, 128 bit (lo, hi) */
    uint64_t sum_w_r2_exact[2];    /* sum W R^2                                       */
    uint64_t sum_w_n2rg2_exact[2]; /* sum W g^2 Rg^2                                  */
    int32_t exact_valid;           /* 1 when the three exact sums are filled          */
    int32_t status;                /* device-side status (RSAW_OK or RSAW_E_RNG)      */
} rsaw_summary;

/*
 * rsaw_gen_chains — grow cfg->n_chains chains and reduce them.
 *
 *   cfg        host pointer; validated before anything is enqueued.
 *   out        host pointer to per-chain device arrays (may be NULL; NULL
 *              members are not written).  The reduction reads log_w, r2,
 *              rg2 and n_grown: when the caller does not supply them the
 *              library uses its own device workspace.
 *   d_summary  device pointer to one rsaw_summary, or NULL to skip the
 *              reduction entirely (growth only).
 *   d_hist_w   device array of cfg->hist_bins doubles (W-weighted histogram
 *              of R^2, w as in the summary), or NULL.
 *   d_hist_n   device array of cfg->hist_bins uint64 (live-chain counts), or
 *              NULL.  Bin of a chain: floor((R^2 B) / ((N-1)^2 + 1)),
 *              clamped to B - 1 (the last bin also holds the R^2 above
 *              (N-1)^2 that diagonal steps or b > 1 can reach).
 *   stream     hipStream_t or NULL.
 *
 * Asynchronous: returns after enqueueing.  The results are deterministic:
 * the same config gives bit-identical outputs run to run.
 * Errors: RSAW_E_INVALID for N < 1, N > 65535, unknown geometry or
 * coord_type, lattice k != 6 (26 for RSAW_LATTICE_26), real-space k outside
 * 1..64, b <= 0,
 * sigma < 0, hist_bins < 0, n_chains >= 2^32 (split larger ensembles
 * over calls with chain_offset);
 * RSAW_E_UNSUPPORTED for N > 16384 in any geometry (no kernel in this
 * build); RSAW_E_OVERFLOW for RSAW_EXACT_W with N > 28 (N > 14 on the
 * 26-neighbour lattice);
 * RSAW_E_NOMEM / RSAW_E_DEVICE for runtime failures.  A Marsaglia or Lemire
 * rejection loop that reaches its cap (probability below 2^-100000) sets
 * d_summary->status = RSAW_E_RNG.
 */
rsaw_status rsaw_gen_chains(const rsaw_config *cfg, const rsaw_chain_out *out,
                            rsaw_summary *d_summary, double *d_hist_w,
                            uint64_t *d_hist_n, void *stream);

/*
 * rsaw_gen_chains_sync — rsaw_gen_chains followed by a copy of the summary
 * to host memory `h_summary` (required) and a synchronisation of `stream`.
 */
rsaw_status rsaw_gen_chains_sync(const rsaw_config *cfg, const rsaw_chain_out *out,
                                 rsaw_summary *h_summary, double *d_hist_w,
                                 uint64_t *d_hist_n, void *stream);

/*
 * rsaw_gen_chains_static — rsaw_gen_chains for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and errors as
 * rsaw_gen_chains; the workspace is a file-scope device array of
 * RSAW_STATIC_SCRATCH_BYTES in the library, one copy per GPU, held until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and records no kernel-timing events.
 *
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (the call clears what must start at zero with a kernel): calls
 * that may overlap on one GPU (other streams, other threads, another call
 * before the previous one has finished reading its results from the
 * workspace) race and must be serialised by the caller.  Results the caller
 * needs must be in `out`, `d_summary` and the histograms, which the caller
 * owns.
 * Errors: as rsaw_gen_chains; RSAW_E_NOMEM when the call needs more
 * workspace than the array holds (rsaw_workspace_size > the limit: e.g.
 * more than about 1.2 million chains without per-chain outputs, or
 * hard-sphere chains beyond 1536 beads, whose HBM bead planes need 48 N KiB
 * per resident block), checked before anything is enqueued;
 * RSAW_E_UNSUPPORTED for a device index above 63.
 */
#define RSAW_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
rsaw_status rsaw_gen_chains_static(const rsaw_config *cfg, const rsaw_chain_out *out,
                                   rsaw_summary *d_summary, double *d_hist_w,
                                   uint64_t *d_hist_n, void *stream);

/*
 * rsaw_gen_batch — grow and reduce n ensembles at once (the same method as
 * rsaw_gen_chains, Sec. 3.3.2-3.3.3, Eqs. 2, 3 and 6, for each ensemble).
 *
 *   cfgs         host array of n configurations, each validated as for
 *                rsaw_gen_chains before anything is enqueued; any geometry,
 *                N, k and size may be mixed.
 *   outs         host array of n rsaw_chain_out (device arrays; NULL
 *                members are not written), or NULL for none.
 *   d_summaries  device array of n rsaw_summary, or NULL to skip every
 *                reduction.
 *   d_hist_w,    host arrays of n device pointers (each as the d_hist_w /
 *   d_hist_n     d_hist_n of rsaw_gen_chains, may be NULL), or NULL.
 *   stream       hipStream_t or NULL.
 *
 * Every ensemble's per-chain outputs and summary are bit-identical to those
 * of a separate rsaw_gen_chains call with the same configuration.  The
 * ensembles share launches: one growth launch per kernel variant (geometry,
 * size class and block shape; an ensemble large enough to fill the GPU
 * alone shares only with ensembles whose LDS need allows as many blocks per
 * CU), whose blocks map to (ensemble, chunk) through a prefix table, and
 * three reduction launches for all of them, instead of four launches per
 * ensemble.  The descriptor tables travel in one copy from
 * a pinned host buffer of the library, reused per (device, stream): a call
 * waits for the previous call's table copy on the same stream (not for its
 * kernels).  Asynchronous otherwise.
 * Errors: as rsaw_gen_chains, with the index of the first invalid ensemble
 * in rsaw_last_error(); RSAW_E_INVALID for n < 0 or cfgs NULL with n > 0.
 * n = 0 does nothing.
 */
rsaw_status rsaw_gen_batch(const rsaw_config *cfgs, const rsaw_chain_out *outs, int32_t n,
                           rsaw_summary *d_summaries, double *const *d_hist_w,
                           uint64_t *const *d_hist_n, void *stream);

/*
 * Planned batch — the batch of rsaw_gen_batch prepared once and launched
 * any number of times, with launches that only enqueue kernels, so that a
 * caller can record them into a HIP graph (stream capture) and replay it.
 *
 * rsaw_batch_plan_create validates as rsaw_gen_batch, then, synchronously
 * and on the current device: allocates the plan's own device workspace
 * (the reduction cells and partials, the per-chain arrays the reduction
 * needs where outs gives none, the HBM bead planes of long hard-sphere
 * chains, and the descriptor tables) and copies the tables into it.  Arguments
 * as rsaw_gen_batch; the output pointers (outs, d_summaries, d_hist_w,
 * d_hist_n) are recorded in the plan and must stay valid while it is
 * launched.  *plan receives the handle.  Call it outside any stream capture.
 * Errors: as rsaw_gen_batch; RSAW_E_INVALID for a NULL plan; RSAW_E_NOMEM
 * if the workspace cannot be allocated.
 *
 * rsaw_batch_plan_launch enqueues the batch on `stream` (hipStream_t or
 * NULL): one accumulator-clearing launch, one growth launch per kernel
 * variant and the segmented reduction; no allocation, copy or memset.
 * Every launch gives outputs bit-identical to rsaw_gen_batch with the same
 * arguments.  Launches of one plan share its workspace: at most one may be
 * in flight at a time.  RSAW_E_INVALID for a NULL plan or a current device
 * other than the plan's; RSAW_E_DEVICE for a failed launch.
 *
 * rsaw_batch_plan_destroy frees the plan (its workspace, on its device)
 * once no launch of it is pending; NULL is ignored.
 */
typedef struct rsaw_batch_plan rsaw_batch_plan;

rsaw_status rsaw_batch_plan_create(const rsaw_config *cfgs, const rsaw_chain_out *outs, int32_t n,
                                   rsaw_summary *d_summaries, double *const *d_hist_w,
                                   uint64_t *const *d_hist_n, rsaw_batch_plan **plan);
rsaw_status rsaw_batch_plan_launch(const rsaw_batch_plan *plan, void *stream);
void rsaw_batch_plan_destroy(rsaw_batch_plan *plan);

/*
 * Serving loop.  A server owns S HIP streams on one device and a scheduler
 * thread.  Each stream has a device workspace of bytes_per_stream (capped
 * at creation so that the S of them fit in 90 % of the device's free
 * memory) and a pinned staging buffer for max_batch requests, allocated
 * once when the server is created; serving then allocates nothing.  Each
 * request is one ensemble (an rsaw_config).  The scheduler forms batches
 * from the head of the arrival queue while the requests' workspace bytes
 * (what rsaw_workspace_size reports for the configuration with a reduction
 * and no per-chain outputs, plus its descriptor-table entries, under 1 KiB)
 * fit in a stream's workspace and the batch holds at most max_batch
 * requests.  It launches each batch with rsaw_gen_batch on a free stream,
 * so a new batch starts while others run.  With size classes (large_ms), at most one large request is in
 * flight and a batch holds at most one, while small requests skip past
 * queued large ones; the size estimate is a per-chain cost model (N^2 scan
 * work, per geometry and k) used for scheduling only.  A completion thread
 * per stream retires the batch's tickets.  Each result is bit-identical to
 * a stand-alone rsaw_gen_chains call with the same configuration, whatever
 * the mix it was served in.
 */
typedef struct rsaw_server rsaw_server;

typedef struct {
    uint64_t bytes_per_stream; /* device workspace of one stream, the admission */
                               /* budget of a batch (default 2 GiB)             */
    int32_t max_batch;         /* requests per batch, 1..4096 (default 256)     */
    int32_t streams;           /* concurrent batches, 1..16 (default 2)         */
    double large_ms;           /* size classes: a request whose estimated time  */
                               /* alone exceeds this is large, and large ones   */
                               /* run one at a time, in arrival order, while    */
                               /* small ones skip past them; 0 = 2 ms, < 0 =    */
                               /* no classes (strict arrival order)             */
} rsaw_server_params;

/*
 * rsaw_server_create — start a server on `device` (params NULL = defaults).
 * *out receives the handle.  RSAW_E_INVALID for out-of-range parameters,
 * RSAW_E_DEVICE for a bad device, RSAW_E_NOMEM if its buffers cannot be
 * allocated.
 */
rsaw_status rsaw_server_create(const rsaw_server_params *params, int32_t device, rsaw_server **out);

/*
 * rsaw_server_submit — queue one request; *ticket identifies it.  The
 * configuration is checked as by rsaw_gen_chains (same statuses).  A
 * request whose workspace bytes do not fit in a stream's workspace is
 * refused with RSAW_E_NOMEM.  Thread-safe.
 */
rsaw_status rsaw_server_submit(rsaw_server *s, const rsaw_config *cfg, uint64_t *ticket);

/*
 * rsaw_server_poll — *done = 1 if the request has finished.  Then its
 * summary is written to *h_summary (host, may be NULL) and times_us
 * receives the queueing and completion latencies from submission in
 * microseconds ({started - submitted, finished - submitted}, host array of
 * 2, may be NULL), and the ticket is released.  Returns the request's
 * status once it has finished, RSAW_OK while it runs, RSAW_E_INVALID for an
 * unknown ticket.
 */
rsaw_status rsaw_server_poll(rsaw_server *s, uint64_t ticket, int32_t *done, rsaw_summary *h_summary,
                             double *times_us);

/*
 * rsaw_server_wait — block until the request finishes, then as
 * rsaw_server_poll.  Each ticket is taken (polled to completion or waited
 * for) once, by one thread.
 */
rsaw_status rsaw_server_wait(rsaw_server *s, uint64_t ticket, rsaw_summary *h_summary, double *times_us);

/*
 * rsaw_server_destroy — finish the batches in flight, fail requests that
 * never started (RSAW_E_DEVICE), stop the threads and free the server.
 */
void rsaw_server_destroy(rsaw_server *s);

/* Static description of a status code. */
const char *rsaw_status_string(rsaw_status s);

/* Message describing the last failure on the calling thread ("" if none). */
const char *rsaw_last_error(void);

/* Library version as an integer: major * 10000 + minor * 100 + patch. */
int32_t rsaw_version(void);

/*
 * rsaw_kernel_timing — per-launch timing of the growth kernel, for
 * benchmarking (off by default).  While enabled (enable != 0), every
 * rsaw_gen_chains / rsaw_gen_chains_sync call that grows chains records a
 * HIP event right before and right after its growth-kernel launch, on the
 * call's stream.  Disabling keeps the pairs already recorded.
 * Returns RSAW_OK.
 */
rsaw_status rsaw_kernel_timing(int32_t enable);

/*
 * rsaw_kernel_time — waits for every event pair recorded since the last
 * call, writes their summed elapsed time in milliseconds to *total_ms and
 * their number to *launches (host pointers, either may be NULL), and
 * forgets them.  RSAW_E_DEVICE if a HIP event call fails (the pairs are
 * forgotten all the same).
 */
rsaw_status rsaw_kernel_time(double *total_ms, uint64_t *launches);

/*
 * rsaw_workspace_size — device bytes of library workspace that
 * rsaw_gen_chains(cfg, out, ...) needs on its stream: the reduction cells,
 * block partials and histogram accumulators (Eqs. 2 and 6), the per-chain
 * arrays the reduction reads that `out` does not supply (26 B per chain
 * with no outputs), and the HBM bead planes of hard-sphere chains beyond
 * the LDS limit (3 N doubles per resident block, at most 2048 blocks).
 *
 *   cfg     the configuration (validated as by rsaw_gen_chains).
 *   out     the per-chain outputs the call will pass (NULL = none).
 *   reduce  nonzero when the call reduces (a summary or a histogram).
 *   bytes   receives the size (host).
 *
 * A pure query: no allocation and no device call.  A stream's workspace
 * grows to the largest need seen (at least 1 MiB) and is then reused.
 * Errors: those of rsaw_gen_chains's validation; RSAW_E_INVALID for a NULL
 * `bytes`.
 */
rsaw_status rsaw_workspace_size(const rsaw_config *cfg, const rsaw_chain_out *out, int32_t reduce,
                                size_t *bytes);

/*
 * rsaw_set_workspace — bind a caller-owned device buffer as the workspace of
 * (current device, stream), the buffer that rsaw_workspace_size describes.
 *
 *   d_ws    device memory of the current device, 256-byte aligned, owned by
 *           the caller (the library never frees it); NULL unbinds it, and
 *           the next call on the stream allocates an internal workspace again.
 *   bytes   its size; at least the bytes of an empty reducing call (a few
 *           hundred bytes).
 *   stream  hipStream_t or NULL (the default stream).
 *
 * While bound, rsaw_gen_chains, rsaw_gen_chains_sync and rsaw_gen_batch on
 * `stream` place their workspace in d_ws and allocate no device memory; a
 * call that needs more than `bytes` (rsaw_workspace_size; for a batch, the
 * sum over its ensembles plus its descriptor tables) fails with
 * RSAW_E_NOMEM before enqueueing anything.  A bound stream's calls
 * therefore only enqueue kernel launches (rsaw_gen_batch also copies its
 * tables from a pinned host buffer), so a caller can capture
 * rsaw_gen_chains into a HIP graph with no earlier warm-up call.  The buffer
 * must stay valid, and must not be used by anything else, while work
 * enqueued with it may run.  Binding releases an internal workspace of the
 * stream after waiting for the stream's queued work (call it outside any
 * capture).  Host-side, per (device, stream).
 * Errors: RSAW_E_INVALID for a misaligned pointer, a size below the minimum,
 * or memory that is not device memory of the current device;
 * RSAW_E_DEVICE for a failed HIP call.
 */
rsaw_status rsaw_set_workspace(void *d_ws, size_t bytes, void *stream);

/*
 * rsaw_fp64_check — evaluate binary64 square roots and quotients on the
 * device as the growth kernels do (no contraction, the same target), for
 * checking that they are correctly rounded: the hard-sphere kernels take
 * the square root of 1 - s in the Marsaglia step (Sec. 3.3.3,
 * q = 2 sqrt(1 - s)) with their own routine for arguments in [2^-60, 1],
 * and divide in the centre of mass and Rg^2.
 *
 *   d_a, d_b        device arrays of n doubles (inputs).
 *   d_sqrt, d_div   device arrays of n doubles: sqrt(a_i) (the kernels'
 *                   routine for a_i in [2^-60, 1], the general device square
 *                   root elsewhere) and a_i / b_i.
 *   n               element count (0 does nothing).
 *   stream          hipStream_t or NULL.  Asynchronous.
 * Errors: RSAW_E_INVALID for a NULL array with n > 0; RSAW_E_DEVICE for a
 * failed launch.
 */
rsaw_status rsaw_fp64_check(const double *d_a, const double *d_b, double *d_sqrt, double *d_div, uint64_t n,
                            void *stream);

/*
 * Lane mapping of the group kernels and its autotuner.
 *
 * Three growth kernels spread one chain over a group of lanes: the
 * six-neighbour lattice for N > 64 (Sec. 3.3.2, Algorithm 1), hard spheres
 * up to N = 1536 (Sec. 3.3.3, Algorithm 2) and the 26-neighbour lattice for
 * N > 64.  Their mapping has two knobs: lanes per chain (2..64, a power of
 * two; 64 / lanes chains share a wavefront, and the lanes split the scan of
 * the chain's earlier monomers) and threads per block (64 or 256, which
 * sets how many chains share a block's LDS and its tables).  A built-in
 * rule picks both from N and k.  A process-wide tuning table can replace
 * the rule per (geometry, k, range of N); it applies to rsaw_gen_chains,
 * rsaw_gen_batch and the server alike.
 *
 * The mapping never changes a result: every legal mapping gives per-chain
 * outputs and summaries bit-identical to the built-in rule's, because the
 * random numbers are keyed by (seed, chain, step, slot), and the candidate
 * tests and the reduction order do not depend on how the lanes split a
 * chain's scan.
 *
 * Legal mappings:
 *   RSAW_LATTICE_SC  lanes 2 (N <= 128 only), 4 (N <= 2048 only), 8, 16,
 *                    32, 64; one 4-byte word per monomer (see
 *                    rsaw_set_byte_box) in the chain's lanes' registers
 *                    where 128 < N <= 64 lanes, and with 2 lanes, else up
 *                    to N = 2048 in LDS where the block can also hold one
 *                    chain's regrowth (all but 64 lanes in 64-thread
 *                    blocks beyond N = 768), else two words in LDS;
 *   RSAW_REAL_HS     lanes 8, 16, 32, 64 with lanes >= k; lanes 64 only
 *                    with 64 threads; N <= 1536;
 *   RSAW_LATTICE_26  lanes 2 (N <= 128 only), 4 (N <= 256 only), 8, 16,
 *                    32, 64; up to N = 4096 one word per monomer, held in
 *                    the chain's lanes' registers for N <= 64 lanes, else
 *                    in LDS where the block can also hold one chain's
 *                    regrowth, else two words in LDS;
 * threads 64 or 256; and the block's LDS (lds_bytes) at most 160 KiB.
 * Calls outside the group kernels' ranges (lattice N <= 64 or exact
 * weights, hard spheres N > 1536) never consult the table.
 */
typedef struct {
    int32_t geometry;   /* RSAW_LATTICE_SC, RSAW_REAL_HS or RSAW_LATTICE_26      */
    int32_t k_trials;   /* k of the calls the entry applies to (6 or 26 on the    */
                        /* lattices)                                              */
    int32_t n_lo, n_hi; /* chain lengths N (monomers) covered, inclusive          */
    int32_t lanes;      /* lanes per chain                                        */
    int32_t threads;    /* threads per block                                      */
    uint64_t lds_bytes; /* dynamic LDS per block; written by the library only     */
} rsaw_mapping;

/*
 * rsaw_mapping_set — add an entry to the tuning table (host-only, no device
 * call).  `m` is a host pointer; lds_bytes is ignored.  The entry must be
 * legal at n_hi (then it is at every smaller N of its range, since the LDS
 * need and the format limits grow with N).  A later entry takes precedence
 * over earlier ones where their ranges overlap.  Thread-safe; calls already
 * enqueued keep the mapping they were launched with.
 * Errors: RSAW_E_INVALID for a NULL `m`, an unknown geometry, k out of
 * range, n_lo < 1, n_hi < n_lo, or a mapping that is not legal at n_hi.
 */
rsaw_status rsaw_mapping_set(const rsaw_mapping *m);

/*
 * rsaw_set_byte_box — tuning and testing knob of the lattice kernels that
 * keep one 32-bit word per monomer (Sec. 3.3.2 growth; simple cubic lattice
 * beyond N = 128 in byte words, 26-neighbour group kernel in byte words up
 * to N = 640 and packed 11/11/10-bit words up to N = 4096): a chain whose
 * tip reaches |x|, |y| or |z| = edge is dropped from that kernel and grown
 * again, from its first draw, in two-word format by the same block.  Each
 * format has its own largest exact edge (127, 62 and 254); edge = 0 (the
 * default) uses those, 1..127 lowers every edge to at most that value,
 * which only sends more chains through the regrowth.  Results never depend
 * on it: every chain is bit-identical either way.  Process-wide; applies
 * to calls enqueued after it.  Host-only.
 * Errors: RSAW_E_INVALID unless 0 <= edge <= 127.
 */
rsaw_status rsaw_set_byte_box(int32_t edge);

/* rsaw_mapping_clear — empty the tuning table (the built-in rule applies
 * again to every later call).  Thread-safe. */
void rsaw_mapping_clear(void);

/*
 * rsaw_mapping_list — copy the tuning table, oldest entry first, into the
 * host array `out` of `capacity` entries (out may be NULL when capacity is
 * 0); *count (host, required) receives the number of entries in the table,
 * which may exceed capacity (then only the first `capacity` are copied).
 * Re-adding the listed entries in order with rsaw_mapping_set rebuilds the
 * same table, e.g. from a saved autotune cache.  Host-only, thread-safe.
 * Errors: RSAW_E_INVALID for a NULL count, capacity < 0, or a NULL out with
 * capacity > 0.
 */
rsaw_status rsaw_mapping_list(rsaw_mapping *out, int32_t capacity, int32_t *count);

/*
 * rsaw_mapping_query — the mapping a rsaw_gen_chains call with `cfg` would
 * launch its growth kernel with, written to the host struct *m (n_lo =
 * n_hi = cfg->n_monomers).  Host-only, no device call.  Kernels without a
 * group mapping report lanes = 1 (one lane per chain: lattice N <= 64, exact
 * weights) or lanes = 64 with lds_bytes = 0 (hard spheres beyond N = 1536,
 * bead planes in HBM).
 * Errors: those of rsaw_gen_chains's validation; RSAW_E_INVALID for a NULL m.
 */
rsaw_status rsaw_mapping_query(const rsaw_config *cfg, rsaw_mapping *m);

/*
 * rsaw_autotune — measure every legal mapping on the device and install the
 * fastest per range of N when it beats the mapping in force (the built-in
 * rule or an earlier entry) by at least 3 %; otherwise the mapping in force
 * stays and nothing is installed for that range.
 *
 *   base       the workload of a probe: geometry, k, n_chains, seed, b, sigma
 *              and flags are taken from it (n_monomers is ignored).
 *   n_edges    host array of n_buckets chain lengths, strictly increasing.
 *              Bucket b covers N in [n_edges[b-1] + 1, n_edges[b]] (from
 *              N = 1 for b = 0) and is probed at N = n_edges[b], its largest
 *              (and most LDS-hungry) member.
 *   n_buckets  1..64.
 *   reps       timed calls per candidate (1..100), after one untimed call.
 *   chosen     host array of n_buckets, or NULL: the mapping each bucket
 *              runs with afterwards (the winner, or the mapping in force; the
 *              built-in one, unchanged, where N has no group kernel).
 *   best_ms    host array of n_buckets, or NULL: the winner's mean time per
 *              call (growth and reduction, HIP events on `stream`).
 *   stream     hipStream_t or NULL.
 *
 * Each probe is a full rsaw_gen_chains call (growth into the library's
 * workspace and a reduction to its internal summary).  The candidates are
 * timed one after another on `stream`, which this call synchronises; other
 * threads' calls are unaffected while it runs and pick up the installed
 * entries afterwards.  The winners go into the tuning table as by
 * rsaw_mapping_set.
 * Errors: RSAW_E_INVALID for a bad base config (as rsaw_gen_chains), NULL
 * or non-increasing n_edges, n_buckets or reps out of range;
 * RSAW_E_DEVICE / RSAW_E_NOMEM for runtime failures (entries of buckets
 * already tuned stay installed).
 */
rsaw_status rsaw_autotune(const rsaw_config *base, const int32_t *n_edges, int32_t n_buckets,
                          int32_t reps, rsaw_mapping *chosen, double *best_ms, void *stream);

/* Release the internal device workspace of every device and the timing
 * events (safe to call repeatedly; later calls re-create them on demand). */
void rsaw_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* RSAW_H */
