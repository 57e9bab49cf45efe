// Argument block and per-block partial of the ensemble reduction kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsaw.h"

namespace rsaw {

constexpr int kNumSums = 8; // S0, S2, wR2, w2R2, w2R2^2, wRg2, w2Rg2, w2Rg2^2
constexpr int kMaxBins = 256;

struct BlockPartial {
    double s[kNumSums];
    uint64_t alive, steps;
    uint64_t ex[6]; // three 128-bit exact sums as (lo, hi)
};

struct ReduceArgs {
    uint64_t n_chains;
    uint64_t chunk; // chains per block, a multiple of 256
    int32_t n_monomers;
    int32_t bins;
    int32_t exact;
    const double *log_w;
    const double *r2;
    const double *rg2;
    const uint16_t *n_grown;
    const uint64_t *w_exact;
    const int64_t *n2rg2;
    const unsigned long long *lmax_bits;
    const int32_t *status;
    BlockPartial *partials;
    unsigned long long *hist_acc; // [4][bins]: limbs 0, 1, 2 of sum w, and counts
};

// One ensemble of a batched reduction.
struct ReduceEntry {
    ReduceArgs r;
    uint32_t n_blocks;           // reduce blocks of this ensemble
    unsigned long long *lmax;    // the cells that r reads, writable for the init
    int32_t *status;
    rsaw_summary *out;
    double *hist_w;
    uint64_t *hist_n;
};

// Batched reduction: with init_only, zero every ensemble's accumulators
// (one block each); otherwise the partials over the concatenated block
// ranges (block0 ascending) and one final block per ensemble.
hipError_t launch_reduce_batch(const ReduceEntry *tab, const uint64_t *block0, int n, uint64_t total_blocks,
                               int max_bins, hipStream_t s, bool init_only);

// Serving-loop admission: device workspace of one ensemble in a batch (its
// regions and table entries), the fixed bytes a batch adds, the staging
// bytes of a batch of n, and an early reservation of a stream's staging.
size_t batch_entry_bytes(const rsaw_config *cfg);
constexpr size_t kBatchFixedBytes = 2048;
size_t batch_stage_bytes(int n);
rsaw_status reserve_staging(hipStream_t s, size_t bytes);
rsaw_status release_stream(hipStream_t s);

hipError_t launch_reduce_init(unsigned long long *lmax_bits, int32_t *status,
                              unsigned long long *hist_acc, int n_acc, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs &a, uint32_t n_blocks, rsaw_summary *out,
                         double *hist_w, uint64_t *hist_n, hipStream_t s);

} // namespace rsaw
