// mgp_batch_internal.h -- device-side records and host helpers of the
// batched kernels, shared by the batch plan and the serving executor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mgp.h"
#include "mgp_device.h"
#include "mgp_internal.h"

namespace mgp {

constexpr uint32_t kNoFilter = 0xFFFFFFFFu;
constexpr uint32_t kBatchMaxN = kMirrorMaxN;
constexpr int kMaxXcd = 8;

// Per-filter record in device memory (read with scalar loads).
struct FilterDev {
    const float* w;
    int32_t* anc;
    const float* states;
    float* out;
    mgp_stats* stats_user;
    float* mirror;       // Megopolis: 2n + kMirrorPad floats, else null
    uint32_t* offsets;   // Megopolis: b_max entries, else null
    double eps;
    uint32_t n;
    uint32_t B_user;
    uint32_t b_max;
    uint32_t key0, key1;
    uint32_t stream_id;
    uint32_t part_base;  // first partial of this filter
    uint32_t nparts;
    uint32_t chunk;
    uint32_t n_w, n_part;
    uint32_t vec;        // the reduction may use float4 loads
    uint32_t rows4;      // the gather may use float4 rows
    uint32_t pad[3];
};

struct RTile {
    uint32_t f, c;
};

struct LTile {
    uint32_t f, start;
};

struct LoopShape {
    int bt, ppt, sched;
};

// Tile table of the accept loop for one launch shape (host side): filters
// placed on `nxcd` XCDs by longest-processing-time first on cost[f], tiles of
// the costlier filters first inside each XCD. Schedule 1 interleaves the XCD
// lists so that block b runs on XCD b mod nxcd (empty slots are kNoFilter);
// schedule 2 concatenates them and fills qoff[0..nxcd].
void build_tile_table(const std::vector<uint32_t>& n, const std::vector<double>& cost, const LoopShape& sh, int nxcd,
                      std::vector<LTile>& table, uint32_t* qoff);

// Enqueues one batched run: the segmented reduction, one finalize block per
// filter, and the accept loop with the fused gather. With n_rt == 0 the
// reduction is skipped: the producer of the weights has already written
// every filter's partials (and, for Megopolis, its mirror).
int enqueue_batch(int variant, const LoopShape& sh, const FilterDev* d_fd, uint32_t count, const RTile* d_rt,
                  uint32_t n_rt, Partial* d_parts, mgp_stats* d_stats, const LTile* d_lt, uint32_t grid,
                  const uint32_t* d_qoff, uint32_t* d_qcount, uint32_t nxcd, uint32_t d, hipStream_t s);

// The finalize step alone (one block per filter: the stats record, B, and
// for Megopolis the offsets) over partials already written.
int enqueue_batch_finalize(const FilterDev* d_fd, uint32_t count, Partial* d_parts, mgp_stats* d_stats,
                           uint32_t* d_qcount, hipStream_t s);

bool batch_shape_supported(int variant, const LoopShape& sh);

}  // namespace mgp
