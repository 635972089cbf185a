// mgp_prefix.h -- the prefix-sum resamplers (multinomial, Algorithm 7;
// systematic, Algorithm 8) as the single-filter entry point and the SIR
// filter enqueue them: one job of R equal-size runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mgp.h"

namespace mgp {

constexpr int kMaxLevels = 8;  // levels of the 16-ary search tree: 16^8 = 2^32 > any n

// One resample of R equal-size filters (runs) at once, run r = blockIdx.y:
// a single filter is R = 1. Every run has its own scan region of the same
// layout (byte offsets below) at region + r region_ld.
struct PrefixJob {
    const float* w;           // run r's weights: w + r w_ld
    uint64_t w_ld;
    const mgp_stats* stats;   // run r's validation and max: stats[r]
    char* region;
    uint64_t region_ld;
    int32_t* anc;             // run r's ancestors: anc + r anc_ld (null: none)
    uint64_t anc_ld;
    const float* states;      // the particle copy x_bar_i = x_{a_i} of run r: rows of
    float* out;               // d floats at states / out + r rows_ld (states null: none)
    uint64_t rows_ld;
    uint32_t d, vec4;
    uint32_t n, nch;
    int log2n;                // ceil(log2 n)
    uint32_t vec;             // the weights of every run 16-byte aligned
    uint32_t key0, key1;
    uint32_t stream0;         // run r draws from stream stream0 + r
    uint64_t o_hdr, o_sum, o_excl, o_bracket, o_incl;
    uint64_t o_level[kMaxLevels + 1];  // level k (1..top) of the tree
    uint32_t count[kMaxLevels + 1];    // its real entries (the last is S), padded with S to a multiple of kFan
    int top;                           // 0 when n <= kFan (level 0 alone)
};

// Fills the region layout and n, nch, log2n of J for runs of n particles;
// returns the bytes of one run's region.
uint64_t prefix_region(uint32_t n, PrefixJob* J);

// Enqueues the scan and search of a job whose stats (validation, max) are
// already on the device: R runs, method MGP_MULTINOMIAL or MGP_SYSTEMATIC.
int enqueue_prefix(const PrefixJob& J, uint32_t R, int method, hipStream_t s);

}  // namespace mgp
