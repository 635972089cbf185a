// mgp_internal.h -- host/device shared definitions of libmgp (not part of the
// public ABI): workspace layout, launch shapes, and the host helpers the
// single-filter, batched and serving paths share.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mgp.h"
#include "mgp_device.h"

namespace mgp {

constexpr int kVersion = 100;               // 0.1.0
constexpr uint32_t kReduceThreads = 256;    // reduce / finalize block
constexpr uint32_t kLoopThreads = 256;      // accept-loop block (4 waves of 64)
constexpr uint32_t kMaxPartials = 4096;     // reduce blocks per filter, at most
constexpr uint32_t kReduceChunk = 2048;     // weights per reduce block (before the kMaxPartials cap)
constexpr uint32_t kDefaultBMax = 65536;
constexpr uint32_t kBMaxLimit = 1u << 24;

// Workspace layout of a single-filter call (byte offsets, 256-aligned):
//   [stats: mgp_stats][partials: kMaxPartials x Partial][offsets: b_max x u32]
//   [mirror: (2n + kMirrorPad) x f32, Megopolis with n <= kMirrorMaxN only]
constexpr size_t kWsStatsOffset = 0;
constexpr size_t kWsPartialsOffset = 256;
constexpr int kMegopolisPPT = 4;  // particles per thread of the mirrored Megopolis loop

struct Partial {
    double w_sum;
    float w_max;
    uint32_t bad;
};
static_assert(sizeof(Partial) == 16, "Partial is 16 bytes");

constexpr size_t kWsOffsetsOffset = kWsPartialsOffset + (size_t)kMaxPartials * sizeof(Partial);

struct FinalizeArgs {
    double eps;
    uint32_t n;
    uint32_t B_user;
    uint32_t b_max;
    uint32_t make_offsets;
    uint32_t key0, key1;
    uint32_t stream_id;
    uint32_t tag;
};

// Tag tying a workspace's stats and offsets to the call that produced them.
__host__ __device__ inline uint32_t call_tag(uint32_t n, int variant, uint64_t seed, uint32_t stream_id)
{
    uint32_t h = 0x811C9DC5u;
    const uint32_t parts[5] = {n, (uint32_t)variant, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id};
    for (int i = 0; i < 5; ++i) h = (h ^ parts[i]) * 0x01000193u;
    return h | 1u;  // never 0
}

// Validated copy of mgp_params with defaults filled in.
struct Params {
    int variant;
    uint32_t B;
    double eps;
    uint64_t seed;
    uint32_t stream_id;
    uint32_t partition_bytes;
    uint32_t b_max;
    uint32_t segment = 32;  // Megopolis segment width, 32 or 64
};

int fail(int code, const char* fmt, ...);
void clear_error();
int check_launch(const char* what);
int normalize_params(const mgp_params* in, Params* out);
size_t workspace_bytes(uint32_t b_max);
size_t workspace_bytes(uint32_t n, const Params& p);
bool uses_mirror(uint32_t n, int variant);
size_t mirror_offset(uint32_t b_max);
uint32_t reduce_blocks(uint32_t n);
uint32_t reduce_chunk(uint32_t n, uint32_t blocks);
int enqueue_reduce_finalize(const float* w, uint32_t n, const Params& p, bool make_offsets, char* ws,
                            mgp_stats* st_user, hipStream_t stream);
// The accept loop (after the reduction and finalize launches); with rc.states
// set, the particle copy x_bar_i = x_{k_i} runs as its epilogue. anc may be
// null when rc copies the rows.
int enqueue_loop(const float* w, uint32_t n, const Params& p, char* ws, int32_t* anc, hipStream_t stream,
                 const RowCopy& rc = RowCopy{});
// The accept loop for m outputs drawn from n weighted inputs (M != N).
int enqueue_loop_m(const float* w, uint32_t n, uint32_t m, const Params& p, char* ws, int32_t* anc,
                   hipStream_t stream, const RowCopy& rc = RowCopy{});
int enqueue_gather(const float* states, uint32_t n_states, uint32_t d, const int32_t* anc, uint32_t n_out,
                   float* out, hipStream_t stream);
// mgp_resample's work: one launch up to 8192 (Megopolis) or 4096 particles,
// two up to 32768 (Megopolis: the finalize step inside the accept loop),
// leaving nothing in the workspace for a prepared loop; else the reduction +
// finalize and the accept loop.
int enqueue_resample(const float* w, uint32_t n, const Params& p, char* ws, mgp_stats* st_user, int32_t* anc,
                     hipStream_t stream, const RowCopy& rc = RowCopy{});

}  // namespace mgp
