// mgp_batch.hip -- many independent filters in one graph launch (gfx950).
//
// A run is three kernels:
//   1. k_batch_reduce   one block per (filter, chunk): fp32 max, fp64 sum and
//                       validation of the chunk, plus the Megopolis mirror
//                       M[k] = w[k mod n] of the filter;
//   2. k_batch_finalize one block per filter: B from eq. (proposition), the
//                       stats record and the Megopolis offsets;
//   3. the accept loop  over (filter, tile) work items, each tile BT * P
//                       particles of one filter, with the particle gather
//                       fused into its epilogue.
// Every filter computes exactly what mgp_resample (+ mgp_gather) computes
// for it: the schedule changes, the numbers do not.
//
// XCD-aware placement: workgroups are dispatched to the 8 XCDs of an MI355X
// in round-robin order of their index, and each XCD has its own 4 MB L2. The
// plan assigns whole filters to XCDs by longest-processing-time first (cost
// N_f * B_f, with B_f from one reduction at plan time) and orders the tile
// table so that every tile of a filter lands on its XCD: a filter's weights
// (at most 2 MB mirrored for N_f = 2^18) are fetched into one L2 only.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "mgp.h"
#include "mgp_device.h"
#include "mgp_internal.h"
#include "mgp_reduce.h"
#include "mgp_batch_internal.h"

namespace mgp {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_batch_reduce(const FilterDev* __restrict__ fd,
                                                                 const RTile* __restrict__ tiles,
                                                                 Partial* __restrict__ parts)
{
    const RTile t = tiles[blockIdx.x];
    const FilterDev& F = fd[t.f];
    const uint64_t start = (uint64_t)t.c * F.chunk;
    const uint64_t stop = start + F.chunk < (uint64_t)F.n ? start + F.chunk : (uint64_t)F.n;
    const uint64_t end = stop > start ? stop : start;
    float mx = 0.0f;
    double s = 0.0;
    uint32_t bad = 0;
    if (F.vec)
        reduce_range<true>(F.w, F.n, start, end, F.mirror, mx, s, bad);
    else
        reduce_range<false>(F.w, F.n, start, end, F.mirror, mx, s, bad);
    if (F.mirror && t.c == 0) mirror_pad(F.w, F.n, F.mirror);
    block_reduce(mx, s, bad);
    if (threadIdx.x == 0) parts[F.part_base + t.c] = Partial{s, mx, bad};
}

__global__ __launch_bounds__(kReduceThreads) void k_batch_finalize(const FilterDev* __restrict__ fd,
                                                                   const Partial* __restrict__ parts,
                                                                   mgp_stats* __restrict__ stats,
                                                                   uint32_t* __restrict__ queues, uint32_t nq)
{
    const FilterDev& F = fd[blockIdx.x];
    FinalizeArgs a;
    a.eps = F.eps;
    a.n = F.n;
    a.B_user = F.B_user;
    a.b_max = F.b_max;
    a.make_offsets = F.offsets ? 1u : 0u;
    a.key0 = F.key0;
    a.key1 = F.key1;
    a.stream_id = F.stream_id;
    a.tag = 0;
    finalize_one(parts + F.part_base, F.nparts, a, &stats[blockIdx.x], F.stats_user, F.offsets);
    // the persistent schedule's queue counters start at zero on every run
    if (blockIdx.x == 0 && threadIdx.x < nq) queues[threadIdx.x] = 0;
}

// x_bar_i = x_{k_i} for one particle (fused gather epilogue).
__device__ __forceinline__ void gather_row(const FilterDev& F, uint32_t i, int32_t k, uint32_t d)
{
    if (!F.states || d == 0) return;
    // outputs are streamed past the L2 (written once, never read here)
    if (F.rows4) {
        const float4* src = reinterpret_cast<const float4*>(F.states);
        float4* dst = reinterpret_cast<float4*>(F.out);
        const uint32_t d4 = d / 4u;
        for (uint32_t c = 0; c < d4; ++c) {
            const float4 v = k >= 0 ? src[(uint64_t)k * d4 + c] : make_float4(NAN, NAN, NAN, NAN);
            float4* o = &dst[(uint64_t)i * d4 + c];
            __builtin_nontemporal_store(v.x, &o->x);
            __builtin_nontemporal_store(v.y, &o->y);
            __builtin_nontemporal_store(v.z, &o->z);
            __builtin_nontemporal_store(v.w, &o->w);
        }
    } else {
        for (uint32_t c = 0; c < d; ++c)
            __builtin_nontemporal_store(k >= 0 ? F.states[(uint64_t)k * d + c] : NAN, &F.out[(uint64_t)i * d + c]);
    }
}

template <int V, int BT, int P>
__device__ __forceinline__ void process_tile(const FilterDev& F, const mgp_stats* __restrict__ st, uint32_t start,
                                             uint32_t d)
{
    const uint32_t n = F.n;
    const uint32_t B = st->B;
    if (st->status != MGP_OK) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t i = start + threadIdx.x + BT * p;
            if (i < n) {
                F.anc[i] = -1;
                gather_row(F, i, -1, d);
            }
        }
        return;
    }
    if constexpr (V == kMegopolis) {
        const uint32_t i0 = start + threadIdx.x;
        uint32_t k[P];
        megopolis_mirror_chain<P, BT>(reinterpret_cast<const char*>(F.mirror), F.offsets, n, B, F.key0, F.key1,
                                      F.stream_id, i0, k);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t i = i0 + BT * p;
            if (i < n) {
                F.anc[i] = (int32_t)k[p];
                gather_row(F, i, (int32_t)k[p], d);
            }
        }
    } else {
        // every lane runs a chain (lanes past n as n - 1, whose group is that
        // of the real lanes of its half-wave: tiles start on multiples of 64),
        // so that C2 shares each group's partition draws across the half-wave
        const LoopParams L{F.w, F.offsets, n, B, F.key0, F.key1, F.stream_id, F.n_w, F.n_part};
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t i = start + threadIdx.x + BT * p;
            const uint32_t ic = i < n ? i : n - 1u;
            const uint32_t k = run_chain<V, true, true>(L, ic);
            if (i < n) {
                F.anc[i] = (int32_t)k;
                gather_row(F, i, (int32_t)k, d);
            }
        }
    }
}

// Minimum waves per SIMD asked of the compiler for the grid-scheduled
// accept loop. C2's shared partition draws raise its register count to 78
// (6 waves); asked for 7 it schedules the loop into 70 registers without
// spilling: 7% and 13% faster at B = 32 and 64, equal at B = 16. The others,
// and the persistent kernel (whose queue logic adds registers), are left to
// the compiler: asked for 7 they would spill.
template <int V>
struct LoopWaves {
    static constexpr int value = V == kC2 ? 7 : 1;
};

// One block per tile, tiles ordered so that block b runs on XCD b mod 8.
template <int V, int BT, int P>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(LoopWaves<V>::value))) void k_batch_loop_grid(const FilterDev* __restrict__ fd,
                                                        const mgp_stats* __restrict__ stats,
                                                        const LTile* __restrict__ tiles, uint32_t d)
{
    const LTile t = tiles[blockIdx.x];
    if (t.f == kNoFilter) return;
    process_tile<V, BT, P>(fd[t.f], &stats[t.f], t.start, d);
}

// Persistent blocks: block b serves the queue of XCD b mod nq first, then
// steals from the others; it exits once every queue is exhausted (each grab
// advances a counter, so every block reaches the exit). A grab claims a
// chunk of tiles sized to what is left (guided self-scheduling: about
// remaining / (2 * blocks per queue), at least 1), because device-scope
// atomics on one counter serialize across the chip.
template <int V, int BT, int P>
__global__ __launch_bounds__(BT) void k_batch_loop_persistent(const FilterDev* __restrict__ fd,
                                                              const mgp_stats* __restrict__ stats,
                                                              const LTile* __restrict__ tiles,
                                                              const uint32_t* __restrict__ qoff,
                                                              uint32_t* __restrict__ qcount, uint32_t nq, uint32_t d)
{
    __shared__ uint32_t s_first, s_last;
    const uint32_t home = blockIdx.x % nq;
    const uint32_t per_queue = (gridDim.x + nq - 1) / nq;
    uint32_t tried = 0;
    uint32_t seen = 0;  // last counter value this block saw on the current queue
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t first = kNoFilter, last = 0;
            while (tried < nq) {
                const uint32_t q = (home + tried) % nq;
                const uint32_t len = qoff[q + 1] - qoff[q];
                const uint32_t left = len > seen ? len - seen : 0;
                uint32_t chunk = left / (2u * per_queue);
                chunk = chunk < 1u ? 1u : (chunk > 64u ? 64u : chunk);
                const uint32_t idx = atomicAdd(&qcount[q], chunk);
                if (idx < len) {
                    first = qoff[q] + idx;
                    last = qoff[q] + (idx + chunk < len ? idx + chunk : len);
                    seen = idx + chunk;
                    break;
                }
                ++tried;
                seen = 0;
            }
            s_first = first;
            s_last = last;
        }
        __syncthreads();
        const uint32_t first = __builtin_amdgcn_readfirstlane(s_first);
        const uint32_t last = __builtin_amdgcn_readfirstlane(s_last);
        __syncthreads();
        if (first == kNoFilter) break;
        for (uint32_t t = first; t < last; ++t) {
            const LTile tile = tiles[t];
            process_tile<V, BT, P>(fd[tile.f], &stats[tile.f], tile.start, d);
        }
    }
}

// ---------------------------------------------------------------------------
// Launch table
// ---------------------------------------------------------------------------
struct LoopArgs {
    const FilterDev* fd;
    const mgp_stats* stats;
    const LTile* tiles;
    const uint32_t* qoff;
    uint32_t* qcount;
    uint32_t nq;
    uint32_t d;
    uint32_t grid;
};

template <int V, int BT, int P>
static void launch_loop_shape(int sched, const LoopArgs& a, hipStream_t s)
{
    if (sched == 1)
        hipLaunchKernelGGL((k_batch_loop_grid<V, BT, P>), dim3(a.grid), dim3(BT), 0, s, a.fd, a.stats, a.tiles, a.d);
    else
        hipLaunchKernelGGL((k_batch_loop_persistent<V, BT, P>), dim3(a.grid), dim3(BT), 0, s, a.fd, a.stats, a.tiles,
                           a.qoff, a.qcount, a.nq, a.d);
}

template <int V>
static bool launch_loop_variant(const LoopShape& sh, const LoopArgs& a, hipStream_t s)
{
    if constexpr (V == kMegopolis) {
        if (sh.bt == 256 && sh.ppt == 4) return launch_loop_shape<V, 256, 4>(sh.sched, a, s), true;
        if (sh.bt == 256 && sh.ppt == 2) return launch_loop_shape<V, 256, 2>(sh.sched, a, s), true;
        if (sh.bt == 256 && sh.ppt == 1) return launch_loop_shape<V, 256, 1>(sh.sched, a, s), true;
        if (sh.bt == 128 && sh.ppt == 4) return launch_loop_shape<V, 128, 4>(sh.sched, a, s), true;
        if (sh.bt == 128 && sh.ppt == 2) return launch_loop_shape<V, 128, 2>(sh.sched, a, s), true;
        if (sh.bt == 64 && sh.ppt == 4) return launch_loop_shape<V, 64, 4>(sh.sched, a, s), true;
        if (sh.bt == 64 && sh.ppt == 8) return launch_loop_shape<V, 64, 8>(sh.sched, a, s), true;
        if (sh.bt == 128 && sh.ppt == 8) return launch_loop_shape<V, 128, 8>(sh.sched, a, s), true;
        return false;
    } else {
        if (sh.ppt != 1) return false;
        if (sh.bt == 256) return launch_loop_shape<V, 256, 1>(sh.sched, a, s), true;
        if (sh.bt == 128) return launch_loop_shape<V, 128, 1>(sh.sched, a, s), true;
        if (sh.bt == 64) return launch_loop_shape<V, 64, 1>(sh.sched, a, s), true;
        return false;
    }
}

static bool launch_loop(int variant, const LoopShape& sh, const LoopArgs& a, hipStream_t s)
{
    switch (variant) {
    case kMetropolis: return launch_loop_variant<kMetropolis>(sh, a, s);
    case kC1: return launch_loop_variant<kC1>(sh, a, s);
    case kC2: return launch_loop_variant<kC2>(sh, a, s);
    default: return launch_loop_variant<kMegopolis>(sh, a, s);
    }
}

template <int V, int BT, int P>
static int occupancy_of()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_loop_persistent<V, BT, P>, BT, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return blocks;
}

template <int V>
static int occupancy_variant(const LoopShape& sh)
{
    if constexpr (V == kMegopolis) {
        if (sh.bt == 256 && sh.ppt == 4) return occupancy_of<V, 256, 4>();
        if (sh.bt == 256 && sh.ppt == 2) return occupancy_of<V, 256, 2>();
        if (sh.bt == 256 && sh.ppt == 1) return occupancy_of<V, 256, 1>();
        if (sh.bt == 128 && sh.ppt == 4) return occupancy_of<V, 128, 4>();
        if (sh.bt == 128 && sh.ppt == 2) return occupancy_of<V, 128, 2>();
        if (sh.bt == 64 && sh.ppt == 8) return occupancy_of<V, 64, 8>();
        if (sh.bt == 128 && sh.ppt == 8) return occupancy_of<V, 128, 8>();
        return occupancy_of<V, 64, 4>();
    } else {
        if (sh.bt == 256) return occupancy_of<V, 256, 1>();
        if (sh.bt == 128) return occupancy_of<V, 128, 1>();
        return occupancy_of<V, 64, 1>();
    }
}

static int persistent_occupancy(int variant, const LoopShape& sh)
{
    switch (variant) {
    case kMetropolis: return occupancy_variant<kMetropolis>(sh);
    case kC1: return occupancy_variant<kC1>(sh);
    case kC2: return occupancy_variant<kC2>(sh);
    default: return occupancy_variant<kMegopolis>(sh);
    }
}

static std::vector<LoopShape> candidate_shapes(int variant)
{
    std::vector<LoopShape> c;
    for (int sched : {1, 2}) {
        if (variant == kMegopolis) {
            c.push_back({256, 4, sched});
            c.push_back({256, 2, sched});
            c.push_back({256, 1, sched});
            c.push_back({128, 4, sched});
            c.push_back({128, 2, sched});
            c.push_back({64, 4, sched});
            c.push_back({64, 8, sched});
            c.push_back({128, 8, sched});
        } else {
            c.push_back({256, 1, sched});
            c.push_back({128, 1, sched});
            c.push_back({64, 1, sched});
        }
    }
    return c;
}

bool batch_shape_supported(int variant, const LoopShape& sh)
{
    for (const LoopShape& c : candidate_shapes(variant))
        if (c.bt == sh.bt && c.ppt == sh.ppt && c.sched == sh.sched) return true;
    return false;
}

void build_tile_table(const std::vector<uint32_t>& n, const std::vector<double>& cost, const LoopShape& sh, int nx,
                      std::vector<LTile>& table, uint32_t* qoff)
{
    const uint32_t tile = (uint32_t)(sh.bt * sh.ppt);
    const int count = (int)n.size();
    // Work items are chunks of whole tiles: a filter is cut into chunks of
    // about total / (16 nx) particles, so that a few large filters still
    // spread over every XCD while small filters stay whole (one L2 each).
    uint64_t total = 0;
    for (uint32_t x : n) total += x;
    uint64_t chunk = (total + 16ull * nx - 1) / (16ull * nx);
    chunk = std::max<uint64_t>(tile, (chunk + tile - 1) / tile * tile);
    struct Item {
        uint32_t f, start, stop;
        double cost;
    };
    std::vector<Item> items;
    for (int f = 0; f < count; ++f) {
        const double per = cost[f] / std::max<uint32_t>(1u, n[f]);
        for (uint64_t st = 0; st < n[f]; st += chunk) {
            const uint32_t stop = (uint32_t)std::min<uint64_t>(n[f], st + chunk);
            items.push_back(Item{(uint32_t)f, (uint32_t)st, stop, per * (stop - st)});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<double> load(nx, 0.0);
    std::vector<std::vector<Item>> per(nx);
    for (const Item& it : items) {
        int best = 0;
        for (int x = 1; x < nx; ++x)
            if (load[x] < load[best]) best = x;
        load[best] += it.cost;
        per[best].push_back(it);
    }
    std::vector<std::vector<LTile>> lists(nx);
    for (int x = 0; x < nx; ++x) {
        // costlier tiles (larger cost per particle) first inside the XCD
        std::stable_sort(per[x].begin(), per[x].end(), [&](const Item& a, const Item& b) {
            return cost[a.f] / n[a.f] > cost[b.f] / n[b.f];
        });
        for (const Item& it : per[x])
            for (uint32_t st = it.start; st < it.stop; st += tile) lists[x].push_back(LTile{it.f, st});
    }
    table.clear();
    for (int x = 0; x <= kMaxXcd; ++x) qoff[x] = 0;
    if (sh.sched == 1) {
        size_t mx = 0;
        for (auto& l : lists) mx = std::max(mx, l.size());
        table.assign(mx * nx, LTile{kNoFilter, 0});
        for (int x = 0; x < nx; ++x)
            for (size_t m = 0; m < lists[x].size(); ++m) table[m * nx + x] = lists[x][m];
    } else {
        for (int x = 0; x < nx; ++x) {
            qoff[x] = (uint32_t)table.size();
            table.insert(table.end(), lists[x].begin(), lists[x].end());
        }
        qoff[nx] = (uint32_t)table.size();
    }
}

int enqueue_batch_finalize(const FilterDev* d_fd, uint32_t count, Partial* d_parts, mgp_stats* d_stats,
                           uint32_t* d_qcount, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_finalize, dim3(count), dim3(kReduceThreads), 0, s, d_fd, d_parts, d_stats, d_qcount,
                       (uint32_t)kMaxXcd);
    return check_launch("batch finalize");
}

int enqueue_batch(int variant, const LoopShape& sh, const FilterDev* d_fd, uint32_t count, const RTile* d_rt,
                  uint32_t n_rt, Partial* d_parts, mgp_stats* d_stats, const LTile* d_lt, uint32_t grid,
                  const uint32_t* d_qoff, uint32_t* d_qcount, uint32_t nxcd, uint32_t d, hipStream_t s)
{
    int rc;
    if (n_rt > 0) {
        hipLaunchKernelGGL(k_batch_reduce, dim3(n_rt), dim3(kReduceThreads), 0, s, d_fd, d_rt, d_parts);
        rc = check_launch("batch reduce");
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_batch_finalize, dim3(count), dim3(kReduceThreads), 0, s, d_fd, d_parts, d_stats, d_qcount,
                       (uint32_t)kMaxXcd);
    rc = check_launch("batch finalize");
    if (rc) return rc;
    LoopArgs a{d_fd, d_stats, d_lt, d_qoff, d_qcount, nxcd, d, grid};
    if (!launch_loop(variant, sh, a, s)) return fail(MGP_EINVAL, "unsupported launch shape bt=%d ppt=%d", sh.bt, sh.ppt);
    return check_launch("batch accept loop");
}

}  // namespace mgp

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
using namespace mgp;

struct mgp_batch_plan {
    int device = 0;
    int count = 0;
    int variant = kMegopolis;
    uint32_t d = 0;
    uint32_t partition_bytes = 128;
    uint32_t b_max = kDefaultBMax;
    int use_graph = 1;
    std::string tune_cache;
    int nxcd = 1;
    int cu_count = 0;
    std::vector<mgp_filter_desc> filters;
    std::vector<FilterDev> fd_host;
    std::vector<uint32_t> est_B;
    // device memory: one allocation holding every table and pool
    char* dmem = nullptr;
    size_t dmem_bytes = 0;
    FilterDev* d_fd = nullptr;
    RTile* d_rtiles = nullptr;
    uint32_t n_rtiles = 0;
    Partial* d_parts = nullptr;
    mgp_stats* d_stats = nullptr;
    uint32_t* d_qcount = nullptr;
    // the accept loop's tile table (rebuilt per launch shape)
    LTile* d_ltiles = nullptr;
    uint32_t* d_qoff = nullptr;
    uint32_t n_ltiles = 0;  // capacity of d_ltiles
    uint32_t n_table = 0;   // entries of the current table
    uint32_t grid = 0;
    LoopShape shape{256, 4, 1};
    int from_cache = 0;
    double est_steps = 0.0;
    int64_t particles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    FilterDev* h_staging = nullptr;  // pinned copy of the filter table for seed updates
    hipEvent_t staging_done = nullptr;
    // per-filter workspaces of the separate-launch comparison path
    char* d_sep = nullptr;
    std::vector<size_t> sep_off;
};

namespace {

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(MGP_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

int validate(const mgp_filter_desc* f, int32_t count, const mgp_batch_config* cfg)
{
    if (!f || !cfg) return fail(MGP_EINVAL, "filters and config must not be NULL");
    if (count < 1) return fail(MGP_EINVAL, "count must be >= 1");
    if (cfg->variant < MGP_METROPOLIS || cfg->variant > MGP_MEGOPOLIS)
        return fail(MGP_EINVAL, "unknown variant %d", cfg->variant);
    if (cfg->d < 0) return fail(MGP_EINVAL, "d must be >= 0");
    const uint32_t pb = cfg->partition_bytes ? cfg->partition_bytes : 128u;
    if (pb < 4u || pb % 4u) return fail(MGP_EINVAL, "partition_bytes must be a positive multiple of 4");
    const uint32_t bmax = cfg->b_max ? cfg->b_max : kDefaultBMax;
    if (bmax > kBMaxLimit) return fail(MGP_ERANGE, "b_max above %u", kBMaxLimit);
    for (int32_t i = 0; i < count; ++i) {
        const mgp_filter_desc& x = f[i];
        if (!x.w_dev || !x.ancestors_dev) return fail(MGP_EINVAL, "filter %d: NULL weights or ancestors", i);
        if (x.n < 1 || (uint32_t)x.n > kBatchMaxN) return fail(MGP_ERANGE, "filter %d: n = %d out of range", i, x.n);
        if (x.reserved) return fail(MGP_EINVAL, "filter %d: reserved must be 0", i);
        if (x.B == 0 && (!(x.epsilon > 0.0) || !(x.epsilon <= 1.0)))
            return fail(MGP_EINVAL, "filter %d: epsilon must be in (0, 1] when B is 0", i);
        if (x.B > bmax) return fail(MGP_ERANGE, "filter %d: B = %u above b_max = %u", i, x.B, bmax);
        if (x.states_dev && (!x.out_states_dev || cfg->d < 1))
            return fail(MGP_EINVAL, "filter %d: states need out_states_dev and d >= 1", i);
    }
    return MGP_OK;
}

std::string cache_key(const mgp_batch_plan* p, const char* arch)
{
    // size class of the batch: filter count, total particles and mean B, in
    // powers of two, plus the variant and state dimension
    double mean_b = p->particles ? p->est_steps / (double)p->particles : 0.0;
    std::ostringstream k;
    k << arch << "/v" << p->variant << "/d" << p->d << "/f" << (int)lround(log2((double)p->count)) << "/n"
      << (int)lround(log2((double)std::max<int64_t>(1, p->particles))) << "/b"
      << (int)lround(log2(std::max(1.0, mean_b)));
    return k.str();
}

std::map<std::string, LoopShape> read_cache(const std::string& path)
{
    std::map<std::string, LoopShape> m;
    std::ifstream in(path);
    std::string key;
    LoopShape s;
    while (in >> key >> s.bt >> s.ppt >> s.sched) m[key] = s;
    return m;
}

void write_cache(const std::string& path, const std::map<std::string, LoopShape>& m)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream out(tmp);
        for (const auto& kv : m) out << kv.first << ' ' << kv.second.bt << ' ' << kv.second.ppt << ' ' << kv.second.sched << '\n';
    }
    rename(tmp.c_str(), path.c_str());
}

// Builds the accept loop's tile table for a launch shape: filters placed on
// XCDs by LPT on N_f * B_f, tiles of heavier filters first inside each XCD.
int build_tiles(mgp_batch_plan* p, const LoopShape& sh, hipStream_t s)
{
    const int nx = p->nxcd;
    std::vector<uint32_t> ns(p->count);
    std::vector<double> cost(p->count);
    for (int f = 0; f < p->count; ++f) {
        ns[f] = (uint32_t)p->filters[f].n;
        cost[f] = (double)ns[f] * std::max<uint32_t>(1u, p->est_B[f]);
    }
    std::vector<LTile> table;
    std::vector<uint32_t> qoff(kMaxXcd + 1, 0);
    build_tile_table(ns, cost, sh, nx, table, qoff.data());
    if (sh.sched == 1) {
        p->grid = (uint32_t)table.size();
    } else {
        // resident blocks per CU of the persistent kernel decide its grid
        const int occ = persistent_occupancy(p->variant, sh);
        uint32_t g = (uint32_t)(p->cu_count * occ);
        g = std::max<uint32_t>(nx, g - g % nx);
        p->grid = std::min<uint32_t>(g, (uint32_t)std::max<size_t>(table.size(), nx));
    }
    if (table.empty()) table.push_back(LTile{kNoFilter, 0});
    // (re)allocate the tile table if it grew
    const size_t need = table.size() * sizeof(LTile);
    if (need > (size_t)p->n_ltiles * sizeof(LTile)) {
        if (p->d_ltiles) HIP_TRY(hipFree(p->d_ltiles));
        p->d_ltiles = nullptr;
        HIP_TRY(hipMalloc(&p->d_ltiles, need));
        p->n_ltiles = (uint32_t)table.size();
    }
    HIP_TRY(hipMemcpyAsync(p->d_ltiles, table.data(), need, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_qoff, qoff.data(), qoff.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    p->shape = sh;
    p->n_table = (uint32_t)table.size();
    return MGP_OK;
}

int enqueue_run(mgp_batch_plan* p, hipStream_t s)
{
    return enqueue_batch(p->variant, p->shape, p->d_fd, (uint32_t)p->count, p->d_rtiles, p->n_rtiles, p->d_parts,
                         p->d_stats, p->d_ltiles, p->grid, p->d_qoff, p->d_qcount, (uint32_t)p->nxcd, p->d, s);
}

int capture_graph(mgp_batch_plan* p)
{
    if (p->exec) HIP_TRY(hipGraphExecDestroy(p->exec));
    if (p->graph) HIP_TRY(hipGraphDestroy(p->graph));
    p->exec = nullptr;
    p->graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_run(p, p->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(MGP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return MGP_OK;
}

// Times one shape: two warm runs, then the best of three.
int time_shape(mgp_batch_plan* p, const LoopShape& sh, hipStream_t s, float* ms_out)
{
    int rc = build_tiles(p, sh, s);
    if (rc) return rc;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best = 1e30f;
    for (int r = 0; r < 5 && rc == MGP_OK; ++r) {
        float ms = 0;
        if (hipEventRecord(a, s) != hipSuccess) rc = fail(MGP_EHIP, "hipEventRecord failed");
        if (!rc) rc = enqueue_run(p, s);
        if (!rc && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&ms, a, b) != hipSuccess))
            rc = fail(MGP_EHIP, "tuning run failed");
        if (r >= 2) best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_out = best;
    return rc;
}

void free_plan(mgp_batch_plan* p)
{
    if (!p) return;
    // best-effort teardown: a failure here leaves nothing to recover
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->staging_done) (void)hipEventDestroy(p->staging_done);
    if (p->h_staging) (void)hipHostFree(p->h_staging);
    if (p->d_ltiles) (void)hipFree(p->d_ltiles);
    if (p->d_sep) (void)hipFree(p->d_sep);
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}

}  // namespace

extern "C" {

int mgp_batch_plan_create(const mgp_filter_desc* filters, int32_t count, const mgp_batch_config* cfg, void* stream,
                          mgp_batch_plan** out)
{
    clear_error();
    if (!out) return fail(MGP_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    int rc = validate(filters, count, cfg);
    if (rc) return rc;
    if (cfg->block_threads || cfg->particles_per_thread || cfg->schedule) {
        const LoopShape want{cfg->block_threads ? cfg->block_threads : 256,
                             cfg->particles_per_thread ? cfg->particles_per_thread
                                                       : (cfg->variant == MGP_MEGOPOLIS ? 4 : 1),
                             cfg->schedule ? cfg->schedule : 1};
        if (!batch_shape_supported(cfg->variant, want))
            return fail(MGP_EINVAL, "unsupported launch shape bt=%d ppt=%d schedule=%d", want.bt, want.ppt, want.sched);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mgp_batch_plan* p = new mgp_batch_plan();
    p->count = count;
    p->variant = cfg->variant;
    p->d = (uint32_t)cfg->d;
    p->partition_bytes = cfg->partition_bytes ? cfg->partition_bytes : 128u;
    p->b_max = cfg->b_max ? cfg->b_max : kDefaultBMax;
    p->use_graph = cfg->use_graph;
    if (cfg->tune_cache) p->tune_cache = cfg->tune_cache;
    p->filters.assign(filters, filters + count);
    auto bail = [&](int code) {
        free_plan(p);
        return code;
    };
    if (hipGetDevice(&p->device) != hipSuccess) return bail(fail(MGP_EHIP, "hipGetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess)
        return bail(fail(MGP_EHIP, "hipGetDeviceProperties failed"));
    p->cu_count = prop.multiProcessorCount;
    p->nxcd = (p->cu_count >= 64 && p->cu_count % kMaxXcd == 0) ? kMaxXcd : 1;

    // ---- layout of the plan's device memory
    const bool mego = p->variant == kMegopolis;
    size_t off = 0;
    const size_t o_fd = off;
    off = align256(off + sizeof(FilterDev) * (size_t)count);
    std::vector<RTile> rt;
    std::vector<uint32_t> chunks(count), nparts(count), part_base(count);
    uint32_t total_parts = 0;
    for (int f = 0; f < count; ++f) {
        const uint32_t n = (uint32_t)filters[f].n;
        nparts[f] = reduce_blocks(n);
        chunks[f] = reduce_chunk(n, nparts[f]);
        part_base[f] = total_parts;
        total_parts += nparts[f];
        for (uint32_t c = 0; c < nparts[f]; ++c) rt.push_back(RTile{(uint32_t)f, c});
    }
    p->n_rtiles = (uint32_t)rt.size();
    const size_t o_rt = off;
    off = align256(off + sizeof(RTile) * rt.size());
    const size_t o_parts = off;
    off = align256(off + sizeof(Partial) * (size_t)total_parts);
    const size_t o_stats = off;
    off = align256(off + sizeof(mgp_stats) * (size_t)count);
    const size_t o_q = off;
    off = align256(off + sizeof(uint32_t) * 2 * (kMaxXcd + 1));
    std::vector<size_t> o_offs(count, 0), o_mirror(count, 0);
    if (mego) {
        for (int f = 0; f < count; ++f) {
            o_offs[f] = off;
            off = align256(off + sizeof(uint32_t) * (size_t)p->b_max);
        }
        for (int f = 0; f < count; ++f) {
            o_mirror[f] = off;
            off = align256(off + sizeof(float) * (2 * (size_t)filters[f].n + kMirrorPad));
        }
    }
    p->dmem_bytes = off;
    if (hipMalloc(&p->dmem, p->dmem_bytes) != hipSuccess)
        return bail(fail(MGP_ENOMEM, "could not allocate %zu bytes for the plan", p->dmem_bytes));
    p->d_fd = reinterpret_cast<FilterDev*>(p->dmem + o_fd);
    p->d_rtiles = reinterpret_cast<RTile*>(p->dmem + o_rt);
    p->d_parts = reinterpret_cast<Partial*>(p->dmem + o_parts);
    p->d_stats = reinterpret_cast<mgp_stats*>(p->dmem + o_stats);
    p->d_qcount = reinterpret_cast<uint32_t*>(p->dmem + o_q);
    p->d_qoff = p->d_qcount + (kMaxXcd + 1);

    p->fd_host.resize(count);
    const uint32_t n_w = p->partition_bytes / 4u;
    for (int f = 0; f < count; ++f) {
        const mgp_filter_desc& x = filters[f];
        FilterDev& F = p->fd_host[f];
        memset(&F, 0, sizeof F);
        F.w = x.w_dev;
        F.anc = x.ancestors_dev;
        F.states = x.states_dev;
        F.out = x.states_dev ? x.out_states_dev : nullptr;
        F.stats_user = x.stats_dev;
        F.mirror = mego ? reinterpret_cast<float*>(p->dmem + o_mirror[f]) : nullptr;
        F.offsets = mego ? reinterpret_cast<uint32_t*>(p->dmem + o_offs[f]) : nullptr;
        F.eps = x.epsilon;
        F.n = (uint32_t)x.n;
        F.B_user = x.B;
        F.b_max = p->b_max;
        F.key0 = (uint32_t)x.seed;
        F.key1 = (uint32_t)(x.seed >> 32);
        F.stream_id = x.stream_id;
        F.part_base = part_base[f];
        F.nparts = nparts[f];
        F.chunk = chunks[f];
        F.n_w = n_w;
        F.n_part = (uint32_t)(((uint64_t)F.n + n_w - 1u) / n_w);
        F.vec = (((uintptr_t)x.w_dev & 15u) == 0 && (!mego || F.n % 4u == 0)) ? 1u : 0u;
        F.rows4 = (p->d % 4u == 0 && ((uintptr_t)x.states_dev & 15u) == 0 && ((uintptr_t)x.out_states_dev & 15u) == 0)
                      ? 1u
                      : 0u;
        p->particles += x.n;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&p->h_staging), sizeof(FilterDev) * (size_t)count) != hipSuccess)
        return bail(fail(MGP_ENOMEM, "could not allocate pinned staging memory"));
    memcpy(p->h_staging, p->fd_host.data(), sizeof(FilterDev) * (size_t)count);
    if (hipEventCreateWithFlags(&p->staging_done, hipEventDisableTiming) != hipSuccess)
        return bail(fail(MGP_EHIP, "hipEventCreate failed"));
    if (hipMemcpyAsync(p->d_fd, p->h_staging, sizeof(FilterDev) * (size_t)count, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(p->d_rtiles, rt.data(), sizeof(RTile) * rt.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(p->staging_done, s) != hipSuccess)
        return bail(fail(MGP_EHIP, "uploading the plan tables failed"));
    if (hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(MGP_EHIP, "hipStreamCreate failed"));

    // ---- one reduction to learn every filter's B (load balance only)
    hipLaunchKernelGGL(k_batch_reduce, dim3(p->n_rtiles), dim3(kReduceThreads), 0, s, p->d_fd, p->d_rtiles, p->d_parts);
    hipLaunchKernelGGL(k_batch_finalize, dim3(p->count), dim3(kReduceThreads), 0, s, p->d_fd, p->d_parts, p->d_stats,
                       p->d_qcount, (uint32_t)kMaxXcd);
    rc = check_launch("plan-time reduction");
    if (rc) return bail(rc);
    std::vector<mgp_stats> st(count);
    if (hipMemcpyAsync(st.data(), p->d_stats, sizeof(mgp_stats) * (size_t)count, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(MGP_EHIP, "plan-time reduction failed"));
    p->est_B.resize(count);
    for (int f = 0; f < count; ++f) {
        p->est_B[f] = st[f].status == MGP_OK ? st[f].B : 0u;
        p->est_steps += (double)filters[f].n * p->est_B[f];
    }

    // ---- launch shape: given, cached, or tuned
    LoopShape chosen{256, mego ? 4 : 1, 1};
    if (cfg->block_threads || cfg->particles_per_thread || cfg->schedule) {
        chosen = LoopShape{cfg->block_threads ? cfg->block_threads : 256,
                           cfg->particles_per_thread ? cfg->particles_per_thread : (mego ? 4 : 1),
                           cfg->schedule ? cfg->schedule : 1};
    } else {
        const std::string key = cache_key(p, prop.gcnArchName);
        std::map<std::string, LoopShape> cache;
        if (!p->tune_cache.empty()) cache = read_cache(p->tune_cache);
        auto it = cache.find(key);
        if (it != cache.end() && batch_shape_supported(p->variant, it->second)) {
            chosen = it->second;
            p->from_cache = 1;
        } else {
            float best = 1e30f;
            for (const LoopShape& sh : candidate_shapes(p->variant)) {
                float ms = 0;
                rc = time_shape(p, sh, s, &ms);
                if (rc) return bail(rc);
                if (ms < best) {
                    best = ms;
                    chosen = sh;
                }
            }
            if (!p->tune_cache.empty()) {
                cache[key] = chosen;
                write_cache(p->tune_cache, cache);
            }
        }
    }
    rc = build_tiles(p, chosen, s);
    if (rc) return bail(rc);
    if (p->use_graph) {
        rc = capture_graph(p);
        if (rc) return bail(rc);
    }
    *out = p;
    return MGP_OK;
}

int mgp_batch_set_seeds(mgp_batch_plan* p, const uint64_t* seeds, void* stream)
{
    clear_error();
    if (!p || !seeds) return fail(MGP_EINVAL, "NULL argument");
    // the previous upload must have left the pinned buffer
    HIP_TRY(hipEventSynchronize(p->staging_done));
    for (int f = 0; f < p->count; ++f) {
        p->fd_host[f].key0 = (uint32_t)seeds[f];
        p->fd_host[f].key1 = (uint32_t)(seeds[f] >> 32);
        p->filters[f].seed = seeds[f];
    }
    memcpy(p->h_staging, p->fd_host.data(), sizeof(FilterDev) * (size_t)p->count);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(p->d_fd, p->h_staging, sizeof(FilterDev) * (size_t)p->count, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(p->staging_done, s));
    return MGP_OK;
}

int mgp_batch_run(mgp_batch_plan* p, void* stream)
{
    clear_error();
    if (!p) return fail(MGP_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->exec) {
        HIP_TRY(hipGraphLaunch(p->exec, s));
        return MGP_OK;
    }
    return enqueue_run(p, s);
}

int mgp_batch_run_separate(mgp_batch_plan* p, void* stream)
{
    clear_error();
    if (!p) return fail(MGP_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->d_sep) {
        size_t total = 0;
        p->sep_off.resize(p->count);
        for (int f = 0; f < p->count; ++f) {
            Params q{p->variant, p->filters[f].B, p->filters[f].epsilon, p->filters[f].seed,
                     p->filters[f].stream_id, p->partition_bytes, p->b_max};
            p->sep_off[f] = total;
            total += align256(workspace_bytes((uint32_t)p->filters[f].n, q));
        }
        if (hipMalloc(&p->d_sep, total) != hipSuccess)
            return fail(MGP_ENOMEM, "could not allocate %zu bytes of per-filter workspaces", total);
    }
    for (int f = 0; f < p->count; ++f) {
        const mgp_filter_desc& x = p->filters[f];
        Params q{p->variant, x.B, x.epsilon, x.seed, x.stream_id, p->partition_bytes, p->b_max};
        char* ws = p->d_sep + p->sep_off[f];
        int rc = enqueue_resample(x.w_dev, (uint32_t)x.n, q, ws, x.stats_dev, x.ancestors_dev, s);
        if (rc) return rc;
        if (x.states_dev) {
            rc = enqueue_gather(x.states_dev, (uint32_t)x.n, p->d, x.ancestors_dev, (uint32_t)x.n, x.out_states_dev, s);
            if (rc) return rc;
        }
    }
    return MGP_OK;
}

int mgp_batch_plan_info(const mgp_batch_plan* p, mgp_batch_info* info)
{
    clear_error();
    if (!p || !info) return fail(MGP_EINVAL, "NULL argument");
    info->filters = p->count;
    info->block_threads = p->shape.bt;
    info->particles_per_thread = p->shape.ppt;
    info->schedule = p->shape.sched;
    info->from_cache = p->from_cache;
    info->xcds = p->nxcd;
    info->particles = p->particles;
    info->tiles = p->n_table;
    info->device_bytes = (int64_t)p->dmem_bytes + (int64_t)p->n_ltiles * (int64_t)sizeof(LTile);
    info->est_particle_steps = p->est_steps;
    info->grid = p->grid;
    return MGP_OK;
}

int mgp_batch_plan_destroy(mgp_batch_plan* p)
{
    clear_error();
    if (!p) return MGP_OK;
    free_plan(p);
    return MGP_OK;
}

}  // extern "C"
