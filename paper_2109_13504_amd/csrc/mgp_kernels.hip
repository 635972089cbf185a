// mgp_kernels.hip -- single-filter kernels for gfx950 and the C ABI of
// include/mgp.h: weight reduction, B selection and Megopolis offsets, the
// four accept loops, and the particle gather.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "mgp.h"
#include "mgp_device.h"
#include "mgp_internal.h"
#include "mgp_reduce.h"

namespace mgp {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MGP_EHIP, "%s: %s", what, hipGetErrorString(e));
    return MGP_OK;
}

// ---------------------------------------------------------------------------
// 1. Reduction: fp32 max, fp64 sum, invalid-weight flag, per block.
//    The block decomposition depends on n only, so the fp64 sum (and B) is
//    the same on every call.
// ---------------------------------------------------------------------------
// Block b reduces w[b*chunk, min(n, (b+1)*chunk)); chunk is a multiple of 4
// and, with Vec, w is 16-byte aligned so float4 loads stay aligned (with a
// mirror, Vec also needs n % 4 == 0). Block 0 also writes the mirror's
// padding.
template <bool Vec>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const float* __restrict__ w, uint32_t n,
                                                           uint32_t chunk, Partial* __restrict__ part,
                                                           float* __restrict__ mirror)
{
    // trailing blocks may start at or past n when chunk was rounded up: their
    // range is empty and they contribute the neutral partial
    const uint64_t start = (uint64_t)blockIdx.x * chunk;
    const uint64_t stop = start + chunk < (uint64_t)n ? start + chunk : (uint64_t)n;
    const uint64_t end = stop > start ? stop : start;
    float mx = 0.0f;
    double s = 0.0;
    uint32_t bad = 0;
    reduce_range<Vec>(w, n, start, end, mirror, mx, s, bad);
    if (mirror && blockIdx.x == 0) mirror_pad(w, n, mirror);
    block_reduce(mx, s, bad);
    if (threadIdx.x == 0) part[blockIdx.x] = Partial{s, mx, bad};
}

// ---------------------------------------------------------------------------
// 2. Finalize: see finalize_one in mgp_reduce.h.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_finalize(const Partial* __restrict__ part, uint32_t nparts,
                                                             FinalizeArgs a, mgp_stats* __restrict__ st,
                                                             mgp_stats* __restrict__ st_user,
                                                             uint32_t* __restrict__ offsets)
{
    finalize_one(part, nparts, a, st, st_user, offsets);
}

// ---------------------------------------------------------------------------
// 3. The accept loop, one particle per thread.
// ---------------------------------------------------------------------------
template <int V, bool Narrow>
__global__ __launch_bounds__(kLoopThreads) void k_resample(const float* __restrict__ w, uint32_t n, uint32_t m,
                                                           const mgp_stats* __restrict__ st,
                                                           const uint32_t* __restrict__ offsets, uint32_t key0,
                                                           uint32_t key1, uint32_t stream_id, uint32_t n_w,
                                                           uint32_t n_part, uint32_t tag, uint32_t b_cap,
                                                           uint32_t seg_mask, int32_t* __restrict__ anc, RowCopy rc)
{
    const uint32_t i = blockIdx.x * kLoopThreads + threadIdx.x;
    const uint32_t B = st->B;
    // the stats must come from the reduction of this very call (same n,
    // variant, seed and stream), and B must fit the workspace
    const bool ok = st->status == MGP_OK && st->tag == tag && st->n == n && B <= b_cap;
    int32_t k = -1;
    if (ok) {
        // every lane runs a chain, also past m (C2 shares each group's
        // partition draws across its half-wave): output i starts at input
        // i mod n, i itself when i < n
        LoopParams P{w, offsets, n, B, key0, key1, stream_id, n_w, n_part, seg_mask};
        const uint32_t pos = i < n ? i : i % n;
        k = (int32_t)run_chain<V, Narrow, true>(P, i, pos);
    }
    if (i >= m) return;
    if (anc) anc[i] = k;
    if (rc.states) copy_row(rc, i, k);
}

// Megopolis over the mirrored weights, kMegopolisPPT particles per thread.
// Rows selects the particle copy of the epilogue: 0 none, D4 > 0 rows of D4
// float4s, -1 any row shape (copy_row).
template <int P, int Rows>
__global__ __launch_bounds__(kLoopThreads) void k_megopolis_mirror(const float* __restrict__ mirror, uint32_t n,
                                                                   uint32_t m, const mgp_stats* __restrict__ st,
                                                                   const uint32_t* __restrict__ offsets,
                                                                   uint32_t key0, uint32_t key1, uint32_t stream_id,
                                                                   uint32_t tag, uint32_t b_cap, uint32_t seg_mask,
                                                                   int32_t* __restrict__ anc, RowCopy rc)
{
    const uint32_t i0 = blockIdx.x * (kLoopThreads * P) + threadIdx.x;
    const uint32_t B = st->B;
    const bool ok = st->status == MGP_OK && st->tag == tag && st->n == n && B <= b_cap;
    uint32_t idx[P];
    int32_t k[P];
    bool live[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        idx[p] = i0 + kLoopThreads * p;
        live[p] = idx[p] < m;
        k[p] = -1;
    }
    if (ok) {
        // every lane runs, also past m (m <= n here): the mirror's padding
        // keeps those loads in bounds, and only real outputs store
        uint32_t kc[P];
        megopolis_mirror_chain<P>(reinterpret_cast<const char*>(mirror), offsets, n, B, key0, key1, stream_id, i0,
                                  kc, seg_mask);
#pragma unroll
        for (int p = 0; p < P; ++p) k[p] = (int32_t)kc[p];
    }
    if (anc) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (live[p]) anc[idx[p]] = k[p];
    }
    if constexpr (Rows > 0) {
        copy_rows_vec4<P, Rows>(rc, idx, k, live);
    } else if constexpr (Rows < 0) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (live[p]) copy_row(rc, idx[p], k[p]);
    }
}

// Megopolis over the mirrored weights for small n: one particle per thread,
// kDeepSteps candidate loads per round trip (megopolis_mirror_chain_deep).
// Used for m <= kDeepMaxM outputs, where the four-particle kernel leaves too
// few waves in flight to hide its round trips.
constexpr int kDeepSteps = 20;
constexpr uint32_t kDeepMaxM = 1u << 18;

__global__ __launch_bounds__(kLoopThreads) void k_megopolis_mirror_deep(const float* __restrict__ mirror, uint32_t n,
                                                                        uint32_t m, const mgp_stats* __restrict__ st,
                                                                        const uint32_t* __restrict__ offsets,
                                                                        uint32_t key0, uint32_t key1,
                                                                        uint32_t stream_id, uint32_t tag,
                                                                        uint32_t b_cap, uint32_t seg_mask,
                                                                        int32_t* __restrict__ anc, RowCopy rc)
{
    const uint32_t i = blockIdx.x * kLoopThreads + threadIdx.x;
    const uint32_t B = st->B;
    const bool ok = st->status == MGP_OK && st->tag == tag && st->n == n && B <= b_cap;
    int32_t k = -1;
    // lanes past m run too (the mirror's padding keeps their loads in bounds)
    if (ok)
        k = (int32_t)megopolis_mirror_chain_deep<kDeepSteps>(reinterpret_cast<const char*>(mirror), offsets, n, B,
                                                             key0, key1, stream_id, i, seg_mask);
    if (i < m) {
        if (anc) anc[i] = k;
        if (rc.states) copy_row(rc, i, k);
    }
}


// mgp_resample of a small filter in one launch (Megopolis up to kSmallMaxN
// particles, the other variants up to kSmallMaxNOther): every block copies
// the weights into LDS as the mirror M[k] = w[k mod n] and repeats the
// reduction of k_reduce and k_finalize chunk by chunk in the same order (so
// the fp64 sum, B and the stats are bit-identical to the three-launch path,
// B by eq. (proposition) of Section 4.1), then runs the chains of its own
// particles against LDS: k_megopolis_split<kSplitSmall> for Megopolis
// (Algorithm 5), k_resample_small for Algorithms 2-4.
constexpr uint32_t kSmallMaxN = 8192;
constexpr uint32_t kSmallMaxNOther = 4096;  // Metropolis, C1, C2: chains without shared indices gain less
constexpr uint32_t kSmallPad = 512;       // lanes past n: slot <= n + 255 + n - 1 + 63 < 2n + 512
constexpr uint32_t kSmallMaxParts = kSmallMaxN / kReduceChunk;
static_assert(kSmallMaxN % kReduceChunk == 0 && kSmallMaxN <= (uint64_t)kReduceChunk * kMaxPartials,
              "the reduction of a small filter has at most kSmallMaxParts chunks");

// The first steps of the one-launch kernels: the LDS mirror
// M[k] = w[k mod n], k < 2n + kSmallPad, then the reduction and B exactly as
// k_reduce and k_finalize compute them (chunks of `chunk` weights with
// k_reduce's thread mapping: float4 folds when fold_vec). Block 0 returns the
// stats. Returns B (0 for invalid weights) in every thread.
__device__ __forceinline__ uint32_t small_prologue(const float* __restrict__ w, uint32_t n, uint32_t nparts,
                                                   uint32_t chunk, uint32_t copy_vec, uint32_t fold_vec,
                                                   const FinalizeArgs& a, mgp_stats* __restrict__ st_ws,
                                                   mgp_stats* __restrict__ st_user, float* __restrict__ M,
                                                   Partial* __restrict__ parts, mgp_stats* __restrict__ st_local)
{
    // 1. the mirror: every load of a thread is issued before its first LDS
    //    store (clamped indices, no branch around a load), so the copy costs
    //    one round trip to L2, not one per element
    if (copy_vec) {  // w 16-byte aligned and n % 4 == 0
        constexpr uint32_t kIt = kSmallMaxN / (4u * kLoopThreads);
        const float4* w4 = reinterpret_cast<const float4*>(w);
        const uint32_t last4 = n / 4u - 1u;
        float4 v[kIt];
#pragma unroll
        for (uint32_t it = 0; it < kIt; ++it) {
            const uint32_t k4 = threadIdx.x + it * kLoopThreads;
            v[it] = w4[k4 < last4 ? k4 : last4];
        }
        // lanes past the end store the last element again, to its own place
#pragma unroll
        for (uint32_t it = 0; it < kIt; ++it) {
            const uint32_t k4 = threadIdx.x + it * kLoopThreads;
            const uint32_t c4 = k4 < last4 ? k4 : last4;
            *reinterpret_cast<float4*>(M + 4u * c4) = v[it];
            *reinterpret_cast<float4*>(M + 4u * c4 + n) = v[it];
        }
    } else {
        constexpr uint32_t kIt = kSmallMaxN / kLoopThreads;
        float v[kIt];
#pragma unroll
        for (uint32_t it = 0; it < kIt; ++it) {
            const uint32_t k = threadIdx.x + it * kLoopThreads;
            v[it] = w[k < n ? k : n - 1u];
        }
#pragma unroll
        for (uint32_t it = 0; it < kIt; ++it) {
            const uint32_t k = threadIdx.x + it * kLoopThreads;
            const uint32_t c = k < n ? k : n - 1u;
            M[c] = v[it];
            M[c + n] = v[it];
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kSmallPad; k += kLoopThreads) M[2u * n + k] = M[k % n];
    __syncthreads();
    // 2. the reduction, one chunk at a time with k_reduce's thread mapping
    for (uint32_t p = 0; p < nparts; ++p) {
        const uint64_t start = (uint64_t)p * chunk;
        const uint64_t stop = start + chunk < (uint64_t)n ? start + chunk : (uint64_t)n;
        const uint64_t end = stop > start ? stop : start;
        float mx = 0.0f;
        double s = 0.0;
        uint32_t bad = 0;
        if (fold_vec)
            reduce_range<true>(M, n, start, end, nullptr, mx, s, bad);
        else
            reduce_range<false>(M, n, start, end, nullptr, mx, s, bad);
        block_reduce(mx, s, bad);
        if (threadIdx.x == 0) parts[p] = Partial{s, mx, bad};
        __syncthreads();
    }
    // 3. B and the stats; block 0 returns them. The workspace record is
    //    marked unusable for mgp_resample_prepared (n = 0): this path leaves
    //    no offsets or mirror there.
    const uint32_t B = finalize_one(parts, nparts, a, st_local, blockIdx.x == 0 ? st_user : nullptr, nullptr);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        mgp_stats r = *st_local;
        r.n = 0;
        r.tag = 0;
        *st_ws = r;
    }
    return B;
}

// The split loop's modes: the B, stats and offsets of a preceding k_finalize
// (kSplitPrepared); the finalize step inside every block over the partials
// of a preceding k_reduce (kSplitFinalize); or, for n <= kSmallMaxN, the whole
// of mgp_resample in one launch with the weights in an LDS mirror
// (kSplitSmall, with small_prologue).
constexpr int kSplitPrepared = 0, kSplitFinalize = 1, kSplitSmall = 2;

// What the split loop needs beyond the prepared workspace.
struct SplitArgs {
    const Partial* parts;  // kSplitFinalize: the reduction's partials
    uint32_t nparts;       // kSplitFinalize, kSplitSmall
    FinalizeArgs a;        // kSplitFinalize, kSplitSmall
    mgp_stats* st_ws;      // kSplitFinalize, kSplitSmall: the workspace record, marked unusable
    mgp_stats* st_user;    // kSplitFinalize, kSplitSmall: the caller's stats or null
    const float* w;        // kSplitSmall: the weights
    uint32_t chunk;        // kSplitSmall: weights per reduction chunk
    uint32_t copy_vec;     // kSplitSmall: float4 copies into LDS
    uint32_t fold_vec;     // kSplitSmall: float4 folds in the reduction
};

constexpr uint32_t kSplitMaxM = 1u << 16;  // beyond, four waves per 64 particles cost more than they hide
// mgp_resample up to this size does the finalize step inside the split loop
// (beyond, its extra registers cost more than the launch it saves)
constexpr uint32_t kSplitFusedMaxN = 1u << 15;

// Megopolis over the mirrored weights for n up to kSplitMaxM, with each
// particle's draws spread over four lanes. A block serves 64 particles: in each pass of
// kSplitPass steps its four waves compute the particles' u draws (one Philox
// call per five steps), their candidates' mirror positions and candidate
// weights, all independent of the chain, into LDS; then wave 0 runs the
// chains, whose serial part is only the product, the compare and two selects
// per step. Every load of a pass is issued before the first LDS store, and
// steps past the pass write a spare row, so nothing branches around a load.
// The arithmetic and the draws are those of megopolis_mirror_chain_deep: the
// ancestors are identical.
// In modes kSplitFinalize (mgp_resample, n <= kSplitFusedMaxN) and
// kSplitSmall every block finds B itself and draws each pass's offsets into
// LDS (waves 1-3 draw the next pass's while wave 0 runs the chains), so the
// finalize launch goes; kSplitSmall also reads the candidates from its LDS
// mirror.
constexpr uint32_t kSplitPass = 20;  // steps per pass: a multiple of 20 (chain rounds) and of 5 (u blocks)
constexpr uint32_t kSplitGroups = kLoopThreads / 64u;
constexpr uint32_t kSplitBlocksPerWave = kSplitPass / (5u * kSplitGroups);
static_assert(kSplitPass % (5u * kSplitGroups) == 0 && kSplitPass % 20u == 0, "whole u blocks per wave and rounds");

template <int Mode>
__global__ __launch_bounds__(kLoopThreads) void k_megopolis_split(const float* __restrict__ mirror, uint32_t n,
                                                                  uint32_t m, const mgp_stats* __restrict__ st,
                                                                  const uint32_t* __restrict__ offsets,
                                                                  uint32_t key0, uint32_t key1, uint32_t stream_id,
                                                                  uint32_t tag, uint32_t b_cap, uint32_t seg_mask,
                                                                  int32_t* __restrict__ anc, SplitArgs f, RowCopy rc)
{
    __shared__ float su[kSplitPass + 1][64];   // row kSplitPass: the spare row
    __shared__ float swj[kSplitPass + 1][64];
    __shared__ uint32_t sjb[kSplitPass + 1][64];
    const uint32_t lane = threadIdx.x & 63u;
    // the wave's index, known to the compiler as wave-uniform: its offsets
    // are scalar loads
    const uint32_t q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t i = blockIdx.x * 64u + lane;
    constexpr bool kOwnOffsets = Mode != kSplitPrepared;
    __shared__ uint32_t soffs[2][kOwnOffsets ? kSplitPass : 1];  // this pass's offsets and the next pass's
    __shared__ __align__(16) float Ms[Mode == kSplitSmall ? 2 * kSmallMaxN + kSmallPad : 1];
    uint32_t B;
    bool ok;
    if constexpr (Mode == kSplitSmall) {
        // the weights into the LDS mirror, the reduction and B (small_prologue)
        __shared__ Partial parts[kSmallMaxParts];
        __shared__ mgp_stats st_local;
        B = small_prologue(f.w, n, f.nparts, f.chunk, f.copy_vec, f.fold_vec, f.a, f.st_ws, f.st_user, Ms, parts,
                           &st_local);
        ok = B > 0;
    } else if constexpr (Mode == kSplitFinalize) {
        // the finalize step in every block, over the partials k_reduce wrote:
        // B and the stats exactly as k_finalize computes them (block 0
        // returns the stats; the workspace record is marked unusable for a
        // prepared loop, which would find no offsets there)
        __shared__ mgp_stats st_local;
        B = finalize_one(f.parts, f.nparts, f.a, &st_local, blockIdx.x == 0 ? f.st_user : nullptr, nullptr);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            mgp_stats r = st_local;
            r.n = 0;
            r.tag = 0;
            *f.st_ws = r;
        }
        ok = B > 0;
    } else {
        B = st->B;
        ok = st->status == MGP_OK && st->tag == tag && st->n == n && B <= b_cap;
    }
    if (!ok) {
        if (q == 0 && i < m) {
            if (anc) anc[i] = -1;
            if (rc.states) copy_row(rc, i, -1);
        }
        return;
    }
    // lanes past m run too (the mirror's padding keeps their loads in bounds)
    const char* M = Mode == kSplitSmall ? reinterpret_cast<const char*>(Ms) : reinterpret_cast<const char*>(mirror);
    const uint32_t ia4 = (i & ~seg_mask) * 4u;
    const uint32_t il4 = (i & seg_mask) * 4u;
    uint32_t kk = i * 4u;
    float wk = *reinterpret_cast<const float*>(M + i * 4u);
    // the offsets of the pass starting at step c0, drawn as k_finalize draws
    // them, by the threads t0, t0 + stride, ... of the block
    auto draw_offsets = [&](uint32_t c0, uint32_t* dst, uint32_t t0, uint32_t stride) {
        const uint32_t cnt = B - c0 < kSplitPass ? B - c0 : kSplitPass;
        for (uint32_t c = t0; c < (cnt + 3u) / 4u; c += stride) {
            const Words x = philox(c0 / 4u + c, kTagOffset, stream_id, 0u, key0, key1);
            const uint32_t o[4] = {x.x0, x.x1, x.x2, x.x3};
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                if (4u * c + r < cnt) dst[4u * c + r] = uniform_index(o[r], n);
        }
    };
    if constexpr (kOwnOffsets) {
        draw_offsets(0u, soffs[0], threadIdx.x, kLoopThreads);
        __syncthreads();
    }
    for (uint32_t b0 = 0, buf = 0; b0 < B; b0 += kSplitPass, buf ^= 1u) {
        const uint32_t cnt = B - b0 < kSplitPass ? B - b0 : kSplitPass;
        // this wave's u blocks q, q + 4, ... of the pass: draws, positions and
        // candidate weights (steps past the pass use step cnt - 1's offset and
        // land in the spare row)
        UBlock ub[kSplitBlocksPerWave];
        uint32_t jb[kSplitBlocksPerWave][5];
        float wj[kSplitBlocksPerWave][5];
#pragma unroll
        for (uint32_t t = 0; t < kSplitBlocksPerWave; ++t) {
            const uint32_t g = q + kSplitGroups * t;
#pragma unroll
            for (uint32_t r = 0; r < 5u; ++r) {
                const uint32_t s = g * 5u + r;
                uint32_t o = kOwnOffsets ? soffs[buf][s < cnt ? s : cnt - 1u] : offsets[b0 + (s < cnt ? s : cnt - 1u)];
                o = o < n ? o : n - 1u;
                const uint32_t oa4 = (o & ~seg_mask) * 4u;
                const uint32_t voff = ia4 | ((il4 + (o & seg_mask) * 4u) & (seg_mask * 4u));
                wj[t][r] = *reinterpret_cast<const float*>(M + oa4 + voff);
                jb[t][r] = voff + oa4;
            }
        }
#pragma unroll
        for (uint32_t t = 0; t < kSplitBlocksPerWave; ++t)
            ub[t] = u_block(philox(b0 / 5u + q + kSplitGroups * t, kTagU, stream_id, i, key0, key1));
#pragma unroll
        for (uint32_t t = 0; t < kSplitBlocksPerWave; ++t) {
#pragma unroll
            for (uint32_t r = 0; r < 5u; ++r) {
                const uint32_t s = (q + kSplitGroups * t) * 5u + r;
                const uint32_t row = s < cnt ? s : kSplitPass;
                su[row][lane] = ub[t].u[r];
                swj[row][lane] = wj[t][r];
                sjb[row][lane] = jb[t][r];
            }
        }
        __syncthreads();
        if (q == 0) {
            uint32_t s0 = 0;
            for (; s0 + 20u <= cnt; s0 += 20u) {
                float uu[20], ww[20];
                uint32_t jj[20];
#pragma unroll
                for (uint32_t s = 0; s < 20u; ++s) {
                    uu[s] = su[s0 + s][lane];
                    ww[s] = swj[s0 + s][lane];
                    jj[s] = sjb[s0 + s][lane];
                }
#pragma unroll
                for (uint32_t s = 0; s < 20u; ++s) {
                    const float prod = uu[s] * wk;
                    const bool acc = prod <= ww[s];
                    kk = acc ? jj[s] : kk;
                    wk = acc ? ww[s] : wk;
                }
            }
            for (; s0 < cnt; ++s0) {
                const float prod = su[s0][lane] * wk;
                const float w = swj[s0][lane];
                const bool acc = prod <= w;
                kk = acc ? sjb[s0][lane] : kk;
                wk = acc ? w : wk;
            }
        } else if constexpr (kOwnOffsets) {
            // while wave 0 runs the chains, the other waves draw the next
            // pass's offsets into the other buffer
            if (b0 + kSplitPass < B) draw_offsets(b0 + kSplitPass, soffs[buf ^ 1u], threadIdx.x - 64u, kLoopThreads - 64u);
        }
        __syncthreads();  // the next pass overwrites the buffers
    }
    if (q == 0 && i < m) {
        const uint32_t k = kk / 4u;
        const int32_t kn = (int32_t)(k >= n ? k - n : k);
        if (anc) anc[i] = kn;
        if (rc.states) copy_row(rc, i, kn);
    }
}


// Metropolis, C1 and C2 (Algorithms 2-4) for a small filter in one launch:
// the same prologue, then each thread runs its particle's chain of k_resample
// against the weights in LDS.
template <int V>
__global__ __launch_bounds__(kLoopThreads) void k_resample_small(const float* __restrict__ w, uint32_t n,
                                                                 uint32_t nparts, uint32_t chunk, uint32_t copy_vec,
                                                                 uint32_t fold_vec, FinalizeArgs a,
                                                                 mgp_stats* __restrict__ st_ws,
                                                                 mgp_stats* __restrict__ st_user, uint32_t n_w,
                                                                 uint32_t n_part, int32_t* __restrict__ anc,
                                                                 RowCopy rc)
{
    __shared__ __align__(16) float M[2 * kSmallMaxN + kSmallPad];
    __shared__ Partial parts[kSmallMaxParts];
    __shared__ mgp_stats st_local;
    const uint32_t B = small_prologue(w, n, nparts, chunk, copy_vec, fold_vec, a, st_ws, st_user, M, parts, &st_local);
    const uint32_t i = blockIdx.x * kLoopThreads + threadIdx.x;
    int32_t k = -1;  // invalid weights: B == 0
    if (B > 0) {
        // every lane runs a chain (lanes past n from n - 1's group, whose
        // partition draws C2 shares across the half-wave)
        const LoopParams P{M, nullptr, n, B, a.key0, a.key1, a.stream_id, n_w, n_part};
        const uint32_t ic = i < n ? i : n - 1u;
        k = (int32_t)run_chain<V, true, true>(P, ic, ic);
    }
    if (i >= n) return;
    if (anc) anc[i] = k;
    if (rc.states) copy_row(rc, i, k);
}

// ---------------------------------------------------------------------------
// 4. Gather: out[i] = states[anc[i]] (rows of d fp32). With d % 4 == 0 and
//    16-byte aligned rows every thread copies one float4; otherwise one
//    float. Out-of-range ancestors give NaN rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather_vec4(const float4* __restrict__ states, uint32_t n_states,
                                                     uint32_t d4, const int32_t* __restrict__ anc, uint64_t total,
                                                     float4* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint64_t row = t / d4;
        const uint32_t c = (uint32_t)(t - row * d4);
        const int32_t k = anc[row];
        float4 v;
        if (k >= 0 && (uint32_t)k < n_states) {
            v = states[(uint64_t)k * d4 + c];
        } else {
            v = make_float4(NAN, NAN, NAN, NAN);
        }
        // the output is written once and not read here: stream it past the
        // L2 so that the ancestor rows being read stay cached
        __builtin_nontemporal_store(v.x, &out[t].x);
        __builtin_nontemporal_store(v.y, &out[t].y);
        __builtin_nontemporal_store(v.z, &out[t].z);
        __builtin_nontemporal_store(v.w, &out[t].w);
    }
}

__global__ __launch_bounds__(256) void k_gather_scalar(const float* __restrict__ states, uint32_t n_states,
                                                       uint32_t d, const int32_t* __restrict__ anc, uint64_t total,
                                                       float* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint64_t row = t / d;
        const uint32_t c = (uint32_t)(t - row * d);
        const int32_t k = anc[row];
        __builtin_nontemporal_store((k >= 0 && (uint32_t)k < n_states) ? states[(uint64_t)k * d + c] : NAN, &out[t]);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
uint32_t reduce_blocks(uint32_t n)
{
    // about kReduceChunk weights per block, at most kMaxPartials blocks
    uint64_t g = ((uint64_t)n + kReduceChunk - 1u) / kReduceChunk;
    if (g > kMaxPartials) g = kMaxPartials;
    if (g < 1) g = 1;
    return (uint32_t)g;
}

uint32_t reduce_chunk(uint32_t n, uint32_t blocks)
{
    uint64_t c = ((uint64_t)n + blocks - 1) / blocks;
    c = (c + 3u) & ~(uint64_t)3u;
    return (uint32_t)c;
}

int normalize_params(const mgp_params* in, Params* out)
{
    if (!in) return fail(MGP_EINVAL, "params is NULL");
    if (in->variant < MGP_METROPOLIS || in->variant > MGP_MEGOPOLIS)
        return fail(MGP_EINVAL, "unknown variant %d", in->variant);
    out->variant = in->variant;
    out->B = in->B;
    out->eps = in->epsilon;
    out->seed = in->seed;
    out->stream_id = in->stream_id;
    out->partition_bytes = in->partition_bytes ? in->partition_bytes : 128u;
    out->b_max = in->b_max ? in->b_max : kDefaultBMax;
    out->segment = in->segment ? in->segment : 32u;
    if (out->segment != 32u && out->segment != 64u)
        return fail(MGP_EINVAL, "segment must be 32 or 64 (got %u)", in->segment);
    if (out->partition_bytes < 4u || out->partition_bytes % 4u != 0u)
        return fail(MGP_EINVAL, "partition_bytes must be a positive multiple of 4 (got %u)", out->partition_bytes);
    if (out->b_max > kBMaxLimit) return fail(MGP_ERANGE, "b_max %u above the limit %u", out->b_max, kBMaxLimit);
    if (out->B == 0) {
        if (!(out->eps > 0.0) || !(out->eps <= 1.0))
            return fail(MGP_EINVAL, "epsilon must be in (0, 1] when B is 0 (got %g)", out->eps);
    } else if (out->B > out->b_max) {
        return fail(MGP_ERANGE, "B = %u above b_max = %u", out->B, out->b_max);
    }
    return MGP_OK;
}

size_t workspace_bytes(uint32_t b_max)
{
    return kWsOffsetsOffset + (((size_t)b_max * 4u + 255u) & ~(size_t)255u);
}

bool uses_mirror(uint32_t n, int variant) { return variant == kMegopolis && n <= kMirrorMaxN; }

size_t mirror_offset(uint32_t b_max) { return workspace_bytes(b_max); }

size_t workspace_bytes(uint32_t n, const Params& p)
{
    size_t b = workspace_bytes(p.b_max);
    if (uses_mirror(n, p.variant)) b += (((size_t)2 * n + kMirrorPad) * 4u + 255u) & ~(size_t)255u;
    return b;
}

// The reduction launch of the three-launch path: partials (and, for
// Megopolis with make_offsets, the mirror) in the workspace. Returns the
// number of partials through *nparts.
static int enqueue_reduce(const float* w, uint32_t n, const Params& p, bool make_offsets, char* ws, uint32_t* nparts,
                          hipStream_t stream)
{
    Partial* part = reinterpret_cast<Partial*>(ws + kWsPartialsOffset);
    float* mirror = (make_offsets && uses_mirror(n, p.variant)) ? reinterpret_cast<float*>(ws + mirror_offset(p.b_max))
                                                                  : nullptr;
    const uint32_t g = reduce_blocks(n);
    const uint32_t chunk = reduce_chunk(n, g);
    const bool vec = (((uintptr_t)w & 15u) == 0) && (!mirror || n % 4u == 0);
    if (vec)
        hipLaunchKernelGGL(k_reduce<true>, dim3(g), dim3(kReduceThreads), 0, stream, w, n, chunk, part, mirror);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(g), dim3(kReduceThreads), 0, stream, w, n, chunk, part, mirror);
    *nparts = g;
    return check_launch("reduce kernel");
}

static FinalizeArgs finalize_args(uint32_t n, const Params& p, bool make_offsets)
{
    FinalizeArgs a;
    a.n = n;
    a.eps = p.eps;
    a.B_user = p.B;
    a.b_max = p.b_max;
    a.make_offsets = make_offsets ? 1u : 0u;
    a.key0 = (uint32_t)p.seed;
    a.key1 = (uint32_t)(p.seed >> 32);
    a.stream_id = p.stream_id;
    a.tag = call_tag(n, p.variant, p.seed, p.stream_id);
    return a;
}

int enqueue_reduce_finalize(const float* w, uint32_t n, const Params& p, bool make_offsets, char* ws,
                            mgp_stats* st_user, hipStream_t stream)
{
    Partial* part = reinterpret_cast<Partial*>(ws + kWsPartialsOffset);
    mgp_stats* st = reinterpret_cast<mgp_stats*>(ws + kWsStatsOffset);
    uint32_t* offs = reinterpret_cast<uint32_t*>(ws + kWsOffsetsOffset);
    uint32_t g = 0;
    int rc = enqueue_reduce(w, n, p, make_offsets, ws, &g, stream);
    if (rc) return rc;
    const FinalizeArgs a = finalize_args(n, p, make_offsets);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kReduceThreads), 0, stream, part, g, a, st, st_user, offs);
    return check_launch("finalize kernel");
}

template <int V>
static void launch_loop(bool narrow, dim3 grid, hipStream_t s, const float* w, uint32_t n, uint32_t m,
                        const mgp_stats* st, const uint32_t* offs, uint32_t k0, uint32_t k1, uint32_t sid,
                        uint32_t n_w, uint32_t n_part, uint32_t tag, uint32_t b_cap, uint32_t seg_mask,
                        int32_t* anc, const RowCopy& rc)
{
    if (narrow)
        hipLaunchKernelGGL((k_resample<V, true>), grid, dim3(kLoopThreads), 0, s, w, n, m, st, offs, k0, k1, sid,
                           n_w, n_part, tag, b_cap, seg_mask, anc, rc);
    else
        hipLaunchKernelGGL((k_resample<V, false>), grid, dim3(kLoopThreads), 0, s, w, n, m, st, offs, k0, k1, sid,
                           n_w, n_part, tag, b_cap, seg_mask, anc, rc);
}

// The four-particle Megopolis loop with the epilogue that fits the row copy.
template <int Rows>
static void launch_mirror(dim3 g, hipStream_t s, const float* mirror, uint32_t n, uint32_t m, const mgp_stats* st,
                          const uint32_t* offs, uint32_t k0, uint32_t k1, uint32_t sid, uint32_t tag, uint32_t cap,
                          uint32_t seg_mask, int32_t* anc, const RowCopy& rc)
{
    hipLaunchKernelGGL((k_megopolis_mirror<kMegopolisPPT, Rows>), g, dim3(kLoopThreads), 0, s, mirror, n, m, st, offs,
                       k0, k1, sid, tag, cap, seg_mask, anc, rc);
}

int enqueue_loop(const float* w, uint32_t n, const Params& p, char* ws, int32_t* anc, hipStream_t stream,
                 const RowCopy& rc)
{
    return enqueue_loop_m(w, n, n, p, ws, anc, stream, rc);
}

int enqueue_loop_m(const float* w, uint32_t n, uint32_t m, const Params& p, char* ws, int32_t* anc,
                   hipStream_t stream, const RowCopy& rc)
{
    const mgp_stats* st = reinterpret_cast<const mgp_stats*>(ws + kWsStatsOffset);
    const uint32_t* offs = reinterpret_cast<const uint32_t*>(ws + kWsOffsetsOffset);
    const uint32_t n_w = p.partition_bytes / 4u;
    const uint32_t n_part = (uint32_t)(((uint64_t)n + n_w - 1u) / n_w);
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const dim3 grid((m + kLoopThreads - 1u) / kLoopThreads);
    const bool narrow = n <= (1u << 30);
    const uint32_t tag = call_tag(n, p.variant, p.seed, p.stream_id);
    const uint32_t cap = p.b_max;
    const uint32_t seg_mask = p.segment - 1u;
    if (uses_mirror(n, p.variant) && m <= n && m <= kDeepMaxM) {
        // few waves: up to 2^16 outputs the draws spread over four lanes, above
        // that twenty steps' loads per round trip, instead of four particles
        // per thread
        const float* mirror = reinterpret_cast<const float*>(ws + mirror_offset(p.b_max));
        if (m <= kSplitMaxM) {
            hipLaunchKernelGGL(k_megopolis_split<kSplitPrepared>, dim3((m + 63u) / 64u), dim3(kLoopThreads), 0, stream,
                               mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, SplitArgs{}, rc);
        } else {
            hipLaunchKernelGGL(k_megopolis_mirror_deep, grid, dim3(kLoopThreads), 0, stream, mirror, n, m, st, offs,
                               k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        }
        return check_launch("megopolis kernel (small n)");
    }
    if (uses_mirror(n, p.variant) && m <= n) {
        constexpr int P = kMegopolisPPT;
        const float* mirror = reinterpret_cast<const float*>(ws + mirror_offset(p.b_max));
        const dim3 g((m + kLoopThreads * P - 1u) / (kLoopThreads * P));
        const uint32_t d4 = rc.vec4 ? rc.d / 4u : 0u;
        if (!rc.states)
            launch_mirror<0>(g, stream, mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        else if (d4 == 1u)
            launch_mirror<1>(g, stream, mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        else if (d4 == 2u)
            launch_mirror<2>(g, stream, mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        else if (d4 == 4u)
            launch_mirror<4>(g, stream, mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        else
            launch_mirror<-1>(g, stream, mirror, n, m, st, offs, k0, k1, p.stream_id, tag, cap, seg_mask, anc, rc);
        return check_launch("megopolis kernel");
    }
    switch (p.variant) {
    case kMetropolis:
        launch_loop<kMetropolis>(narrow, grid, stream, w, n, m, st, offs, k0, k1, p.stream_id, n_w, n_part, tag, cap, seg_mask, anc,
                         rc);
        break;
    case kC1:
        launch_loop<kC1>(narrow, grid, stream, w, n, m, st, offs, k0, k1, p.stream_id, n_w, n_part, tag, cap, seg_mask, anc,
                         rc);
        break;
    case kC2:
        launch_loop<kC2>(narrow, grid, stream, w, n, m, st, offs, k0, k1, p.stream_id, n_w, n_part, tag, cap, seg_mask, anc,
                         rc);
        break;
    default:
        launch_loop<kMegopolis>(narrow, grid, stream, w, n, m, st, offs, k0, k1, p.stream_id, n_w, n_part, tag, cap, seg_mask, anc,
                         rc);
        break;
    }
    return check_launch("resample kernel");
}

// mgp_resample with n <= kSmallMaxN (Megopolis) or kSmallMaxNOther: one
// launch of k_megopolis_split<kSplitSmall> or k_resample_small. The reduction
// uses the chunks, thread mapping and fold width that enqueue_reduce_finalize
// uses for the same n, variant and weight alignment (float4 folds need a
// 16-byte aligned w, and with a mirror n % 4 == 0).
int enqueue_small(const float* w, uint32_t n, const Params& p, char* ws, mgp_stats* st_user, int32_t* anc,
                  hipStream_t stream, const RowCopy& rc)
{
    const uint32_t g = reduce_blocks(n);
    const uint32_t chunk = reduce_chunk(n, g);
    const bool aligned = ((uintptr_t)w & 15u) == 0;
    const uint32_t copy_vec = (aligned && n % 4u == 0) ? 1u : 0u;
    const uint32_t fold_vec = p.variant == kMegopolis ? copy_vec : (aligned ? 1u : 0u);
    const FinalizeArgs a = finalize_args(n, p, false);
    mgp_stats* st_ws = reinterpret_cast<mgp_stats*>(ws + kWsStatsOffset);
    const dim3 grid((n + kLoopThreads - 1u) / kLoopThreads);
    const uint32_t n_w = p.partition_bytes / 4u;
    const uint32_t n_part = (uint32_t)(((uint64_t)n + n_w - 1u) / n_w);
    switch (p.variant) {
    case kMegopolis: {
            SplitArgs f{};
            f.nparts = g;
            f.a = a;
            f.st_ws = st_ws;
            f.st_user = st_user;
            f.w = w;
            f.chunk = chunk;
            f.copy_vec = copy_vec;
            f.fold_vec = copy_vec;
            hipLaunchKernelGGL(k_megopolis_split<kSplitSmall>, dim3((n + 63u) / 64u), dim3(kLoopThreads), 0, stream,
                               nullptr, n, n, nullptr, nullptr, a.key0, a.key1, p.stream_id, a.tag, p.b_max,
                               p.segment - 1u, anc, f, rc);
            break;
        }
    case kMetropolis:
        hipLaunchKernelGGL(k_resample_small<kMetropolis>, grid, dim3(kLoopThreads), 0, stream, w, n, g, chunk,
                           copy_vec, fold_vec, a, st_ws, st_user, n_w, n_part, anc, rc);
        break;
    case kC1:
        hipLaunchKernelGGL(k_resample_small<kC1>, grid, dim3(kLoopThreads), 0, stream, w, n, g, chunk, copy_vec,
                           fold_vec, a, st_ws, st_user, n_w, n_part, anc, rc);
        break;
    default:
        hipLaunchKernelGGL(k_resample_small<kC2>, grid, dim3(kLoopThreads), 0, stream, w, n, g, chunk, copy_vec,
                           fold_vec, a, st_ws, st_user, n_w, n_part, anc, rc);
        break;
    }
    return check_launch("resample kernel (one launch)");
}

int enqueue_resample(const float* w, uint32_t n, const Params& p, char* ws, mgp_stats* st_user, int32_t* anc,
                     hipStream_t stream, const RowCopy& rc)
{
    if (n <= (p.variant == kMegopolis ? kSmallMaxN : kSmallMaxNOther))
        return enqueue_small(w, n, p, ws, st_user, anc, stream, rc);
    if (p.variant == kMegopolis && n <= kSplitFusedMaxN) {
        // two launches: the reduction (partials and mirror), then the split
        // accept loop with the finalize step done in every block
        uint32_t g = 0;
        const int err = enqueue_reduce(w, n, p, true, ws, &g, stream);
        if (err) return err;
        SplitArgs f{};
        f.parts = reinterpret_cast<const Partial*>(ws + kWsPartialsOffset);
        f.nparts = g;
        f.a = finalize_args(n, p, false);
        f.st_ws = reinterpret_cast<mgp_stats*>(ws + kWsStatsOffset);
        f.st_user = st_user;
        const float* mirror = reinterpret_cast<const float*>(ws + mirror_offset(p.b_max));
        hipLaunchKernelGGL(k_megopolis_split<kSplitFinalize>, dim3((n + 63u) / 64u), dim3(kLoopThreads), 0, stream,
                           mirror, n, n, nullptr, nullptr, f.a.key0, f.a.key1, p.stream_id, f.a.tag, p.b_max,
                           p.segment - 1u, anc, f, rc);
        return check_launch("megopolis kernel (finalize and split loop)");
    }
    int err = enqueue_reduce_finalize(w, n, p, p.variant == kMegopolis, ws, st_user, stream);
    if (err) return err;
    return enqueue_loop(w, n, p, ws, anc, stream, rc);
}

// One element (or float4) per thread up to 2^20 blocks, grid-stride beyond.
static uint32_t gather_blocks(uint64_t total)
{
    const uint64_t b = (total + 255u) / 256u;
    return (uint32_t)(b < (1u << 20) ? (b ? b : 1) : (1u << 20));
}

int enqueue_gather(const float* states, uint32_t n_states, uint32_t d, const int32_t* anc, uint32_t n_out,
                   float* out, hipStream_t stream)
{
    if (n_out == 0) return MGP_OK;
    const bool vec = (d % 4u == 0u) && (((uintptr_t)states & 15u) == 0) && (((uintptr_t)out & 15u) == 0);
    if (vec) {
        const uint32_t d4 = d / 4u;
        const uint64_t total = (uint64_t)n_out * d4;
        const dim3 grid(gather_blocks(total));
        hipLaunchKernelGGL(k_gather_vec4, grid, dim3(256), 0, stream, reinterpret_cast<const float4*>(states),
                           n_states, d4, anc, total, reinterpret_cast<float4*>(out));
    } else {
        const uint64_t total = (uint64_t)n_out * d;
        const dim3 grid(gather_blocks(total));
        hipLaunchKernelGGL(k_gather_scalar, grid, dim3(256), 0, stream, states, n_states, d, anc, total, out);
    }
    return check_launch("gather kernel");
}

}  // namespace mgp

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace mgp;

extern "C" {

const char* mgp_last_error(void) { return g_err; }

int mgp_version(void) { return kVersion; }

int mgp_workspace_size(int32_t n, const mgp_params* params, size_t* bytes)
{
    clear_error();
    if (!bytes) return fail(MGP_EINVAL, "bytes is NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    *bytes = workspace_bytes((uint32_t)n, p);
    return MGP_OK;
}

// Whether n_out rows of d floats at out overlap n_in rows at in.
static bool overlaps(const float* in, int32_t n_in, const float* out, int32_t n_out, int32_t d)
{
    const uint64_t in_bytes = (uint64_t)n_in * (uint64_t)d * 4u;
    const uint64_t out_bytes = (uint64_t)n_out * (uint64_t)d * 4u;
    const uintptr_t a0 = (uintptr_t)in, a1 = a0 + in_bytes;
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + out_bytes;
    return out_bytes && a0 < b1 && b0 < a1;
}

// The row copy of the fused entry points: n rows of d floats from states to
// out; float4 moves when d % 4 == 0 and both buffers are 16-byte aligned.
static int row_copy_args(const float* states, int32_t n, int32_t d, float* out, RowCopy* rc)
{
    if (!states || !out) return fail(MGP_EINVAL, "states_dev and out_dev must not be NULL");
    if (d < 1) return fail(MGP_EINVAL, "d must be >= 1 (got %d)", d);
    if (overlaps(states, n, out, n, d)) return fail(MGP_EINVAL, "out_dev overlaps states_dev");
    rc->states = states;
    rc->out = out;
    rc->d = (uint32_t)d;
    rc->vec4 = (d % 4 == 0 && ((uintptr_t)states & 15u) == 0 && ((uintptr_t)out & 15u) == 0) ? 1u : 0u;
    return MGP_OK;
}

static int check_workspace(void* ws, size_t ws_bytes, uint32_t n, const Params& p)
{
    if (!ws) return fail(MGP_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(MGP_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = workspace_bytes(n, p);
    if (ws_bytes < need) return fail(MGP_ERANGE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return MGP_OK;
}

int mgp_compute_B(const float* w_dev, int32_t n, const mgp_params* params, mgp_stats* stats_dev,
                  void* workspace_dev, size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev) return fail(MGP_EINVAL, "w_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    rc = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (rc) return rc;
    return enqueue_reduce_finalize(w_dev, (uint32_t)n, p, p.variant == kMegopolis,
                                   static_cast<char*>(workspace_dev), stats_dev, static_cast<hipStream_t>(stream));
}

int mgp_resample_prepared(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                          void* workspace_dev, size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev || !ancestors_dev) return fail(MGP_EINVAL, "w_dev and ancestors_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    rc = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (rc) return rc;
    return enqueue_loop(w_dev, (uint32_t)n, p, static_cast<char*>(workspace_dev), ancestors_dev,
                        static_cast<hipStream_t>(stream));
}

int mgp_resample(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                 mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev || !ancestors_dev) return fail(MGP_EINVAL, "w_dev and ancestors_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    rc = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (rc) return rc;
    return enqueue_resample(w_dev, (uint32_t)n, p, static_cast<char*>(workspace_dev), stats_dev, ancestors_dev,
                            static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free mgp_resample: the workspace is a fixed array in the code
// object's device memory instead of a caller buffer. Each device that runs
// the library holds its own copy of it until the process ends.
// ---------------------------------------------------------------------------
static_assert(MGP_NOALLOC_SCRATCH_BYTES % 256 == 0, "the scratch size is a multiple of the workspace alignment");
static __device__ __align__(256) unsigned char scratch[MGP_NOALLOC_SCRATCH_BYTES];

namespace mgp {

constexpr int kMaxDevices = 64;

// The device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address). Null
// after a failure, with the error message set.
static void* scratch_on_current_device(int* rc)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *rc = fail(MGP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *rc = fail(MGP_EINVAL, "device %d is beyond the %d devices the scratch table covers", dev, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *rc = fail(MGP_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return nullptr;
        }
        addr[dev] = p;
    }
    *rc = MGP_OK;
    return addr[dev];
}

}  // namespace mgp

extern "C" {

int mgp_resample_noalloc(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                         mgp_stats* stats_dev, void* stream)
{
    clear_error();
    if (!w_dev || !ancestors_dev) return fail(MGP_EINVAL, "w_dev and ancestors_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    const size_t need = workspace_bytes((uint32_t)n, p);
    if (need > (size_t)MGP_NOALLOC_SCRATCH_BYTES)
        return fail(MGP_ERANGE, "n = %d with these params needs %zu bytes of workspace; the static scratch holds %zu",
                    n, need, (size_t)MGP_NOALLOC_SCRATCH_BYTES);
    void* ws = scratch_on_current_device(&rc);
    if (!ws) return rc;
    return enqueue_resample(w_dev, (uint32_t)n, p, static_cast<char*>(ws), stats_dev, ancestors_dev,
                            static_cast<hipStream_t>(stream));
}

int mgp_resample_m(const float* w_dev, int32_t n, int32_t m, const mgp_params* params, int32_t* ancestors_dev,
                   mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev || !ancestors_dev) return fail(MGP_EINVAL, "w_dev and ancestors_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    if (m < 1) return fail(MGP_EINVAL, "m must be >= 1 (got %d)", m);
    Params p;
    int rc = normalize_params(params, &p);
    if (rc) return rc;
    rc = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (rc) return rc;
    char* ws = static_cast<char*>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = enqueue_reduce_finalize(w_dev, (uint32_t)n, p, p.variant == kMegopolis, ws, stats_dev, s);
    if (rc) return rc;
    return enqueue_loop_m(w_dev, (uint32_t)n, (uint32_t)m, p, ws, ancestors_dev, s);
}

int mgp_gather(const float* states_dev, int32_t n_states, int32_t d, const int32_t* ancestors_dev, int32_t n_out,
               float* out_dev, void* stream)
{
    clear_error();
    if (!states_dev || !ancestors_dev || !out_dev) return fail(MGP_EINVAL, "NULL pointer argument");
    if (n_states < 1 || d < 1 || n_out < 0) return fail(MGP_EINVAL, "need n_states >= 1, d >= 1, n_out >= 0");
    if (overlaps(states_dev, n_states, out_dev, n_out, d)) return fail(MGP_EINVAL, "out_dev overlaps states_dev");
    return enqueue_gather(states_dev, (uint32_t)n_states, (uint32_t)d, ancestors_dev, (uint32_t)n_out, out_dev,
                          static_cast<hipStream_t>(stream));
}

int mgp_resample_gather(const float* w_dev, int32_t n, const mgp_params* params, const float* states_dev, int32_t d,
                        int32_t* ancestors_dev, float* out_dev, mgp_stats* stats_dev, void* workspace_dev,
                        size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev) return fail(MGP_EINVAL, "w_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    RowCopy rc;
    int err = row_copy_args(states_dev, n, d, out_dev, &rc);
    if (err) return err;
    Params p;
    err = normalize_params(params, &p);
    if (err) return err;
    err = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (err) return err;
    return enqueue_resample(w_dev, (uint32_t)n, p, static_cast<char*>(workspace_dev), stats_dev, ancestors_dev,
                            static_cast<hipStream_t>(stream), rc);
}

int mgp_resample_gather_prepared(const float* w_dev, int32_t n, const mgp_params* params, const float* states_dev,
                                 int32_t d, int32_t* ancestors_dev, float* out_dev, void* workspace_dev,
                                 size_t workspace_bytes_, void* stream)
{
    clear_error();
    if (!w_dev) return fail(MGP_EINVAL, "w_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    RowCopy rc;
    int err = row_copy_args(states_dev, n, d, out_dev, &rc);
    if (err) return err;
    Params p;
    err = normalize_params(params, &p);
    if (err) return err;
    err = check_workspace(workspace_dev, workspace_bytes_, (uint32_t)n, p);
    if (err) return err;
    return enqueue_loop(w_dev, (uint32_t)n, p, static_cast<char*>(workspace_dev), ancestors_dev,
                        static_cast<hipStream_t>(stream), rc);
}

}  // extern "C"
