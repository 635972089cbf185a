// mgp_prefix.hip -- the prefix-sum resamplers of the C ABI (include/mgp.h):
// multinomial (Algorithm 7) and systematic (Algorithm 8) resampling, the
// unbiased comparison methods of Section 6.5 and Table 2.
//
// Both give output i the first input j whose inclusive prefix sum of weights
// exceeds a threshold t_i (multinomial: an independent uniform t_i per
// output; systematic: t_i = (i + u) S / N from one uniform u). The weights
// enter the prefix sum as 64-bit fixed point, q = floor(w 2^K), with K from
// the largest weight such that the total S stays below 2^62: integer sums are
// exact in any order, so the parallel scan here and a sequential sum give the
// same prefix and the same ancestors.
//
// The search runs down a 16-ary tree over the prefix sums: level 0 is the
// inclusive sums themselves, level k holds every 16^k-th of them (the sum at
// the end of each group of 16^k inputs), and the top level has at most 16
// entries. A lane reads one 128-byte row of 16 sums per level and counts the
// sums <= t, which is the child to descend into.
//
// Launches: the reduction and finalize step of the other resamplers
// (validation, max, fp64 sum), then
//   k_prefix_chunks   per chunk of kChunk weights: the fixed-point chunk sum
//   k_prefix_top      one block: exclusive sums over the chunks, the header
//   k_prefix_scan     per chunk: the inclusive sums (coalesced through LDS)
//                     and the tree's entries that fall in the chunk
//   multinomial:      k_prefix_multinomial, a descent per output (eight
//                     lanes share each row read)
//   systematic:       k_prefix_brackets, a descent for every 256th output,
//                     then k_prefix_systematic, a bisection per output between
//                     the two brackets of its group (thresholds rise with i)
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "mgp.h"
#include "mgp_device.h"
#include "mgp_internal.h"
#include "mgp_prefix.h"

namespace mgp {

constexpr uint32_t kPrefixThreads = 256;
constexpr uint32_t kPrefixPer = 8;                        // weights per thread in a chunk
constexpr uint32_t kChunk = kPrefixThreads * kPrefixPer;  // 2048 weights per chunk
constexpr uint32_t kFan = 16;                             // the tree's fan-out: one 128-byte row of sums
constexpr uint32_t kTagMultinomial = 6u;
constexpr uint32_t kTagSystematic = 7u;

// What the scan leaves for the search (in the workspace).
struct PrefixHeader {
    uint64_t total;  // S, the sum of the fixed-point weights (0: invalid weights)
    int32_t K;       // the fixed-point exponent
    int32_t valid;   // 1 when the weights passed validation
};

template <typename T>
__device__ __forceinline__ T* at(const PrefixJob& J, uint64_t off)
{
    return reinterpret_cast<T*>(J.region + (uint64_t)blockIdx.y * J.region_ld + off);
}

// K = 62 - ceil(log2 n) - E for w_max = m 2^E, m in [0.5, 1).
__device__ __forceinline__ int fixed_exponent(float w_max, int log2n_ceil)
{
    int E = 0;
    frexp((double)w_max, &E);
    return 62 - log2n_ceil - E;
}

// q = floor(w 2^K) for a finite w >= 0, from its fields: w = m 2^(e - 150)
// with m = 2^23 + mantissa for a normal w (biased exponent e >= 1), and
// w = mantissa 2^-149 for a subnormal one; the shift by e - 150 + K is exact
// (a right shift floors).
__device__ __forceinline__ uint64_t fixed_weight(float w, int K)
{
    const uint32_t bits = __float_as_uint(w) & 0x7FFFFFFFu;  // -0.0 is 0
    const uint32_t e = bits >> 23;
    const uint64_t m = e ? (uint64_t)((bits & 0x7FFFFFu) | 0x800000u) : (uint64_t)bits;
    const int sh = (e ? (int)e - 150 : -149) + K;
    if (sh >= 0) return m << sh;
    return sh <= -64 ? 0u : m >> (-sh);
}

// Block-wide exclusive scan of one uint64 per thread; returns the thread's
// exclusive prefix and the block total through *total.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* total)
{
    __shared__ uint64_t wave_sums[kPrefixThreads / 64];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, 64);
        if ((int)lane >= off) x += y;
    }
    if (lane == 63u) wave_sums[wv] = x;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPrefixThreads / 64; ++k) {
        const uint64_t s = wave_sums[k];
        if (k < wv) before += s;
        all += s;
    }
    __syncthreads();  // wave_sums is reused by the next call
    *total = all;
    return before + x - v;
}

// The fixed-point weights of this thread's kPrefixPer consecutive inputs of
// chunk `chunk` of the run (0 past n).
__device__ __forceinline__ void load_fixed(const PrefixJob& J, uint32_t chunk, int K, uint64_t (&q)[kPrefixPer])
{
    const float* __restrict__ w = J.w + (uint64_t)blockIdx.y * J.w_ld;
    const uint64_t base = (uint64_t)chunk * kChunk + (uint64_t)threadIdx.x * kPrefixPer;
    if (J.vec && base + kPrefixPer <= J.n) {
        const float4 a = *reinterpret_cast<const float4*>(w + base);
        const float4 b = *reinterpret_cast<const float4*>(w + base + 4);
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) q[e] = fixed_weight(v[e], K);
    } else {
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) q[e] = base + e < J.n ? fixed_weight(w[base + e], K) : 0u;
    }
}

__global__ __launch_bounds__(kPrefixThreads) void k_prefix_chunks(PrefixJob J)
{
    const mgp_stats& st = J.stats[blockIdx.y];
    uint64_t* chunk_sum = at<uint64_t>(J, J.o_sum);
    if (st.status != MGP_OK) {
        if (threadIdx.x == 0) chunk_sum[blockIdx.x] = 0;
        return;
    }
    uint64_t q[kPrefixPer];
    load_fixed(J, blockIdx.x, fixed_exponent(st.w_max, J.log2n), q);
    uint64_t s = 0;
#pragma unroll
    for (uint32_t e = 0; e < kPrefixPer; ++e) s += q[e];
    uint64_t total = 0;
    block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

// One block per run: chunk_excl[c] = sum of chunk_sum[0..c), and the header.
// The chunk sums go through LDS a tile of kChunk at a time, so that the
// loads and stores are coalesced; each thread scans kPrefixPer consecutive
// sums of the tile, and the tile's total carries into the next.
__global__ __launch_bounds__(kPrefixThreads) void k_prefix_top(PrefixJob J)
{
    __shared__ uint64_t tile[kChunk];
    const uint64_t* chunk_sum = at<uint64_t>(J, J.o_sum);
    uint64_t* chunk_excl = at<uint64_t>(J, J.o_excl);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < J.nch; base += kChunk) {
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) {
            const uint32_t c = base + e * kPrefixThreads + threadIdx.x;
            tile[e * kPrefixThreads + threadIdx.x] = c < J.nch ? chunk_sum[c] : 0u;
        }
        __syncthreads();
        uint64_t v[kPrefixPer];
        uint64_t s = 0;
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) {
            v[e] = tile[threadIdx.x * kPrefixPer + e];
            s += v[e];
        }
        uint64_t total = 0;
        uint64_t run = carry + block_exclusive_scan(s, &total);
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) {
            tile[threadIdx.x * kPrefixPer + e] = run;
            run += v[e];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t e = 0; e < kPrefixPer; ++e) {
            const uint32_t c = base + e * kPrefixThreads + threadIdx.x;
            if (c < J.nch) chunk_excl[c] = tile[e * kPrefixThreads + threadIdx.x];
        }
        carry += total;
        __syncthreads();  // the tile is overwritten next
    }
    if (threadIdx.x == 0) {
        const mgp_stats& st = J.stats[blockIdx.y];
        const bool ok = st.status == MGP_OK;
        PrefixHeader h;
        h.total = ok ? carry : 0u;
        h.K = ok ? fixed_exponent(st.w_max, J.log2n) : 0;
        h.valid = ok ? 1 : 0;
        *at<PrefixHeader>(J, J.o_hdr) = h;
    }
}

// The inclusive sums of one chunk: computed per thread over its kPrefixPer
// inputs, passed through LDS so that each store instruction writes 512
// contiguous bytes. Positions past n hold S (level 0 is padded to whole
// chunks). The tree's entries that fall in the chunk are written here too:
// level k entry m is the sum at position (m + 1) 16^k - 1, and the thread
// holding position n - 1 writes the last real entry (S) and the padding of
// every level.
__global__ __launch_bounds__(kPrefixThreads) void k_prefix_scan(PrefixJob J)
{
    __shared__ uint64_t stage[kChunk];
    const PrefixHeader h = *at<PrefixHeader>(J, J.o_hdr);
    if (!h.valid) return;
    uint64_t q[kPrefixPer];
    load_fixed(J, blockIdx.x, h.K, q);
    uint64_t s = 0;
#pragma unroll
    for (uint32_t e = 0; e < kPrefixPer; ++e) s += q[e];
    uint64_t total = 0;
    uint64_t run = at<uint64_t>(J, J.o_excl)[blockIdx.x] + block_exclusive_scan(s, &total);
    const uint64_t base = (uint64_t)blockIdx.x * kChunk;
    const uint64_t mine = base + (uint64_t)threadIdx.x * kPrefixPer;
#pragma unroll
    for (uint32_t e = 0; e < kPrefixPer; ++e) {
        run += q[e];
        stage[threadIdx.x * kPrefixPer + e] = run;
        const uint64_t p = mine + e;
        if (p < J.n && (p + 1u) % kFan == 0u) {
            // level k entry (p + 1) / 16^k - 1 for every k with 16^k | p + 1
            uint64_t g = (p + 1u) / kFan;
            for (int k = 1; k <= J.top; ++k) {
                at<uint64_t>(J, J.o_level[k])[g - 1u] = run;
                if (g % kFan != 0u) break;
                g /= kFan;
            }
        }
        if (p == (uint64_t)J.n - 1u) {
            for (int k = 1; k <= J.top; ++k) {
                uint64_t* lv = at<uint64_t>(J, J.o_level[k]);
                const uint32_t end = (J.count[k] + kFan - 1u) / kFan * kFan;
                for (uint32_t m = J.count[k] - 1u; m < end; ++m) lv[m] = run;
            }
        }
    }
    __syncthreads();
    uint64_t* incl = at<uint64_t>(J, J.o_incl);
#pragma unroll
    for (uint32_t e = 0; e < kPrefixPer; ++e)
        incl[base + e * kPrefixThreads + threadIdx.x] = stage[e * kPrefixThreads + threadIdx.x];
}

// The first j with incl[j] > t (t < S): down the tree, one row of kFan sums
// per level.
__device__ __forceinline__ uint32_t descend(const PrefixJob& J, uint64_t t)
{
    uint64_t g = 0;
    for (int k = J.top; k >= 0; --k) {
        const uint64_t* row = at<uint64_t>(J, k ? J.o_level[k] : J.o_incl) + g * kFan;
        uint64_t v[kFan];
#pragma unroll
        for (uint32_t m = 0; m < kFan; m += 2) {
            const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(row + m);
            v[m] = x.x;
            v[m + 1] = x.y;
        }
        uint32_t c = 0;
#pragma unroll
        for (uint32_t m = 0; m < kFan; ++m) c += v[m] <= t ? 1u : 0u;
        g = g * kFan + c;
    }
    return (uint32_t)g;
}

// The first j in [lo, lo + len) with a[j] > t, given a[lo + len - 1] > t.
__device__ __forceinline__ uint32_t first_above(const uint64_t* __restrict__ a, uint32_t lo, uint32_t len, uint64_t t)
{
    while (len > 1u) {
        const uint32_t half = len / 2u;
        lo = a[lo + half - 1u] <= t ? lo + half : lo;  // [lo, lo + half) all <= t: skip them
        len -= half;
    }
    return lo;
}

// The threshold of output i of run r in [0, S).
template <int Method>
__device__ __forceinline__ uint64_t prefix_threshold(const PrefixJob& J, uint64_t S, uint32_t i)
{
    const uint32_t sid = J.stream0 + blockIdx.y;
    if constexpr (Method == MGP_MULTINOMIAL) {
        // Algorithm 7: u ~ U[0, S), one 64-bit draw per output
        const Words x = philox(0u, kTagMultinomial, sid, i, J.key0, J.key1);
        const uint64_t r = (uint64_t)x.x0 | ((uint64_t)x.x1 << 32);
        return __umul64hi(r, S);
    } else {
        // Algorithm 8: u = (i + u_t) / N after one draw u_t ~ U[0, 1), in fp64
        // with each operation rounded once
        const Words x = philox(0u, kTagSystematic, sid, 0u, J.key0, J.key1);
        const uint64_t r = (uint64_t)x.x0 | ((uint64_t)x.x1 << 32);
        const double ut = (double)(r >> 11) * 0x1p-53;
        const double c = __ddiv_rn((double)S, (double)J.n);
        const double v = __dmul_rn(__dadd_rn((double)i, ut), c);
        const uint64_t t = (uint64_t)floor(v);
        return t < S ? t : S - 1u;
    }
}

// Output i of run r: the ancestor and, when the job copies rows, the row
// (a NaN row for invalid weights, a = -1).
__device__ __forceinline__ void emit(const PrefixJob& J, uint32_t i, int32_t a)
{
    const uint64_t r = blockIdx.y;
    if (J.anc) J.anc[r * J.anc_ld + i] = a;
    if (J.states) {
        const RowCopy rc{J.states + r * J.rows_ld, J.out + r * J.rows_ld, J.d, J.vec4};
        copy_row(rc, i, a);
    }
}

// Multinomial: the descents of a wave's 64 outputs, eight lanes to a row.
// A lane that read a whole 128-byte row by itself would make each load
// instruction of the wave touch 64 lines, and the address path, not the
// memory, would bound the kernel. Here the lanes of an octet (8 lanes) read
// the 16-byte quarters of one row together, so an instruction touches 8
// lines: lane l serves outputs r*8 + l/8 (r = 0..7) of the wave, reading
// their rows' quarter l mod 8, and the octet adds up its counts. Lane l draws
// the threshold of output l, and gets back the ancestor of output l, by
// cross-lane permutes. Every lane of the wave runs to the end (outputs past n
// search too, and are not stored).
__global__ __launch_bounds__(kPrefixThreads) void k_prefix_multinomial(PrefixJob J)
{
    constexpr uint32_t kOct = 8;  // lanes per row; also the outputs per lane
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t i = blockIdx.x * kPrefixThreads + threadIdx.x;
    const PrefixHeader h = *at<PrefixHeader>(J, J.o_hdr);
    if (!h.valid) {
        if (i < J.n) emit(J, i, -1);
        return;
    }
    const uint64_t t_mine = prefix_threshold<MGP_MULTINOMIAL>(J, h.total, i < J.n ? i : J.n - 1u);
    const uint32_t oct = lane / kOct, quarter = lane % kOct;
    uint64_t t[kOct];
    uint32_t g[kOct];
#pragma unroll
    for (uint32_t r = 0; r < kOct; ++r) {
        const int src = (int)(r * kOct + oct);
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)t_mine, src, 64);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(t_mine >> 32), src, 64);
        t[r] = (uint64_t)lo | ((uint64_t)hi << 32);
        g[r] = 0u;
    }
    for (int k = J.top; k >= 0; --k) {
        const uint64_t* lv = at<uint64_t>(J, k ? J.o_level[k] : J.o_incl) + quarter * 2u;
        ulonglong2 v[kOct];
#pragma unroll
        for (uint32_t r = 0; r < kOct; ++r) v[r] = *reinterpret_cast<const ulonglong2*>(lv + (uint64_t)g[r] * kFan);
        // counts of up to 16 per row, one byte each: outputs 0-3 in c0, 4-7 in c1
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (uint32_t r = 0; r < kOct; ++r) {
            const uint32_t c = (v[r].x <= t[r] ? 1u : 0u) + (v[r].y <= t[r] ? 1u : 0u);
            if (r < 4) c0 |= c << (8u * r);
            else c1 |= c << (8u * (r - 4u));
        }
#pragma unroll
        for (int off = 1; off < (int)kOct; off <<= 1) {
            c0 += (uint32_t)__shfl_xor((int)c0, off, 64);
            c1 += (uint32_t)__shfl_xor((int)c1, off, 64);
        }
#pragma unroll
        for (uint32_t r = 0; r < kOct; ++r)
            g[r] = g[r] * kFan + (((r < 4 ? c0 : c1) >> (8u * (r % 4u))) & 0xFFu);
    }
    // output l's ancestor is g[l / 8] of the octet l mod 8
    uint32_t a = 0;
#pragma unroll
    for (uint32_t r = 0; r < kOct; ++r) {
        const uint32_t x = (uint32_t)__shfl((int)g[r], (int)((lane % kOct) * kOct), 64);
        if (lane / kOct == r) a = x;
    }
    if (i < J.n) emit(J, i, (int32_t)a);
}

// Systematic, first pass: the ancestors of outputs 0, G, 2G, ... (G =
// kPrefixThreads) and n - 1, which bracket those of every output between.
__global__ __launch_bounds__(kPrefixThreads) void k_prefix_brackets(PrefixJob J, uint32_t nb)
{
    const uint32_t b = blockIdx.x * kPrefixThreads + threadIdx.x;
    const PrefixHeader h = *at<PrefixHeader>(J, J.o_hdr);
    if (b > nb || !h.valid) return;
    const uint32_t i = b < nb ? b * kPrefixThreads : J.n - 1u;
    at<uint32_t>(J, J.o_bracket)[b] = descend(J, prefix_threshold<MGP_SYSTEMATIC>(J, h.total, i));
}

// Systematic, second pass: output i's ancestor lies between the brackets of
// its group of G outputs (the thresholds, and so the ancestors, rise with
// i). When the bracketed sums fit kStageMax entries the block reads them into
// LDS once (coalesced) and bisects there; otherwise each lane bisects in
// memory.
constexpr uint32_t kStageMax = 2048;

__global__ __launch_bounds__(kPrefixThreads) void k_prefix_systematic(PrefixJob J)
{
    __shared__ uint64_t stage[kStageMax];
    const uint32_t i = blockIdx.x * kPrefixThreads + threadIdx.x;
    const PrefixHeader h = *at<PrefixHeader>(J, J.o_hdr);
    if (!h.valid) {
        if (i < J.n) emit(J, i, -1);
        return;
    }
    const uint32_t* bracket = at<uint32_t>(J, J.o_bracket);
    const uint64_t* incl = at<uint64_t>(J, J.o_incl);
    const uint32_t lo = bracket[blockIdx.x], hi = bracket[blockIdx.x + 1u];
    const uint32_t len = hi - lo + 1u;
    const uint64_t t = prefix_threshold<MGP_SYSTEMATIC>(J, h.total, i < J.n ? i : J.n - 1u);
    if (len <= kStageMax) {  // the same for every lane of the block
        for (uint32_t k = threadIdx.x; k < len; k += kPrefixThreads) stage[k] = incl[lo + k];
        __syncthreads();
        if (i < J.n) emit(J, i, (int32_t)(lo + first_above(stage, 0u, len, t)));
    } else if (i < J.n) {
        emit(J, i, (int32_t)first_above(incl, lo, len, t));
    }
}

static uint64_t align256(uint64_t b) { return (b + 255u) & ~(uint64_t)255u; }

// The layout of one run's scan region: [header][chunk sums][chunk exclusive
// sums][brackets][tree levels 1..top][level 0: the inclusive sums, whole
// chunks]. Returns the region's size.
uint64_t prefix_region(uint32_t n, PrefixJob* J)
{
    const uint64_t nch = ((uint64_t)n + kChunk - 1u) / kChunk;
    uint64_t o = 0;
    J->o_hdr = o;
    o += 256u;
    J->o_sum = o;
    o += align256(nch * 8u);
    J->o_excl = o;
    o += align256(nch * 8u);
    J->o_bracket = o;
    o += align256(((uint64_t)n / kPrefixThreads + 2u) * 4u);
    // level k has ceil(n / 16^k) real entries; the top is the first with <= 16
    uint64_t cnt = n;
    J->top = 0;
    while (cnt > kFan) {
        cnt = (cnt + kFan - 1u) / kFan;
        ++J->top;
        J->count[J->top] = (uint32_t)cnt;
        J->o_level[J->top] = o;
        o += align256((cnt + kFan - 1u) / kFan * kFan * 8u);
    }
    J->o_incl = o;
    o += align256(nch * kChunk * 8u);
    J->n = n;
    J->nch = (uint32_t)nch;
    int L = 0;
    while (((uint64_t)1 << L) < (uint64_t)n) ++L;
    J->log2n = L;
    return o;
}

// Enqueues the scan and search of a job whose stats (validation, max) are
// already on the device: R runs, method MGP_MULTINOMIAL or MGP_SYSTEMATIC.
int enqueue_prefix(const PrefixJob& J, uint32_t R, int method, hipStream_t s)
{
    const dim3 chunks(J.nch, R);
    hipLaunchKernelGGL(k_prefix_chunks, chunks, dim3(kPrefixThreads), 0, s, J);
    hipLaunchKernelGGL(k_prefix_top, dim3(1, R), dim3(kPrefixThreads), 0, s, J);
    hipLaunchKernelGGL(k_prefix_scan, chunks, dim3(kPrefixThreads), 0, s, J);
    int err = check_launch("prefix-sum kernels");
    if (err) return err;
    const uint32_t nb = (J.n + kPrefixThreads - 1u) / kPrefixThreads;  // groups of outputs
    if (method == MGP_MULTINOMIAL) {
        hipLaunchKernelGGL(k_prefix_multinomial, dim3(nb, R), dim3(kPrefixThreads), 0, s, J);
    } else {
        hipLaunchKernelGGL(k_prefix_brackets, dim3(nb / kPrefixThreads + 1u, R), dim3(kPrefixThreads), 0, s, J, nb);
        hipLaunchKernelGGL(k_prefix_systematic, dim3(nb, R), dim3(kPrefixThreads), 0, s, J);
    }
    return check_launch("prefix-sum search kernel");
}

}  // namespace mgp

using namespace mgp;

extern "C" {

int mgp_prefix_workspace_size(int32_t n, size_t* bytes)
{
    clear_error();
    if (!bytes) return fail(MGP_EINVAL, "bytes is NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    PrefixJob J{};
    *bytes = workspace_bytes(1u) + prefix_region((uint32_t)n, &J);
    return MGP_OK;
}

int mgp_resample_prefix(const float* w_dev, int32_t n, int32_t method, uint64_t seed, uint32_t stream_id,
                        int32_t* ancestors_dev, mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes_,
                        void* stream)
{
    clear_error();
    if (!w_dev || !ancestors_dev) return fail(MGP_EINVAL, "w_dev and ancestors_dev must not be NULL");
    if (n < 1) return fail(MGP_EINVAL, "n must be >= 1 (got %d)", n);
    if (method != MGP_MULTINOMIAL && method != MGP_SYSTEMATIC)
        return fail(MGP_EINVAL, "unknown prefix-sum method %d", method);
    if (!workspace_dev) return fail(MGP_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace_dev & 255u) != 0) return fail(MGP_EINVAL, "workspace must be 256-byte aligned");
    const uint32_t un = (uint32_t)n;
    PrefixJob J{};
    const size_t need = workspace_bytes(1u) + prefix_region(un, &J);
    if (workspace_bytes_ < need) return fail(MGP_ERANGE, "workspace has %zu bytes, needs %zu", workspace_bytes_, need);
    char* ws = static_cast<char*>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // validation, max and fp64 sum: the reduction and finalize step of the
    // other resamplers (one explicit iteration, no offsets, no mirror)
    Params p;
    p.variant = kMetropolis;
    p.B = 1;
    p.eps = 0.5;
    p.seed = seed;
    p.stream_id = stream_id;
    p.partition_bytes = 128;
    p.b_max = 1;
    const int err = enqueue_reduce_finalize(w_dev, un, p, false, ws, stats_dev, s);
    if (err) return err;
    J.w = w_dev;
    J.stats = reinterpret_cast<const mgp_stats*>(ws + kWsStatsOffset);
    J.region = ws + workspace_bytes(1u);
    J.anc = ancestors_dev;
    J.vec = ((uintptr_t)w_dev & 15u) == 0 ? 1u : 0u;
    J.key0 = (uint32_t)seed;
    J.key1 = (uint32_t)(seed >> 32);
    J.stream0 = stream_id;
    return enqueue_prefix(J, 1u, method, s);
}

}  // extern "C"
