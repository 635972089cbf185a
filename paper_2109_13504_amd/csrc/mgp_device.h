// mgp_device.h -- device-side building blocks of the resampling kernels for
// gfx950: the counter-based generator, the u and index maps, the candidate
// index of each variant, and the accept loop of one particle.
//
// Definitions (Algorithms 2-5 of "The Megopolis Resampler", arXiv 2109.13504):
//   - particle i starts at k = i and runs B steps; at step b a candidate j is
//     drawn and accepted when u * w_k <= w_j (the ratio test u <= w_j / w_k in
//     product form, evaluated in fp32, ties accept);
//   - Metropolis: j ~ U{0, N-1}; C1: j uniform in the partition the particle's
//     32-group drew once; C2: the group redraws its partition every step;
//     Megopolis: j = (i - i mod 32 + o_b - o_b mod 32 + (i + o_b) mod 32) mod N
//     with offsets o_b shared by every particle.
// Random streams: Philox4x32-10 (Salmon et al., SC'11), key = seed,
// counter = (block, tag, stream_id, index). The per-particle index sits in the
// last counter word so that the first round is wave-uniform (scalar unit)
// and rounds 2 and 3 carry one uniform multiply each.
//   tag 0: u, index i, block b/5, five u per call
//   tag 1: j, index i, block b/4, word b%4
//   tag 2: Megopolis offsets, index 0, block b/4, word b%4
//   tag 3: C1 partition, index i/32, block 0, word 0
//   tag 4: C2 partition, index i/32, block b/4, word b%4
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mgp {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

constexpr uint32_t kTagU = 0u;
constexpr uint32_t kTagJ = 1u;
constexpr uint32_t kTagOffset = 2u;
constexpr uint32_t kTagC1Part = 3u;
constexpr uint32_t kTagC2Part = 4u;

constexpr int kMetropolis = 0;
constexpr int kC1 = 1;
constexpr int kC2 = 2;
constexpr int kMegopolis = 3;

constexpr uint32_t kSegment = 32u;  // weights per wrapped segment (the paper's warp width)

struct Words {
    uint32_t x0, x1, x2, x3;
};

// a ^ b ^ c in one VALU instruction (gfx950 three-input bitwise op, truth
// table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 on counter (c0, c1, c2, c3) with key (k0, k1). Each round
// takes both 32x32 -> 64-bit products as one v_mad_u64_u32 each. With the
// per-lane index in c3 and the other words wave-uniform, rounds 1-3 still
// hold uniform values that the compiler keeps on the scalar unit, so those
// use plain xors; from round 4 on every word is per lane and each pair of
// xors is one three-input op.
__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0, n2;
        if (r < 3) {
            n0 = hi1 ^ c1 ^ k0;
            n2 = hi0 ^ c3 ^ k1;
        } else {
            n0 = xor3(hi1, c1, k0);
            n2 = xor3(hi0, c3, k1);
        }
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Words{c0, c1, c2, c3};
}

// U{0, n-1} from a 32-bit word: floor(x * n / 2^32).
__device__ __forceinline__ uint32_t uniform_index(uint32_t x, uint32_t n) { return __umulhi(x, n); }

// u = (m + 1) 2^-24 for a 24-bit m; m 2^-24 + 2^-24 is exact, so the fused
// multiply-add rounds nothing.
__device__ __forceinline__ float u_from_bits(uint32_t m) { return __fmaf_rn((float)m, 0x1p-24f, 0x1p-24f); }

// The five u of one tag-0 call.
struct UBlock {
    float u[5];
};

__device__ __forceinline__ UBlock u_block(const Words& x)
{
    UBlock r;
    r.u[0] = u_from_bits(x.x0 >> 8);
    r.u[1] = u_from_bits(x.x1 >> 8);
    r.u[2] = u_from_bits(x.x2 >> 8);
    r.u[3] = u_from_bits(x.x3 >> 8);
    r.u[4] = u_from_bits((x.x0 & 0xFFu) | ((x.x1 & 0xFFu) << 8) | ((x.x2 & 0xFFu) << 16));
    return r;
}

__device__ __forceinline__ uint32_t word(const Words& x, uint32_t r)
{
    return r == 0 ? x.x0 : r == 1 ? x.x1 : r == 2 ? x.x2 : x.x3;
}

// Megopolis candidate: aligned segment of i plus aligned part of o, rotated by
// (i + o) mod S inside the segment (S = seg_mask + 1, 32 or 64, a wave-uniform
// value); the sum is <= i + o <= 2N - 2, so one
// conditional subtraction is the mod N. min(j, j - n) in unsigned arithmetic
// picks j - n exactly when j >= n (n <= 2^31).
__device__ __forceinline__ uint32_t megopolis_index(uint32_t i_aligned, uint32_t i_low, uint32_t o, uint32_t n,
                                                    uint32_t seg_mask)
{
    const uint32_t j = i_aligned + (o & ~seg_mask) + ((i_low + o) & seg_mask);
    const uint32_t jm = j - n;
    return jm < j ? jm : j;
}

// C1/C2 candidate inside partition p of n_w weights (the last one cut at n).
__device__ __forceinline__ uint32_t partition_index(uint32_t p, uint32_t jword, uint32_t n, uint32_t n_w)
{
    const uint32_t start = p * n_w;
    const uint32_t rest = n - start;
    const uint32_t width = rest < n_w ? rest : n_w;
    return start + uniform_index(jword, width);
}

// Loads w[j]. With `Narrow` the byte offset fits 32 bits (n <= 2^30), which
// lets the compiler use the scalar-base + 32-bit vector-offset form.
template <bool Narrow>
__device__ __forceinline__ float load_weight(const float* __restrict__ w, uint32_t j)
{
    if constexpr (Narrow) {
        return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(w) + (j << 2));
    } else {
        return w[(size_t)j];
    }
}

// Per-call parameters of the accept loop (all wave-uniform).
struct LoopParams {
    const float* w;
    const uint32_t* offsets;  // Megopolis offsets o_0..o_{B-1}, each < n
    uint32_t n;
    uint32_t B;
    uint32_t key0, key1;
    uint32_t stream_id;
    uint32_t n_w;     // C1/C2: weights per partition
    uint32_t n_part;  // C1/C2: number of partitions, ceil(n / n_w)
    uint32_t seg_mask = kSegment - 1u;  // Megopolis: segment width - 1
};

// o_b, clamped below n so that a workspace not written by this call's
// reduction can never steer a load out of bounds (wave-uniform, scalar unit).
__device__ __forceinline__ uint32_t offset_at(const LoopParams& P, uint32_t b)
{
    const uint32_t o = P.offsets[b];
    return o < P.n ? o : P.n - 1u;
}

// Steps per unrolled block: Megopolis needs only the 5-step u blocks; the
// others also use 4-step j blocks, so they unroll over lcm(4, 5) = 20.
template <int V>
struct Unroll {
    static constexpr uint32_t value = (V == kMegopolis) ? 5u : 20u;
};

// What a chain carries from block to block, and what is fixed for it.
struct ChainState {
    uint32_t k;  // current ancestor
    float wk;    // its weight
};

struct ChainFixed {
    uint32_t i;          // particle (random draws, C1/C2 group)
    uint32_t group;      // i / 32
    uint32_t i_aligned;  // Megopolis: segment base of the start position
    uint32_t i_low;      // Megopolis: place of the start position in its segment
    uint32_t c1_part;    // C1: the group's partition
};

// The particle index as an opaque value: an empty volatile asm statement
// that the compiler may not move out of the branch it sits in, so that a
// generator call taking its result stays behind that branch's test instead
// of being computed ahead of it for steps that do not run. No instruction
// is emitted.
__device__ __forceinline__ uint32_t pinned(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Steps q U .. q U + cnt - 1 of a chain (cnt = U for a whole block; the last
// block of B mod U steps passes Partial and its count). The candidates and
// their weights come first: they do not depend on the chain, so all of the
// block's loads are in flight together; then the serial accept steps.
// Partial skips the steps past cnt (cnt is wave-uniform), including their
// generator calls and loads.
template <int V, bool Narrow, bool Shared, bool Partial>
__device__ __forceinline__ void chain_block(const LoopParams& P, const ChainFixed& F, uint32_t q, uint32_t cnt,
                                            ChainState& c)
{
    constexpr uint32_t U = Unroll<V>::value;
    constexpr bool kShare = Shared && V == kC2;
    const float* __restrict__ w = P.w;
    UBlock ub;
    Words jb{}, pb{}, pmine{};
    uint32_t jj[U];
    float wj[U];
    if constexpr (kShare) {
        // lane k (< U / 4) of the half-wave: the call of block q U / 4 + k
        const uint32_t k = __lane_id() & 31u;
        pmine = philox(q * (U / 4) + (k < U / 4 ? k : 0u), kTagC2Part, P.stream_id, F.group, P.key0, P.key1);
    }
#pragma unroll
    for (uint32_t s = 0; s < U; ++s) {
        if (Partial && s >= cnt) continue;
        const uint32_t b = q * U + s;
        uint32_t j;
        if constexpr (V == kMegopolis) {
            j = megopolis_index(F.i_aligned, F.i_low, offset_at(P, b), P.n, P.seg_mask);
        } else {
            if (s % 4 == 0) {
                const uint32_t blk = q * (U / 4) + s / 4;
                const uint32_t pi = Partial ? pinned(F.i) : F.i;
                jb = philox(blk, kTagJ, P.stream_id, pi, P.key0, P.key1);
                if constexpr (V == kC2 && !kShare) {
                    const uint32_t pg = Partial ? pinned(F.group) : F.group;
                    pb = philox(blk, kTagC2Part, P.stream_id, pg, P.key0, P.key1);
                }
            }
            const uint32_t jw = word(jb, s % 4);
            if constexpr (V == kMetropolis) {
                j = uniform_index(jw, P.n);
            } else if constexpr (V == kC1) {
                j = partition_index(F.c1_part, jw, P.n, P.n_w);
            } else {
                uint32_t pw;
                if constexpr (kShare)
                    pw = (uint32_t)__shfl((int)word(pmine, s % 4), (int)((__lane_id() & 32u) + s / 4), 64);
                else
                    pw = word(pb, s % 4);
                j = partition_index(uniform_index(pw, P.n_part), jw, P.n, P.n_w);
            }
        }
        jj[s] = j;
        wj[s] = load_weight<Narrow>(w, j);
    }
#pragma unroll
    for (uint32_t s = 0; s < U; ++s) {
        if (Partial && s >= cnt) continue;
        if (s % 5 == 0) {
            const uint32_t pi = Partial ? pinned(F.i) : F.i;
            ub = u_block(philox(q * (U / 5) + s / 5, kTagU, P.stream_id, pi, P.key0, P.key1));
        }
        const float p = ub.u[s % 5] * c.wk;
        const bool acc = p <= wj[s];
        c.k = acc ? jj[s] : c.k;
        c.wk = acc ? wj[s] : c.wk;
    }
}

// The B-step chain of particle i; returns its ancestor. The chain starts at
// input position pos (i itself when inputs and outputs are the same
// particles, i mod n for M != N resampling): the Megopolis segment
// arithmetic uses pos, the random draws and the C1/C2 group use i. The steps
// run in blocks of U (Unroll), the last B mod U of them as one partial block.
// Shared (C2 only): every lane of the wave runs a chain, and the 32 lanes of
// each half-wave hold the 32 particles of one group (i - lane a multiple of
// 32 within the half-wave). The group's partition draw of each step is the
// same for its 32 particles, so instead of each lane calling the generator
// once per four steps, lane k of the half-wave makes the call of the k-th
// four-step block of the block's twenty steps and the others read its words
// with a cross-lane permute: one call per lane per twenty steps.
template <int V, bool Narrow, bool Shared = false>
__device__ __forceinline__ uint32_t run_chain(const LoopParams& P, uint32_t i, uint32_t pos)
{
    ChainFixed F;
    F.i = i;
    F.group = i / kSegment;
    F.i_aligned = pos & ~P.seg_mask;
    F.i_low = pos & P.seg_mask;
    F.c1_part = 0;
    if constexpr (V == kC1) {
        const Words px = philox(0u, kTagC1Part, P.stream_id, F.group, P.key0, P.key1);
        F.c1_part = uniform_index(px.x0, P.n_part);
    }
    ChainState c{pos, load_weight<Narrow>(P.w, pos)};
    constexpr uint32_t U = Unroll<V>::value;
    const uint32_t nblk = P.B / U;
    for (uint32_t q = 0; q < nblk; ++q) chain_block<V, Narrow, Shared, false>(P, F, q, U, c);
    const uint32_t rest = P.B - nblk * U;
    if (rest) chain_block<V, Narrow, Shared, true>(P, F, nblk, rest, c);
    return c.k;
}

template <int V, bool Narrow, bool Shared = false>
__device__ __forceinline__ uint32_t run_chain(const LoopParams& P, uint32_t i)
{
    return run_chain<V, Narrow, Shared>(P, i, i);
}

// ---------------------------------------------------------------------------
// Megopolis over a mirrored weight array.
//
// M[k] = w[k mod n] for k < 2n + kMirrorPad. The candidate of Algorithm 5,
// (i_aligned + o_aligned + (i + o) mod 32) mod N, is then simply
// M[i_aligned + o_aligned + (i + o) mod 32]: the sum is at most 2n - 2 for a
// real particle, so the mod N moves from every load to the one final
// ancestor. Each thread carries P particles i0 + BT p (BT = block size);
// they share i mod 32, so all P candidates of a step are the slot-0
// candidate plus BT p, and the P loads differ only in their immediate byte
// offset (4 BT p). The segment width S = seg_mask + 1 (32 or 64) divides BT,
// so the P particles of a thread also share i mod S.
// Byte offsets must fit 32 bits: 4 (2n + kMirrorPad) < 2^32.
// ---------------------------------------------------------------------------
constexpr uint32_t kMirrorPad = 2048;             // >= 256 P + 32 for P <= 4
constexpr uint32_t kMirrorMaxN = (1u << 29) - 4096;

template <int P, int BT = 256>
__device__ __forceinline__ void megopolis_mirror_chain(const char* __restrict__ M, const uint32_t* __restrict__ offs,
                                                       uint32_t n, uint32_t B, uint32_t key0, uint32_t key1,
                                                       uint32_t stream_id, uint32_t i0, uint32_t (&anc_out)[P],
                                                       uint32_t seg_mask = kSegment - 1u)
{
    static_assert(BT % 64 == 0 && BT * P + 64 <= kMirrorPad, "particles of a thread must fit the padding");
    static_assert(4 * BT * (P - 1) < 4096, "the immediate offset of the last particle must fit 12 bits");
    constexpr uint32_t kStrideBytes = 4u * BT;  // particle p sits BT particles after p - 1
    const uint32_t ia4 = (i0 & ~seg_mask) * 4u;
    const uint32_t il4 = (i0 & seg_mask) * 4u;
    uint32_t kk[P];  // ancestor as the slot-0 byte offset into M
    float wk[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        kk[p] = i0 * 4u;
        wk[p] = *reinterpret_cast<const float*>(M + i0 * 4u + kStrideBytes * p);
    }
    const uint32_t nblk = B / 5u;
    for (uint32_t q = 0; q < nblk; ++q) {
        uint32_t jb[5];
        float wj[5][P];
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s) {
            uint32_t o = offs[q * 5u + s];
            o = o < n ? o : n - 1u;
            const uint32_t oa4 = (o & ~seg_mask) * 4u;
            const uint32_t t4 = (il4 + (o & seg_mask) * 4u) & (seg_mask * 4u);
            const uint32_t voff = ia4 | t4;
            const char* base = M + oa4;
#pragma unroll
            for (int p = 0; p < P; ++p) wj[s][p] = *reinterpret_cast<const float*>(base + voff + kStrideBytes * p);
            jb[s] = voff + oa4;
        }
        UBlock ub[P];
#pragma unroll
        for (int p = 0; p < P; ++p) ub[p] = u_block(philox(q, kTagU, stream_id, i0 + BT * p, key0, key1));
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float prod = ub[p].u[s] * wk[p];
                const bool acc = prod <= wj[s][p];
                kk[p] = acc ? jb[s] : kk[p];
                wk[p] = acc ? wj[s][p] : wk[p];
            }
        }
    }
    // remaining B mod 5 steps
    if (nblk * 5u < B) {
        UBlock ub[P];
#pragma unroll
        for (int p = 0; p < P; ++p) ub[p] = u_block(philox(nblk, kTagU, stream_id, i0 + BT * p, key0, key1));
        for (uint32_t b = nblk * 5u; b < B; ++b) {
            uint32_t o = offs[b];
            o = o < n ? o : n - 1u;
            const uint32_t oa4 = (o & ~seg_mask) * 4u;
            const uint32_t t4 = (il4 + (o & seg_mask) * 4u) & (seg_mask * 4u);
            const uint32_t voff = ia4 | t4;
            const char* base = M + oa4;
            const uint32_t r = b - nblk * 5u;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float wjv = *reinterpret_cast<const float*>(base + voff + kStrideBytes * p);
                const float u = r == 0 ? ub[p].u[0] : r == 1 ? ub[p].u[1] : r == 2 ? ub[p].u[2] : ub[p].u[3];
                const float prod = u * wk[p];
                const bool acc = prod <= wjv;
                kk[p] = acc ? voff + oa4 : kk[p];
                wk[p] = acc ? wjv : wk[p];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        uint32_t k = kk[p] / 4u + BT * p;
        anc_out[p] = k >= n ? k - n : k;
    }
}

// Megopolis over the mirror, one particle per thread, with the candidate
// weights of D steps (D a multiple of 5) loaded before the first of them is
// used. The candidates do not depend on the accept results, so one round
// trip to memory serves D steps; for small n, where too few waves are in
// flight to hide the latency of the B/5 rounds of the chain above, this cuts
// the number of round trips by D/5. The arithmetic and the random draws are
// those of megopolis_mirror_chain, so the ancestors are identical.
template <int D>
__device__ __forceinline__ uint32_t megopolis_mirror_chain_deep(const char* __restrict__ M,
                                                                const uint32_t* __restrict__ offs, uint32_t n,
                                                                uint32_t B, uint32_t key0, uint32_t key1,
                                                                uint32_t stream_id, uint32_t i, uint32_t seg_mask)
{
    static_assert(D % 5 == 0, "a round covers whole blocks of five u draws");
    const uint32_t ia4 = (i & ~seg_mask) * 4u;
    const uint32_t il4 = (i & seg_mask) * 4u;
    uint32_t kk = i * 4u;
    float wk = *reinterpret_cast<const float*>(M + i * 4u);
    // steps [0, B5) in rounds of D, then whole blocks of 5, then the rest
    const uint32_t nrnd = B / D;
    for (uint32_t q = 0; q < nrnd; ++q) {
        float wj[D];
        uint32_t jb[D];
#pragma unroll
        for (uint32_t s = 0; s < D; ++s) {
            uint32_t o = offs[q * D + s];
            o = o < n ? o : n - 1u;
            const uint32_t oa4 = (o & ~seg_mask) * 4u;
            const uint32_t voff = ia4 | ((il4 + (o & seg_mask) * 4u) & (seg_mask * 4u));
            wj[s] = *reinterpret_cast<const float*>(M + oa4 + voff);
            jb[s] = voff + oa4;
        }
#pragma unroll
        for (uint32_t g = 0; g < D / 5; ++g) {
            const UBlock ub = u_block(philox(q * (D / 5) + g, kTagU, stream_id, i, key0, key1));
#pragma unroll
            for (uint32_t s = 0; s < 5; ++s) {
                const float prod = ub.u[s] * wk;
                const bool acc = prod <= wj[g * 5 + s];
                kk = acc ? jb[g * 5 + s] : kk;
                wk = acc ? wj[g * 5 + s] : wk;
            }
        }
    }
    for (uint32_t b0 = nrnd * D; b0 < B; b0 += 5u) {
        const uint32_t cnt = B - b0 < 5u ? B - b0 : 5u;
        float wj[5];
        uint32_t jb[5];
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s) {
            if (s < cnt) {
                uint32_t o = offs[b0 + s];
                o = o < n ? o : n - 1u;
                const uint32_t oa4 = (o & ~seg_mask) * 4u;
                const uint32_t voff = ia4 | ((il4 + (o & seg_mask) * 4u) & (seg_mask * 4u));
                wj[s] = *reinterpret_cast<const float*>(M + oa4 + voff);
                jb[s] = voff + oa4;
            }
        }
        const UBlock ub = u_block(philox(b0 / 5u, kTagU, stream_id, i, key0, key1));
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s) {
            if (s < cnt) {
                const float prod = ub.u[s] * wk;
                const bool acc = prod <= wj[s];
                kk = acc ? jb[s] : kk;
                wk = acc ? wj[s] : wk;
            }
        }
    }
    const uint32_t k = kk / 4u;
    return k >= n ? k - n : k;
}

// ---------------------------------------------------------------------------
// The particle copy that closes Algorithms 2-5, x_bar_i = x_{k_i}: rows of d
// fp32 states, row-major, streamed to the output past the L2 (written once,
// never read here). The accept loops run it as an epilogue while the
// ancestors are still in registers; the stand-alone gather runs it over an
// ancestor array. A negative ancestor (invalid weights) gives a NaN row.
// ---------------------------------------------------------------------------
struct RowCopy {
    const float* states;  // input rows; null: nothing is copied
    float* out;           // one row per output particle
    uint32_t d;           // floats per row
    uint32_t vec4;        // d % 4 == 0 and both buffers 16-byte aligned: float4 moves
};

__device__ __forceinline__ void store_stream(float4* p, const float4& v)
{
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
}

// Output row i from input row k, one lane, any d: up to four vectors (or
// four floats) loaded before the first of them is stored, so a row of up to
// 16 floats costs one round trip.
__device__ __forceinline__ void copy_row(const RowCopy& g, uint32_t i, int32_t k)
{
    const float4 nan4 = make_float4(NAN, NAN, NAN, NAN);
    const uint64_t kr = k < 0 ? 0u : (uint64_t)k;
    if (g.vec4) {
        const uint32_t d4 = g.d >> 2;
        const float4* src = reinterpret_cast<const float4*>(g.states) + kr * d4;
        float4* dst = reinterpret_cast<float4*>(g.out) + (uint64_t)i * d4;
        for (uint32_t c = 0; c < d4; c += 4u) {
            float4 v[4];
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u)
                if (c + u < d4) v[u] = k < 0 ? nan4 : src[c + u];
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u)
                if (c + u < d4) store_stream(dst + c + u, v[u]);
        }
    } else {
        const float* src = g.states + kr * g.d;
        float* dst = g.out + (uint64_t)i * g.d;
        for (uint32_t c = 0; c < g.d; c += 4u) {
            float v[4];
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u)
                if (c + u < g.d) v[u] = k < 0 ? NAN : src[c + u];
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u)
                if (c + u < g.d) __builtin_nontemporal_store(v[u], dst + c + u);
        }
    }
}

// The rows of P outputs of one lane with D4 float4s per row known at compile
// time (g.vec4 set): every load of the P rows is issued before the first
// store. Outputs with live[p] false are skipped.
template <int P, int D4>
__device__ __forceinline__ void copy_rows_vec4(const RowCopy& g, const uint32_t (&i)[P], const int32_t (&k)[P],
                                               const bool (&live)[P])
{
    const float4* __restrict__ src = reinterpret_cast<const float4*>(g.states);
    float4* __restrict__ dst = reinterpret_cast<float4*>(g.out);
    float4 v[P][D4];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t kr = k[p] < 0 ? 0u : (uint64_t)k[p];
#pragma unroll
        for (int c = 0; c < D4; ++c)
            if (live[p]) v[p][c] = k[p] < 0 ? make_float4(NAN, NAN, NAN, NAN) : src[kr * D4 + c];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int c = 0; c < D4; ++c)
            if (live[p]) store_stream(dst + (uint64_t)i[p] * D4 + c, v[p][c]);
    }
}

}  // namespace mgp
