// mgp_reduce.h -- device code shared by the single-filter and batched paths:
// the weight reduction (fp32 max, fp64 sum, validation, optional mirror
// write) and the finalize step that turns it into B (eq. (proposition)),
// the stats record and the Megopolis offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mgp.h"
#include "mgp_device.h"
#include "mgp_internal.h"

namespace mgp {

__device__ __forceinline__ void fold(float v, float& mx, double& s, uint32_t& bad)
{
    bad |= (!(v >= 0.0f) || v == INFINITY) ? 1u : 0u;
    mx = fmaxf(mx, v);
    s += (double)v;
}

// Block-wide reduction of (max, sum, bad); result valid in thread 0.
__device__ __forceinline__ void block_reduce(float& mx, double& s, uint32_t& bad)
{
    __shared__ float smx[kReduceThreads / 64];
    __shared__ double ssum[kReduceThreads / 64];
    __shared__ uint32_t sbad[kReduceThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        s += __shfl_xor(s, off, 64);
        bad |= __shfl_xor(bad, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        smx[wv] = mx;
        ssum[wv] = s;
        sbad[wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = smx[0];
        s = ssum[0];
        bad = sbad[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            mx = fmaxf(mx, smx[k]);
            s += ssum[k];
            bad |= sbad[k];
        }
    }
}

// Reduces w[start, end) into (mx, s, bad) per thread and, with a mirror,
// writes M[i] = M[i + n] = w[i] for the range. With Vec, w + start is
// 16-byte aligned and (with a mirror) n % 4 == 0.
template <bool Vec>
__device__ __forceinline__ void reduce_range(const float* __restrict__ w, uint32_t n, uint64_t start, uint64_t end,
                                             float* __restrict__ mirror, float& mx, double& s, uint32_t& bad)
{
    if constexpr (Vec) {
        const uint64_t end4 = start + ((end - start) & ~(uint64_t)3);
        for (uint64_t i = start + 4ull * threadIdx.x; i < end4; i += 4ull * blockDim.x) {
            const float4 v = *reinterpret_cast<const float4*>(w + i);
            if (mirror) {
                *reinterpret_cast<float4*>(mirror + i) = v;
                *reinterpret_cast<float4*>(mirror + n + i) = v;
            }
            fold(v.x, mx, s, bad);
            fold(v.y, mx, s, bad);
            fold(v.z, mx, s, bad);
            fold(v.w, mx, s, bad);
        }
        for (uint64_t i = end4 + threadIdx.x; i < end; i += blockDim.x) {
            const float v = w[i];
            if (mirror) {
                mirror[i] = v;
                mirror[n + i] = v;
            }
            fold(v, mx, s, bad);
        }
    } else {
        for (uint64_t i = start + threadIdx.x; i < end; i += blockDim.x) {
            const float v = w[i];
            if (mirror) {
                mirror[i] = v;
                mirror[n + i] = v;
            }
            fold(v, mx, s, bad);
        }
    }
}

// The padding M[2n + k] = w[k mod n], k < kMirrorPad (one block writes it).
__device__ __forceinline__ void mirror_pad(const float* __restrict__ w, uint32_t n, float* __restrict__ mirror)
{
    for (uint32_t k = threadIdx.x; k < kMirrorPad; k += blockDim.x) mirror[2ull * n + k] = w[k % n];
}

// ---------------------------------------------------------------------------
// 2. Finalize: combine the partials, pick B by eq. (proposition), write the
//    stats, and generate the Megopolis offsets o_0..o_{B-1} (Algorithm 5's
//    offsets are drawn before the particle loop; here in parallel, four per
//    Philox call).
// ---------------------------------------------------------------------------
// Returns B (0 for invalid weights) in every thread.
__device__ __forceinline__ uint32_t finalize_one(const Partial* __restrict__ part, uint32_t nparts, const FinalizeArgs& a,
                             mgp_stats* __restrict__ st, mgp_stats* __restrict__ st_user,
                             uint32_t* __restrict__ offsets)
{
    __shared__ uint32_t sB;
    float mx = 0.0f;
    double s = 0.0;
    uint32_t bad = 0;
    for (uint32_t p = threadIdx.x; p < nparts; p += blockDim.x) {
        const Partial q = part[p];
        mx = fmaxf(mx, q.w_max);
        s += q.w_sum;
        bad |= q.bad;
    }
    block_reduce(mx, s, bad);
    if (threadIdx.x == 0) {
        mgp_stats r;
        r.w_sum = s;
        r.w_max = mx;
        r.n = a.n;
        r.clamped = 0;
        r.tag = a.tag;
        r.ratio = 0.0;
        r.b_raw = 0.0;
        if (bad || !(mx > 0.0f)) {
            r.status = MGP_EWEIGHTS;
            r.B = 0;
        } else {
            r.status = MGP_OK;
            const double mean = s / (double)a.n;
            const double ratio = mean / (double)mx;
            r.ratio = ratio;
            if (a.B_user > 0) {
                r.B = a.B_user;
            } else {
                const double raw = ratio >= 1.0 ? 1.0 : log(a.eps) / log1p(-ratio);
                r.b_raw = raw;
                double c = ceil(raw);
                if (c < 1.0) c = 1.0;
                if (c > (double)a.b_max) {
                    c = (double)a.b_max;
                    r.clamped = 1;
                }
                r.B = (uint32_t)c;
            }
        }
        *st = r;
        if (st_user) *st_user = r;
        sB = r.B;
    }
    __syncthreads();
    const uint32_t B = sB;
    if (a.make_offsets && B > 0) {
        const uint32_t calls = (B + 3u) / 4u;
        for (uint32_t c = threadIdx.x; c < calls; c += blockDim.x) {
            const Words x = philox(c, kTagOffset, a.stream_id, 0u, a.key0, a.key1);
            const uint32_t o[4] = {x.x0, x.x1, x.x2, x.x3};
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                const uint32_t b = 4u * c + r;
                if (b < B) offsets[b] = uniform_index(o[r], a.n);
            }
        }
    }
    return B;
}

}  // namespace mgp
