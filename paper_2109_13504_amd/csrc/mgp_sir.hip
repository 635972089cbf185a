// mgp_sir.hip -- the modified SIR particle filter of Section 7 (Algorithm 6)
// for many independent runs at once (gfx950).
//
// Model, eqs. (predict-end2end) and (update-end2end):
//   x_t = x_{t-1}/2 + 25 x_{t-1} / (1 + x_{t-1}^2) + 8 cos(1.2 t) + v,  v ~ N(0, 10)
//   z_t = x_t^2 / 20 + n,  n ~ N(0, 1)
// and the weight of a particle is the likelihood p(z_t | x_t) without its
// constant factor, exp(-(z_t - x_t^2/20)^2 / 2) (Algorithm 6 drops the
// normalisation because the Metropolis-family resamplers do not need it).
//
// One step of R runs (one filter per run, each n particles) is:
//   stage 1  k_sir_predict_update  one thread per four particles of every
//                                  run; fp64 arithmetic, x and w stored as
//                                  fp32; it also writes the resampler's
//                                  per-block partials and the Megopolis
//                                  mirror (the reduction the batched
//                                  resampler would otherwise run);
//   stage 2  the batched resampler from its finalize step on (B, offsets,
//            validation), then the accept loop with the fused gather
//            x_bar_i = x_{k_i}, one filter per run;
//   stage 3  k_sir_mean_block + k_sir_mean_final: x_hat_t = sum(x_bar) / n
//            in fp64, in a fixed order that depends on n only; in a graph of
//            steps the next step's stage 1 computes the block sums instead.
// The noise v of particle i in run r at step t is sqrt(10) times a standard
// normal from Box-Muller in its two-output form: Philox4x32-10 at counter
// (t, 5, r, floor(i / 4)) under the filter's seed gives two word pairs, pair
// (i / 2) mod 2 serves particles 2 floor(i / 2) (cosine) and its odd
// neighbour (sine). The resample of step t runs under key seed + t * 2^32
// with stream r.
//
// A run whose weights all underflow to zero at some step (its resample
// reports MGP_EWEIGHTS, with -1 ancestors) keeps its predicted particles for
// that step: stage 3 copies them into x_bar, its estimate is their mean, and
// the next prediction starts from them.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "mgp.h"
#include "mgp_batch_internal.h"
#include "mgp_device.h"
#include "mgp_internal.h"
#include "mgp_prefix.h"
#include "mgp_reduce.h"

namespace mgp {

constexpr uint32_t kTagSirNoise = 5u;
constexpr uint32_t kSirThreads = 256;
constexpr uint32_t kRowAlign = 64;     // floats: every run's row starts 256-byte aligned
constexpr double kPi = 3.14159265358979323846;

// Box-Muller in its two-output form for one pair of 32-bit words (a, b):
// u1 = (a + 1) 2^-32 in (0, 1], u2 = b 2^-32 in [0, 1), radius
// sqrt(-2 ln u1); the cosine output goes to the even particle of the pair,
// the sine output to the odd one.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& even, double& odd)
{
    const double u1 = ((double)a + 1.0) * 0x1p-32;
    const double u2 = (double)b * 0x1p-32;
    const double radius = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * kPi * u2, &sn, &cs);
    even = radius * cs;
    odd = radius * sn;
}

// Stage 1 for particles 4m .. 4m+3 of run blockIdx.y, m the thread's global
// index: one Philox call (t, 5, r, m) gives two Box-Muller pairs, one normal
// per particle. The kernel is bound by fp64 VALU issue, so it also does the
// resampler's per-weight work while the weights are in registers: the
// block's partial (fp32 max, fp64 sum, validity) for the finalize step, and
// for Megopolis the mirror M[i] = M[i + n] = w_i (plus M[2n + k] = w_{k mod n}
// for k < kMirrorPad). With mean_part it also writes the block's sum of its
// input particles, the previous step's x_bar, in the order of k_sir_mean_block,
// so that a graph of steps needs no separate pass for stage 3.
__global__ __launch_bounds__(kSirThreads) void k_sir_predict_update(float* __restrict__ xbar, float* x,
                                                                    float* __restrict__ w,
                                                                    const double* __restrict__ z,
                                                                    const mgp_stats* __restrict__ stats,
                                                                    FilterDev* __restrict__ fd,
                                                                    Partial* __restrict__ parts,
                                                                    double* __restrict__ mean_part, uint64_t ld,
                                                                    uint32_t zld, uint32_t n, uint32_t t,
                                                                    double drift, double sigma_v, uint32_t key0,
                                                                    uint32_t key1)
{
    const uint32_t r = blockIdx.y;
    const uint32_t m = blockIdx.x * kSirThreads + threadIdx.x;
    float* mirror = fd[r].mirror;
    const uint32_t part_base = fd[r].part_base;
    // the resample of this step runs under key seed + t * 2^32
    if (blockIdx.x == 0 && threadIdx.x == 0) fd[r].key1 = key1 + t;
    const uint32_t i0 = 4u * m;
    float mx = 0.0f;
    double s = 0.0, prev_sum = 0.0;
    uint32_t bad = 0;
    if (i0 < n) {
        const uint64_t at = (uint64_t)r * ld + i0;  // rows are 256-byte aligned
        const bool full = i0 + 4u <= n;
        // a run whose last resample failed continues from its predicted particles
        const bool failed = stats[r].status != MGP_OK;
        const float* src = failed ? x : xbar;
        float xin[4];
        if (full) {
            const float4 v = *reinterpret_cast<const float4*>(src + at);
            xin[0] = v.x;
            xin[1] = v.y;
            xin[2] = v.z;
            xin[3] = v.w;
        } else {
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) xin[k] = i0 + k < n ? src[at + k] : 0.0f;
        }
        if (mean_part) {
            // the previous step's estimate: its x_bar (x for a failed run,
            // which then also becomes its x_bar), summed as mean_block does
            for (uint32_t k = 0; k < 4 && i0 + k < n; ++k) {
                prev_sum += (double)xin[k];
                if (failed) xbar[at + k] = xin[k];
            }
        }
        const Words q = philox(t, kTagSirNoise, r, m, key0, key1);
        double e[4];
        box_muller(q.x0, q.x1, e[0], e[1]);
        box_muller(q.x2, q.x3, e[2], e[3]);
        const double zt = z[(uint64_t)r * zld + t];
        float xo[4], wo[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const double xp = (double)xin[k];
            const double xn = xp / 2.0 + 25.0 * xp / (1.0 + xp * xp) + drift + sigma_v * e[k];
            xo[k] = (float)xn;
            const double xd = (double)xo[k];
            const double res = zt - xd * xd / 20.0;
            wo[k] = (float)exp(-0.5 * res * res);
        }
        if (full) {
            *reinterpret_cast<float4*>(x + at) = make_float4(xo[0], xo[1], xo[2], xo[3]);
            const float4 w4 = make_float4(wo[0], wo[1], wo[2], wo[3]);
            *reinterpret_cast<float4*>(w + at) = w4;
            if (mirror && (n & 3u) == 0) {
                *reinterpret_cast<float4*>(mirror + i0) = w4;
                *reinterpret_cast<float4*>(mirror + n + i0) = w4;
            } else if (mirror) {
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k) {
                    mirror[i0 + k] = wo[k];
                    mirror[n + i0 + k] = wo[k];
                }
            }
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) fold(wo[k], mx, s, bad);
        } else {
            for (uint32_t k = 0; k < 4 && i0 + k < n; ++k) {
                x[at + k] = xo[k];
                w[at + k] = wo[k];
                if (mirror) {
                    mirror[i0 + k] = wo[k];
                    mirror[n + i0 + k] = wo[k];
                }
                fold(wo[k], mx, s, bad);
            }
        }
        if (mirror && i0 < kMirrorPad) {
            // the padding after the two copies: M[2n + k] = w_{k mod n}
            for (uint32_t k = 0; k < 4 && i0 + k < n; ++k)
                for (uint32_t c = i0 + k; c < kMirrorPad; c += n) mirror[2ull * n + c] = wo[k];
        }
    }
    block_reduce(mx, s, bad);
    if (threadIdx.x == 0) parts[part_base + blockIdx.x] = Partial{s, mx, bad};
    if (mean_part) {
        __syncthreads();  // block_reduce's shared slots are reused
        float dmx = 0.0f;
        uint32_t dbad = 0;
        block_reduce(dmx, prev_sum, dbad);
        if (threadIdx.x == 0) mean_part[(uint64_t)r * gridDim.x + blockIdx.x] = prev_sum;
    }
}

// Stage 3, first pass: the fp64 sum of each group of 1024 particles
// [1024 g, 1024 g + 1024) of run blockIdx.y, four consecutive particles per
// thread in index order, then the block reduction: the decomposition of
// k_sir_predict_update, so that both give the same sums. A block covers
// kMeanGroups groups and issues all their loads before reducing. It sums
// x_bar, or, when that run's resample failed, x, which it then copies into
// x_bar.
constexpr uint32_t kMeanGroups = 8;

__global__ __launch_bounds__(kSirThreads) void k_sir_mean_block(float* __restrict__ xbar,
                                                                const float* __restrict__ x,
                                                                const mgp_stats* __restrict__ stats, uint64_t ld,
                                                                uint32_t n, uint32_t nparts,
                                                                double* __restrict__ partial)
{
    const uint32_t r = blockIdx.y;
    const bool failed = stats[r].status != MGP_OK;
    const float* src = (failed ? x : xbar) + (uint64_t)r * ld;
    float* dst = xbar + (uint64_t)r * ld;
    float v[kMeanGroups][4];
#pragma unroll
    for (uint32_t g = 0; g < kMeanGroups; ++g) {
        const uint32_t i0 = 4u * ((blockIdx.x * kMeanGroups + g) * kSirThreads + threadIdx.x);
        if (i0 + 4u <= n) {
            const float4 q = *reinterpret_cast<const float4*>(src + i0);  // rows are 256-byte aligned
            v[g][0] = q.x;
            v[g][1] = q.y;
            v[g][2] = q.z;
            v[g][3] = q.w;
        } else {
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) v[g][k] = i0 + k < n ? src[i0 + k] : 0.0f;
        }
    }
    for (uint32_t g = 0; g < kMeanGroups; ++g) {
        const uint32_t grp = blockIdx.x * kMeanGroups + g;
        if (grp >= nparts) break;  // uniform across the block
        const uint32_t i0 = 4u * (grp * kSirThreads + threadIdx.x);
        double s = 0.0;
        for (uint32_t k = 0; k < 4 && i0 + k < n; ++k) {
            s += (double)v[g][k];
            if (failed) dst[i0 + k] = v[g][k];
        }
        float mx = 0.0f;
        uint32_t bad = 0;
        block_reduce(mx, s, bad);
        if (threadIdx.x == 0) partial[(uint64_t)r * nparts + grp] = s;
        __syncthreads();  // block_reduce's shared slots are reused by the next group
    }
}

// Stage 3, second pass: x_hat_t = sum / n for run blockIdx.x, plus the B and
// status of that run's resample at step t.
__global__ __launch_bounds__(kReduceThreads) void k_sir_mean_final(const double* __restrict__ partial,
                                                                   uint32_t nparts, uint32_t n,
                                                                   const mgp_stats* __restrict__ stats,
                                                                   double* __restrict__ est,
                                                                   uint32_t* __restrict__ b_hist,
                                                                   int32_t* __restrict__ st_hist, uint32_t T,
                                                                   uint32_t t)
{
    const uint32_t r = blockIdx.x;
    double s = 0.0;
    for (uint32_t c = threadIdx.x; c < nparts; c += kReduceThreads) s += partial[(uint64_t)r * nparts + c];
    float mx = 0.0f;
    uint32_t bad = 0;
    block_reduce(mx, s, bad);
    if (threadIdx.x == 0) {
        const uint64_t at = (uint64_t)r * T + (t - 1);
        est[at] = s / (double)n;
        b_hist[at] = stats[r].B;
        st_hist[at] = stats[r].status;
    }
}

}  // namespace mgp

// ---------------------------------------------------------------------------
// Filter object
// ---------------------------------------------------------------------------
using namespace mgp;

struct mgp_sir_filter {
    mgp_sir_config cfg{};
    int device = 0;
    int nxcd = 1;
    uint32_t n = 0, R = 0, T = 0;
    uint64_t ld = 0;          // row stride (floats) of x, w, x_bar, ancestors
    uint32_t zld = 0;         // T + 1
    uint32_t key0 = 0, key1 = 0;
    double sigma_v = 0.0;
    LoopShape shape{256, 4, 1};
    int prefix_method = -1;   // MGP_MULTINOMIAL or MGP_SYSTEMATIC for a prefix-sum stage 2
    PrefixJob job{};          // its scan regions (one per run) and run strides
    char* dmem = nullptr;
    size_t dmem_bytes = 0;
    float *x = nullptr, *w = nullptr, *xbar = nullptr;
    int32_t* anc = nullptr;
    double* z = nullptr;
    double* est = nullptr;
    uint32_t* b_hist = nullptr;
    int32_t* st_hist = nullptr;
    double* mean_part = nullptr;
    FilterDev* d_fd = nullptr;
    uint32_t nparts = 0;      // stage-1 blocks (and resampler partials) per run
    Partial* d_parts = nullptr;
    mgp_stats* d_stats = nullptr;
    uint32_t* d_qcount = nullptr;
    uint32_t* d_qoff = nullptr;
    LTile* d_lt = nullptr;
    uint32_t grid = 0;
    // host-side order of the stages: step next_t, stage next_stage (1..3);
    // next_t == 0 until the first reset
    uint32_t next_t = 0;
    int next_stage = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(MGP_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

int validate(const mgp_sir_config* c)
{
    if (!c) return fail(MGP_EINVAL, "config is NULL");
    if (c->variant < MGP_METROPOLIS || c->variant > MGP_SIR_SYSTEMATIC)
        return fail(MGP_EINVAL, "unknown variant %d", c->variant);
    const bool prefix = c->variant == MGP_SIR_MULTINOMIAL || c->variant == MGP_SIR_SYSTEMATIC;
    if (c->runs < 1 || c->runs > 65535) return fail(MGP_ERANGE, "runs = %d outside [1, 65535]", c->runs);
    if (c->n < 1 || (uint32_t)c->n > kBatchMaxN) return fail(MGP_ERANGE, "n = %d out of range", c->n);
    if ((uint64_t)c->runs * (uint64_t)c->n > (1ull << 32)) return fail(MGP_ERANGE, "runs * n above 2^32");
    if (c->steps < 1) return fail(MGP_EINVAL, "steps must be >= 1");
    const uint32_t pb = c->partition_bytes ? c->partition_bytes : 128u;
    if (pb < 4u || pb % 4u) return fail(MGP_EINVAL, "partition_bytes must be a positive multiple of 4");
    const uint32_t bmax = c->b_max ? c->b_max : kDefaultBMax;
    if (bmax > kBMaxLimit) return fail(MGP_ERANGE, "b_max above %u", kBMaxLimit);
    if (!prefix && c->B == 0 && (!(c->epsilon > 0.0) || !(c->epsilon <= 1.0)))
        return fail(MGP_EINVAL, "epsilon must be in (0, 1] when B is 0");
    if (!prefix && c->B > bmax) return fail(MGP_ERANGE, "B = %u above b_max = %u", c->B, bmax);
    if (c->reserved || c->reserved2) return fail(MGP_EINVAL, "reserved must be 0");
    if (!prefix && (c->block_threads || c->particles_per_thread)) {
        const LoopShape want{c->block_threads ? c->block_threads : 256,
                             c->particles_per_thread ? c->particles_per_thread : (c->variant == MGP_MEGOPOLIS ? 4 : 1),
                             1};
        if (!batch_shape_supported(c->variant, want))
            return fail(MGP_EINVAL, "unsupported launch shape bt=%d ppt=%d", want.bt, want.ppt);
    }
    return MGP_OK;
}

int check_stage(mgp_sir_filter* f, int32_t t, int stage)
{
    if (f->next_t == 0) return fail(MGP_EINVAL, "the filter has no particles: call mgp_sir_reset first");
    if (t < 1 || (uint32_t)t > f->T) return fail(MGP_ERANGE, "step %d outside [1, %u]", t, f->T);
    if ((uint32_t)t != f->next_t || stage != f->next_stage)
        return fail(MGP_EINVAL, "out of order: step %d stage %d called, step %u stage %d expected", t, stage, f->next_t,
                    f->next_stage);
    return MGP_OK;
}

void advance(mgp_sir_filter* f)
{
    if (++f->next_stage > 3) {
        f->next_stage = 1;
        ++f->next_t;
    }
}

// Stage 1 of step t; with with_mean it also writes the block sums of step
// t - 1's estimate.
int enqueue_predict(mgp_sir_filter* f, uint32_t t, bool with_mean, hipStream_t s)
{
    const double drift = 8.0 * cos(1.2 * (double)t);
    const dim3 grid(f->nparts, f->R);
    hipLaunchKernelGGL(k_sir_predict_update, grid, dim3(kSirThreads), 0, s, f->xbar, f->x, f->w, f->z, f->d_stats,
                       f->d_fd, f->d_parts, with_mean ? f->mean_part : nullptr, f->ld, f->zld, f->n, t, drift,
                       f->sigma_v, f->key0, f->key1);
    return check_launch("SIR predict/update");
}

int enqueue_resample(mgp_sir_filter* f, uint32_t t, hipStream_t s)
{
    if (f->prefix_method >= 0) {
        // stage 1 wrote the partials: the finalize step for each run's stats
        // (validation, max), then the prefix-sum method with the copy
        // x_bar_i = x_{a_i}, under key seed + t 2^32 and stream r
        int rc = enqueue_batch_finalize(f->d_fd, f->R, f->d_parts, f->d_stats, f->d_qcount, s);
        if (rc) return rc;
        PrefixJob J = f->job;
        J.key1 = f->key1 + t;
        return enqueue_prefix(J, f->R, f->prefix_method, s);
    }
    // stage 1 wrote the partials and the mirror: finalize and accept loop only
    return enqueue_batch(f->cfg.variant, f->shape, f->d_fd, f->R, nullptr, 0u, f->d_parts, f->d_stats, f->d_lt,
                         f->grid, f->d_qoff, f->d_qcount, (uint32_t)f->nxcd, 1u, s);
}

// The per-run combine of stage 3 for step t: x_hat_t = (sum of the block
// sums) / n, and the history of B and status.
int enqueue_mean_final(mgp_sir_filter* f, uint32_t t, hipStream_t s)
{
    hipLaunchKernelGGL(k_sir_mean_final, dim3(f->R), dim3(kReduceThreads), 0, s, f->mean_part, f->nparts, f->n,
                       f->d_stats, f->est, f->b_hist, f->st_hist, f->T, t);
    return check_launch("SIR mean (final)");
}

int enqueue_estimate(mgp_sir_filter* f, uint32_t t, hipStream_t s)
{
    const dim3 grid((f->nparts + kMeanGroups - 1) / kMeanGroups, f->R);
    hipLaunchKernelGGL(k_sir_mean_block, grid, dim3(kSirThreads), 0, s, f->xbar, f->x, f->d_stats, f->ld, f->n,
                       f->nparts, f->mean_part);
    int rc = check_launch("SIR mean (block sums)");
    if (rc) return rc;
    return enqueue_mean_final(f, t, s);
}

// Steps 1..T. Stage 1 of step t + 1 reads step t's x_bar anyway, so it also
// produces step t's block sums; the combine for step t then runs before
// step t + 1's resample rewrites the stats. Only step T has a separate pass.
int enqueue_steps(mgp_sir_filter* f, hipStream_t s)
{
    for (uint32_t t = 1; t <= f->T; ++t) {
        int rc = enqueue_predict(f, t, t > 1, s);
        if (!rc && t > 1) rc = enqueue_mean_final(f, t - 1, s);
        if (!rc) rc = enqueue_resample(f, t, s);
        if (rc) return rc;
    }
    return enqueue_estimate(f, f->T, s);
}

int capture(mgp_sir_filter* f)
{
    HIP_TRY(hipStreamBeginCapture(f->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(f, f->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(f->capture_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(MGP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    f->graph = g;
    HIP_TRY(hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0));
    return MGP_OK;
}

void free_filter(mgp_sir_filter* f)
{
    if (!f) return;
    // best-effort teardown: a failure here leaves nothing to recover
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    if (f->capture_stream) (void)hipStreamDestroy(f->capture_stream);
    if (f->dmem) (void)hipFree(f->dmem);
    delete f;
}

}  // namespace

extern "C" {

int mgp_sir_create(const mgp_sir_config* cfg, void* stream, mgp_sir_filter** out)
{
    clear_error();
    if (!out) return fail(MGP_EINVAL, "filter pointer is NULL");
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    mgp_sir_filter* f = new mgp_sir_filter();
    auto bail = [&](int code) {
        free_filter(f);
        return code;
    };
    f->cfg = *cfg;
    f->cfg.partition_bytes = cfg->partition_bytes ? cfg->partition_bytes : 128u;
    f->cfg.b_max = cfg->b_max ? cfg->b_max : kDefaultBMax;
    f->n = (uint32_t)cfg->n;
    f->R = (uint32_t)cfg->runs;
    f->T = (uint32_t)cfg->steps;
    f->zld = f->T + 1;
    f->ld = ((uint64_t)f->n + kRowAlign - 1) / kRowAlign * kRowAlign;
    f->key0 = (uint32_t)cfg->seed;
    f->key1 = (uint32_t)(cfg->seed >> 32);
    f->sigma_v = sqrt(10.0);
    const bool mego = cfg->variant == MGP_MEGOPOLIS;
    const bool prefix = cfg->variant == MGP_SIR_MULTINOMIAL || cfg->variant == MGP_SIR_SYSTEMATIC;
    f->prefix_method = prefix ? (cfg->variant == MGP_SIR_MULTINOMIAL ? MGP_MULTINOMIAL : MGP_SYSTEMATIC) : -1;
    f->shape = LoopShape{cfg->block_threads ? cfg->block_threads : 256,
                         cfg->particles_per_thread ? cfg->particles_per_thread : (mego ? 4 : 1), 1};
    if (hipGetDevice(&f->device) != hipSuccess) return bail(fail(MGP_EHIP, "hipGetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, f->device) != hipSuccess)
        return bail(fail(MGP_EHIP, "hipGetDeviceProperties failed"));
    f->nxcd = (prop.multiProcessorCount >= 64 && prop.multiProcessorCount % kMaxXcd == 0) ? kMaxXcd : 1;

    // ---- accept-loop tiles: R equal filters, XCD-balanced
    const uint32_t B_fixed = prefix ? 1u : cfg->B;  // prefix-sum stage 2: the finalize step only validates
    std::vector<uint32_t> ns(f->R, f->n);
    std::vector<double> cost(f->R, (double)f->n * std::max<uint32_t>(1u, B_fixed ? B_fixed : 32u));
    std::vector<LTile> table;
    std::vector<uint32_t> qoff(kMaxXcd + 1, 0);
    build_tile_table(ns, cost, f->shape, f->nxcd, table, qoff.data());
    if (table.empty()) table.push_back(LTile{kNoFilter, 0});
    f->grid = (uint32_t)table.size();

    // ---- one allocation: particles, weights, histories, resampler tables
    // one partial per stage-1 block of kSirThreads threads x 4 particles
    const uint32_t nparts = (f->n + 4u * kSirThreads - 1u) / (4u * kSirThreads);
    f->nparts = nparts;
    const uint32_t offs_cap = B_fixed ? B_fixed : f->cfg.b_max;
    const size_t rows = (size_t)f->R * f->ld;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t o_x = take(rows * sizeof(float));
    const size_t o_w = take(rows * sizeof(float));
    const size_t o_xbar = take(rows * sizeof(float));
    const size_t o_anc = take(rows * sizeof(int32_t));
    const size_t o_z = take((size_t)f->R * f->zld * sizeof(double));
    const size_t o_est = take((size_t)f->R * f->T * sizeof(double));
    const size_t o_bh = take((size_t)f->R * f->T * sizeof(uint32_t));
    const size_t o_sh = take((size_t)f->R * f->T * sizeof(int32_t));
    const size_t o_mp = take((size_t)f->R * nparts * sizeof(double));
    const size_t o_fd = take((size_t)f->R * sizeof(FilterDev));
    const size_t o_parts = take((size_t)f->R * nparts * sizeof(Partial));
    const size_t o_stats = take((size_t)f->R * sizeof(mgp_stats));
    const size_t o_q = take(sizeof(uint32_t) * 2 * (kMaxXcd + 1));
    const size_t o_lt = take(table.size() * sizeof(LTile));
    const size_t mirror_row = align256(sizeof(float) * (2 * (size_t)f->n + kMirrorPad));
    const size_t offs_row = align256(sizeof(uint32_t) * (size_t)offs_cap);
    const size_t o_offs = mego ? take((size_t)f->R * offs_row) : 0;
    const size_t o_mirror = mego ? take((size_t)f->R * mirror_row) : 0;
    const size_t prefix_row = prefix ? align256(prefix_region(f->n, &f->job)) : 0;
    const size_t o_prefix = prefix ? take((size_t)f->R * prefix_row) : 0;
    f->dmem_bytes = off;
    if (hipMalloc(&f->dmem, f->dmem_bytes) != hipSuccess)
        return bail(fail(MGP_ENOMEM, "could not allocate %zu bytes for the filter", f->dmem_bytes));
    f->x = reinterpret_cast<float*>(f->dmem + o_x);
    f->w = reinterpret_cast<float*>(f->dmem + o_w);
    f->xbar = reinterpret_cast<float*>(f->dmem + o_xbar);
    f->anc = reinterpret_cast<int32_t*>(f->dmem + o_anc);
    f->z = reinterpret_cast<double*>(f->dmem + o_z);
    f->est = reinterpret_cast<double*>(f->dmem + o_est);
    f->b_hist = reinterpret_cast<uint32_t*>(f->dmem + o_bh);
    f->st_hist = reinterpret_cast<int32_t*>(f->dmem + o_sh);
    f->mean_part = reinterpret_cast<double*>(f->dmem + o_mp);
    f->d_fd = reinterpret_cast<FilterDev*>(f->dmem + o_fd);
    f->d_parts = reinterpret_cast<Partial*>(f->dmem + o_parts);
    f->d_stats = reinterpret_cast<mgp_stats*>(f->dmem + o_stats);
    f->d_qcount = reinterpret_cast<uint32_t*>(f->dmem + o_q);
    f->d_qoff = f->d_qcount + (kMaxXcd + 1);
    f->d_lt = reinterpret_cast<LTile*>(f->dmem + o_lt);

    if (prefix) {
        PrefixJob& J = f->job;
        J.w = f->w;
        J.w_ld = f->ld;
        J.stats = f->d_stats;
        J.region = f->dmem + o_prefix;
        J.region_ld = prefix_row;
        J.anc = f->anc;
        J.anc_ld = f->ld;
        J.states = f->x;
        J.out = f->xbar;
        J.rows_ld = f->ld;
        J.d = 1;
        J.vec4 = 0;
        J.vec = 1;  // rows are 256-byte aligned
        J.key0 = f->key0;
        J.key1 = f->key1;
        J.stream0 = 0;
    }
    std::vector<FilterDev> fd(f->R);
    const uint32_t n_w = f->cfg.partition_bytes / 4u;
    for (uint32_t r = 0; r < f->R; ++r) {
        FilterDev& F = fd[r];
        memset(&F, 0, sizeof F);
        F.w = f->w + (size_t)r * f->ld;
        F.anc = f->anc + (size_t)r * f->ld;
        F.states = f->x + (size_t)r * f->ld;
        F.out = f->xbar + (size_t)r * f->ld;
        F.stats_user = nullptr;
        F.mirror = mego ? reinterpret_cast<float*>(f->dmem + o_mirror + (size_t)r * mirror_row) : nullptr;
        F.offsets = mego ? reinterpret_cast<uint32_t*>(f->dmem + o_offs + (size_t)r * offs_row) : nullptr;
        F.eps = cfg->epsilon;
        F.n = f->n;
        F.B_user = B_fixed;
        F.b_max = f->cfg.b_max;
        F.key0 = f->key0;
        F.key1 = f->key1;  // replaced by key1 + t at every step
        F.stream_id = r;
        F.part_base = r * nparts;
        F.nparts = nparts;
        F.chunk = 4u * kSirThreads;
        F.n_w = n_w;
        F.n_part = (uint32_t)(((uint64_t)f->n + n_w - 1u) / n_w);
        F.vec = (!mego || f->n % 4u == 0) ? 1u : 0u;  // rows are 256-byte aligned
        F.rows4 = 0;
    }
    if (hipMemcpyAsync(f->d_fd, fd.data(), fd.size() * sizeof(FilterDev), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f->d_lt, table.data(), table.size() * sizeof(LTile), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f->d_qoff, qoff.data(), qoff.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(f->z, 0, (size_t)f->R * f->zld * sizeof(double), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(MGP_EHIP, "uploading the filter tables failed"));
    if (hipStreamCreateWithFlags(&f->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(MGP_EHIP, "hipStreamCreate failed"));
    if (cfg->use_graph) {
        rc = capture(f);
        if (rc) return bail(rc);
    }
    *out = f;
    return MGP_OK;
}

int mgp_sir_set_measurements(mgp_sir_filter* f, const double* z_host, void* stream)
{
    clear_error();
    if (!f || !z_host) return fail(MGP_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(f->z, z_host, (size_t)f->R * f->zld * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MGP_OK;
}

int mgp_sir_reset(mgp_sir_filter* f, const float* x0_dev, void* stream)
{
    clear_error();
    if (!f || !x0_dev) return fail(MGP_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpy2DAsync(f->xbar, f->ld * sizeof(float), x0_dev, (size_t)f->n * sizeof(float),
                             (size_t)f->n * sizeof(float), f->R, hipMemcpyDeviceToDevice, s));
    // status MGP_OK for every run: step 1 predicts from x_bar_0
    HIP_TRY(hipMemsetAsync(f->d_stats, 0, (size_t)f->R * sizeof(mgp_stats), s));
    HIP_TRY(hipMemsetAsync(f->est, 0, (size_t)f->R * f->T * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(f->b_hist, 0, (size_t)f->R * f->T * sizeof(uint32_t), s));
    HIP_TRY(hipMemsetAsync(f->st_hist, 0, (size_t)f->R * f->T * sizeof(int32_t), s));
    f->next_t = 1;
    f->next_stage = 1;
    return MGP_OK;
}

int mgp_sir_predict_update(mgp_sir_filter* f, int32_t t, void* stream)
{
    clear_error();
    if (!f) return fail(MGP_EINVAL, "filter is NULL");
    int rc = check_stage(f, t, 1);
    if (!rc) rc = enqueue_predict(f, (uint32_t)t, false, static_cast<hipStream_t>(stream));
    if (!rc) advance(f);
    return rc;
}

int mgp_sir_resample(mgp_sir_filter* f, int32_t t, void* stream)
{
    clear_error();
    if (!f) return fail(MGP_EINVAL, "filter is NULL");
    int rc = check_stage(f, t, 2);
    if (!rc) rc = enqueue_resample(f, (uint32_t)t, static_cast<hipStream_t>(stream));
    if (!rc) advance(f);
    return rc;
}

int mgp_sir_estimate(mgp_sir_filter* f, int32_t t, void* stream)
{
    clear_error();
    if (!f) return fail(MGP_EINVAL, "filter is NULL");
    int rc = check_stage(f, t, 3);
    if (!rc) rc = enqueue_estimate(f, (uint32_t)t, static_cast<hipStream_t>(stream));
    if (!rc) advance(f);
    return rc;
}

int mgp_sir_run(mgp_sir_filter* f, void* stream)
{
    clear_error();
    if (!f) return fail(MGP_EINVAL, "filter is NULL");
    int rc = check_stage(f, 1, 1);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (f->exec) {
        HIP_TRY(hipGraphLaunch(f->exec, s));
    } else {
        rc = enqueue_steps(f, s);
        if (rc) return rc;
    }
    f->next_t = f->T + 1;
    f->next_stage = 1;
    return MGP_OK;
}

int mgp_sir_results(mgp_sir_filter* f, double* est_host, uint32_t* B_host, int32_t* status_host, void* stream)
{
    clear_error();
    if (!f) return fail(MGP_EINVAL, "filter is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t cnt = (size_t)f->R * f->T;
    if (est_host) HIP_TRY(hipMemcpyAsync(est_host, f->est, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    if (B_host) HIP_TRY(hipMemcpyAsync(B_host, f->b_hist, cnt * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (status_host) HIP_TRY(hipMemcpyAsync(status_host, f->st_hist, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MGP_OK;
}

int mgp_sir_get_buffers(const mgp_sir_filter* f, mgp_sir_buffers* b)
{
    clear_error();
    if (!f || !b) return fail(MGP_EINVAL, "NULL argument");
    b->x_dev = f->x;
    b->w_dev = f->w;
    b->xbar_dev = f->xbar;
    b->ancestors_dev = f->anc;
    b->ld = (int64_t)f->ld;
    b->device_bytes = (int64_t)f->dmem_bytes;
    b->accept_grid = (int64_t)f->grid;
    b->block_threads = f->shape.bt;
    b->particles_per_thread = f->shape.ppt;
    return MGP_OK;
}

int mgp_sir_copy_buffer(const mgp_sir_filter* f, int32_t which, void* dst_dev, void* stream)
{
    clear_error();
    if (!f || !dst_dev) return fail(MGP_EINVAL, "NULL argument");
    const void* src = which == MGP_SIR_X      ? (const void*)f->x
                      : which == MGP_SIR_W    ? (const void*)f->w
                      : which == MGP_SIR_XBAR ? (const void*)f->xbar
                      : which == MGP_SIR_ANCESTORS ? (const void*)f->anc
                                                   : nullptr;
    if (!src) return fail(MGP_EINVAL, "unknown buffer %d", which);
    HIP_TRY(hipMemcpy2DAsync(dst_dev, (size_t)f->n * 4u, src, f->ld * 4u, (size_t)f->n * 4u, f->R,
                             hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return MGP_OK;
}

int mgp_sir_destroy(mgp_sir_filter* f)
{
    clear_error();
    if (!f) return MGP_OK;
    free_filter(f);
    return MGP_OK;
}

}  // extern "C"
