/* A plain C client of libmgp: no Python, no torch. It reads n fp32 weights
 * and n x d fp32 states from files, resamples them with mgp_resample
 * (Megopolis, B from epsilon) and mgp_gather on a stream of its own, and
 * writes the ancestors, the gathered states and B to files, so that a test
 * can compare them with the oracle.
 *
 * usage: c_client <weights.f32> <states.f32> <n> <d> <seed> <out_anc.i32> <out_states.f32> <out_B.txt> */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mgp.h"

static int read_file(const char* path, void* buf, size_t bytes)
{
    FILE* f = fopen(path, "rb");
    if (!f) return -1;
    size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    return got == bytes ? 0 : -1;
}

static int write_file(const char* path, const void* buf, size_t bytes)
{
    FILE* f = fopen(path, "wb");
    if (!f) return -1;
    size_t put = fwrite(buf, 1, bytes, f);
    fclose(f);
    return put == bytes ? 0 : -1;
}

#define CHECK_HIP(call)                                                   \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));   \
            return 2;                                                     \
        }                                                                 \
    } while (0)

#define CHECK_MGP(call)                                                   \
    do {                                                                  \
        int r_ = (call);                                                  \
        if (r_ != MGP_OK) {                                               \
            fprintf(stderr, "%s: %d %s\n", #call, r_, mgp_last_error());  \
            return 3;                                                     \
        }                                                                 \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: %s weights states n d seed out_anc out_states out_B\n", argv[0]);
        return 1;
    }
    const int32_t n = atoi(argv[3]), d = atoi(argv[4]);
    const uint64_t seed = strtoull(argv[5], NULL, 10);
    if (n < 1 || d < 1) return 1;
    float* w = malloc(sizeof(float) * (size_t)n);
    float* st = malloc(sizeof(float) * (size_t)n * d);
    int32_t* anc = malloc(sizeof(int32_t) * (size_t)n);
    float* out = malloc(sizeof(float) * (size_t)n * d);
    if (!w || !st || !anc || !out) return 1;
    if (read_file(argv[1], w, sizeof(float) * (size_t)n) || read_file(argv[2], st, sizeof(float) * (size_t)n * d))
        return 1;

    mgp_params p = {0};
    p.variant = MGP_MEGOPOLIS;
    p.B = 0;
    p.epsilon = 0.01;
    p.seed = seed;
    size_t ws_bytes = 0;
    CHECK_MGP(mgp_workspace_size(n, &p, &ws_bytes));

    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    float *w_dev, *st_dev, *out_dev;
    int32_t* anc_dev;
    void* ws_dev;
    mgp_stats* stats_dev;
    CHECK_HIP(hipMalloc((void**)&w_dev, sizeof(float) * (size_t)n));
    CHECK_HIP(hipMalloc((void**)&st_dev, sizeof(float) * (size_t)n * d));
    CHECK_HIP(hipMalloc((void**)&out_dev, sizeof(float) * (size_t)n * d));
    CHECK_HIP(hipMalloc((void**)&anc_dev, sizeof(int32_t) * (size_t)n));
    CHECK_HIP(hipMalloc(&ws_dev, ws_bytes));
    CHECK_HIP(hipMalloc((void**)&stats_dev, sizeof(mgp_stats)));
    CHECK_HIP(hipMemcpy(w_dev, w, sizeof(float) * (size_t)n, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(st_dev, st, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice));

    CHECK_MGP(mgp_resample(w_dev, n, &p, anc_dev, stats_dev, ws_dev, ws_bytes, s));
    CHECK_MGP(mgp_gather(st_dev, n, d, anc_dev, n, out_dev, s));
    CHECK_HIP(hipStreamSynchronize(s));

    mgp_stats stats;
    CHECK_HIP(hipMemcpy(&stats, stats_dev, sizeof stats, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(anc, anc_dev, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(out, out_dev, sizeof(float) * (size_t)n * d, hipMemcpyDeviceToHost));
    if (stats.status != MGP_OK) {
        fprintf(stderr, "status %d\n", stats.status);
        return 4;
    }
    FILE* fb = fopen(argv[8], "w");
    if (!fb) return 1;
    fprintf(fb, "%u\n", stats.B);
    fclose(fb);
    if (write_file(argv[6], anc, sizeof(int32_t) * (size_t)n) || write_file(argv[7], out, sizeof(float) * (size_t)n * d))
        return 1;

    (void)hipFree(w_dev);
    (void)hipFree(st_dev);
    (void)hipFree(out_dev);
    (void)hipFree(anc_dev);
    (void)hipFree(ws_dev);
    (void)hipFree(stats_dev);
    (void)hipStreamDestroy(s);
    free(w);
    free(st);
    free(anc);
    free(out);
    return 0;
}
