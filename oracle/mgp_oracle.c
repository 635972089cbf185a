/*
 * mgp_oracle.c -- plain, single-threaded CPU reference for Metropolis-family
 * parallel resampling (Metropolis, Metropolis-C1, Metropolis-C2, Megopolis),
 * after "The Megopolis Resampler: Memory Coalesced Resampling on GPUs"
 * (Chesser, Nguyen, Ranasinghe; arXiv 2109.13504).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library. The HIP
 * product library never links, loads or calls it, and the two share no code,
 * headers, tables or helpers. Build it with
 *     gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -lm
 * so that every fp32 product is one IEEE round-to-nearest-even multiply
 * (x86-64 SSE, FLT_EVAL_METHOD == 0, denormals kept).
 *
 * What it computes, and where the paper defines it:
 *   - Metropolis resample            : Algorithm 2 (Section 3)
 *   - Metropolis-C1 / -C2 resample   : Algorithms 3 and 4 (Section 3.1)
 *   - Megopolis resample             : Algorithm 5 (Section 4)
 *   - number of iterations B         : eq. (bcalc) in Section 3 and
 *                                      eq. (proposition), Section 4.1
 *   - particle copy x_bar_i = x_k    : last statement of Algorithms 2-5
 *   - M != N resampling              : the closing discussion (Section 8)
 *   - SIR application (predict, update, estimate): Algorithm 6, Section 7
 *   - multinomial and systematic resampling through a prefix sum of the
 *     weights (the unbiased comparison methods): Algorithms 7 and 8
 *     (the appendix), Section 6.5
 *
 * The paper fixes the algorithms but not the random-number generator (it used
 * a stateful generator on its GPU). Here every random draw is a pure function
 * of (seed, stream, index, iteration) through the counter-based generator
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11), so each particle's chain can be recomputed alone.
 * Stream layout (the HIP library implements the same layout independently):
 *
 *   key     = (low 32 bits of seed, high 32 bits of seed)
 *   counter = (block, tag, stream_id, index)
 *
 *   tag 0  u draws        index = particle i, block = b / 5, five u per call
 *   tag 1  j draws        index = particle i, block = b / 4, word b % 4
 *   tag 2  Megopolis o_b  index = 0,          block = b / 4, word b % 4
 *   tag 3  C1 partition   index = group g,    block = 0,     word 0
 *   tag 4  C2 partition   index = group g,    block = b / 4, word b % 4
 *   tag 5  SIR noise      index = i / 4,      block = step t, Box-Muller pairs
 *   tag 6  multinomial    index = output i,   block = 0,     words 0-1: one 64-bit draw
 *   tag 7  systematic     index = 0,          block = 0,     words 0-1: one 64-bit draw
 *
 * with group g = floor(i / 32) (the paper's warp index). Maps from 32-bit words:
 *   u in (0,1]   : m = 24 random bits, u = (m + 1) * 2^-24   (exact in fp32)
 *                  call words x0..x3 give m = x_r >> 8 for r < 4 and
 *                  m = (x0 & 255) | (x1 & 255) << 8 | (x2 & 255) << 16 for r = 4
 *   U{0, n-1}    : floor(x * n / 2^32)
 *
 * Each function computes what its definition states, one particle and one
 * step at a time, with no blocking, fusion or reordering.
 *
 * Parity unpinned: the paper does not fix the stream layout above, the two
 * word-to-number maps, the clamps of B (at least 1, at most b_max, 1 when the
 * mean weight reaches the largest), the C1/C2 partition of a ragged last
 * group, the SIR noise layout and prior, the M != N start positions, or the
 * fixed-point form of the prefix sums. These are this library's readings,
 * checked here by self-consistency and by the statistical tests (uniformity,
 * moments, the paper's bias and MSE figures), not by values the paper prints.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define OR_METROPOLIS 0
#define OR_C1 1
#define OR_C2 2
#define OR_MEGOPOLIS 3

#define OR_TAG_U 0u
#define OR_TAG_J 1u
#define OR_TAG_OFFSET 2u
#define OR_TAG_C1_PART 3u
#define OR_TAG_C2_PART 4u

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_EWEIGHTS (-6)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-box on a  */
/* 4 x 32-bit counter; the 2 x 32-bit key is advanced by the Weyl constants   */
/* between rounds.                                                            */
/* ------------------------------------------------------------------------ */
void mgp_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void draw_words(uint64_t seed, uint32_t tag, uint32_t stream_id, uint32_t index,
                       uint32_t block, uint32_t x[4])
{
    uint32_t ctr[4] = {block, tag, stream_id, index};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    mgp_oracle_philox4x32_10(ctr, key, x);
}

/* U{0, n-1} from one 32-bit word. */
static uint32_t uniform_index(uint32_t x, uint32_t n)
{
    return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

/* u ~ U(0,1] for particle i at iteration b (the "u ~ U[0,1]" draw of
 * Algorithms 2-5). */
float mgp_oracle_draw_u(uint64_t seed, uint32_t stream_id, uint32_t i, uint32_t b)
{
    uint32_t x[4];
    draw_words(seed, OR_TAG_U, stream_id, i, b / 5u, x);
    uint32_t r = b % 5u;
    uint32_t m;
    if (r < 4u)
        m = x[r] >> 8;
    else
        m = (x[0] & 0xFFu) | ((x[1] & 0xFFu) << 8) | ((x[2] & 0xFFu) << 16);
    float mf = (float)(m + 1u); /* <= 2^24, exact */
    return mf * 0x1p-24f;       /* power-of-two scaling, exact */
}

/* The b-th Megopolis offset o_b ~ U{0, N-1}, shared by every particle
 * (Algorithm 5, offsets drawn as a separate task before the particle loop). */
uint32_t mgp_oracle_offset(uint64_t seed, uint32_t stream_id, uint32_t n, uint32_t b)
{
    uint32_t x[4];
    draw_words(seed, OR_TAG_OFFSET, stream_id, 0u, b / 4u, x);
    return uniform_index(x[b % 4u], n);
}

void mgp_oracle_offsets(uint64_t seed, uint32_t stream_id, uint32_t n, uint32_t B, uint32_t* o)
{
    for (uint32_t b = 0; b < B; ++b)
        o[b] = mgp_oracle_offset(seed, stream_id, n, b);
}

/* Megopolis candidate index (Algorithm 5, Section 4). With segments of S
 * consecutive weights (the paper's S is its 32-thread warp; `segment`, a power
 * of two, allows e.g. 64 for a 64-lane wavefront), an offset o does two
 * things to particle i: it moves i's segment floor(o / S) segments forward,
 * and it rotates i's place inside the segment by o mod S. The candidate is
 * that place in that segment, wrapped around the N weights. */
uint32_t mgp_oracle_megopolis_index_s(uint32_t i, uint32_t o, uint32_t n, uint32_t segment)
{
    uint64_t dest_segment = (uint64_t)(i / segment) + (uint64_t)(o / segment);
    uint64_t place = ((uint64_t)(i % segment) + (uint64_t)(o % segment)) % segment;
    return (uint32_t)((dest_segment * segment + place) % (uint64_t)n);
}

/* The paper's segment is its 32-thread warp. */
uint32_t mgp_oracle_megopolis_index(uint32_t i, uint32_t o, uint32_t n)
{
    return mgp_oracle_megopolis_index_s(i, o, n, 32u);
}

/* Metropolis-C1/C2 candidate index (Algorithms 3 and 4): a partition p of
 * N_w = P_size / 4 weights, then j uniform inside it. The paper's
 * N_part = 4N / P_size is read as ceil(N / N_w) and the last partition is cut
 * at N, so that every index is valid for any N. */
static uint32_t partition_index(uint32_t n, uint32_t n_w, uint32_t part_word, uint32_t j_word)
{
    uint32_t n_part = (uint32_t)(((uint64_t)n + n_w - 1u) / n_w);
    uint32_t p = uniform_index(part_word, n_part);
    uint64_t start = (uint64_t)p * n_w;
    uint64_t width = (uint64_t)n - start;
    if (width > n_w) width = n_w;
    return (uint32_t)(start + uniform_index(j_word, (uint32_t)width));
}

/* Candidate index j for particle i at iteration b, for each variant.
 * `offsets` holds o_0..o_{B-1} (Megopolis only). `pos` is the input position
 * the particle's chain started from (i itself when inputs and outputs are
 * the same particles; i mod N when M != N): the Megopolis segment arithmetic
 * uses it, while the random draws and the C1/C2 group use i. */
static uint32_t proposal(int variant, uint32_t n, uint32_t n_w, uint32_t segment, uint64_t seed,
                         uint32_t stream_id, const uint32_t* offsets, uint32_t i, uint32_t pos, uint32_t b)
{
    uint32_t x[4], px[4];
    switch (variant) {
    case OR_METROPOLIS: /* j ~ U{0, N-1} (Algorithm 2) */
        draw_words(seed, OR_TAG_J, stream_id, i, b / 4u, x);
        return uniform_index(x[b % 4u], n);
    case OR_C1: /* one partition per group for all b (Algorithm 3) */
        draw_words(seed, OR_TAG_C1_PART, stream_id, i / 32u, 0u, px);
        draw_words(seed, OR_TAG_J, stream_id, i, b / 4u, x);
        return partition_index(n, n_w, px[0], x[b % 4u]);
    case OR_C2: /* a new partition per group at every b (Algorithm 4) */
        draw_words(seed, OR_TAG_C2_PART, stream_id, i / 32u, b / 4u, px);
        draw_words(seed, OR_TAG_J, stream_id, i, b / 4u, x);
        return partition_index(n, n_w, px[b % 4u], x[b % 4u]);
    default: /* OR_MEGOPOLIS */
        return mgp_oracle_megopolis_index_s(pos, offsets[b], n, segment);
    }
}

static int check_common(int variant, int32_t n, uint32_t partition_bytes)
{
    if (n < 1) return OR_EINVAL;
    if (variant < OR_METROPOLIS || variant > OR_MEGOPOLIS) return OR_EINVAL;
    if ((variant == OR_C1 || variant == OR_C2) &&
        (partition_bytes < 4u || partition_bytes % 4u != 0u))
        return OR_EINVAL;
    return OR_OK;
}

/* One particle's chain: k <- pos (= i for M = N), then B accept/reject steps against candidate
 * j with the ratio test u <= w_j / w_k written as the fp32 product
 * u * w_k <= w_j (ties accept). Returns the ancestor k. */
static int32_t run_chain(const float* w, uint32_t n, int variant, uint32_t B, uint64_t seed,
                         uint32_t stream_id, uint32_t n_w, uint32_t segment, const uint32_t* offsets,
                         uint32_t i, uint32_t pos, uint64_t* accepts)
{
    uint32_t k = pos;
    for (uint32_t b = 0; b < B; ++b) {
        uint32_t j = proposal(variant, n, n_w, segment, seed, stream_id, offsets, i, pos, b);
        float u = mgp_oracle_draw_u(seed, stream_id, i, b);
        float p = u * w[k];
        if (p <= w[j]) {
            k = j;
            if (accepts) *accepts += 1u;
        }
    }
    return (int32_t)k;
}

/* Full resample: ancestors for all N particles. The offsets of a Megopolis
 * call are generated first, then the particle loop runs. `offsets_scratch`
 * must hold B entries (Megopolis only; may be NULL otherwise). */
int mgp_oracle_resample(const float* w, int32_t n, int variant, uint32_t B, uint64_t seed,
                        uint32_t stream_id, uint32_t partition_bytes, uint32_t* offsets_scratch,
                        int32_t* ancestors, uint64_t* accepts)
{
    int rc = check_common(variant, n, partition_bytes);
    if (rc) return rc;
    if (variant == OR_MEGOPOLIS) {
        if (!offsets_scratch) return OR_EINVAL;
        mgp_oracle_offsets(seed, stream_id, (uint32_t)n, B, offsets_scratch);
    }
    if (accepts) *accepts = 0;
    uint32_t n_w = partition_bytes / 4u;
    for (uint32_t i = 0; i < (uint32_t)n; ++i)
        ancestors[i] = run_chain(w, (uint32_t)n, variant, B, seed, stream_id, n_w, 32u,
                                 offsets_scratch, i, i, accepts);
    return OR_OK;
}

/* M != N resampling (the paper's closing discussion: for D-PMC-style use the
 * Megopolis offsets range over the number of inputs): m ancestors from n
 * weighted inputs. Output i in [0, m) starts its chain at input i mod n;
 * offsets o_b ~ U{0, n-1} and candidates are taken over the n inputs, with
 * the Megopolis segment arithmetic on the start position; the u and j draws
 * and the C1/C2 group floor(i / 32) are those of output i. With m == n this
 * is mgp_oracle_resample. `segment` is the Megopolis segment width (32, the
 * paper's, or 64). */
int mgp_oracle_resample_m(const float* w, int32_t n, int32_t m, int variant, uint32_t B, uint64_t seed,
                          uint32_t stream_id, uint32_t partition_bytes, uint32_t segment,
                          uint32_t* offsets_scratch, int32_t* ancestors)
{
    int rc = check_common(variant, n, partition_bytes);
    if (rc) return rc;
    if (m < 1) return OR_EINVAL;
    if (segment != 32u && segment != 64u) return OR_EINVAL;
    if (variant == OR_MEGOPOLIS) {
        if (!offsets_scratch) return OR_EINVAL;
        mgp_oracle_offsets(seed, stream_id, (uint32_t)n, B, offsets_scratch);
    }
    uint32_t n_w = partition_bytes / 4u;
    for (uint32_t i = 0; i < (uint32_t)m; ++i)
        ancestors[i] = run_chain(w, (uint32_t)n, variant, B, seed, stream_id, n_w, segment, offsets_scratch,
                                 i, i % (uint32_t)n, NULL);
    return OR_OK;
}

/* Ancestors of the particles idx[0..count) only: the same chains as
 * mgp_oracle_resample (each chain is independent of the others), with the
 * Megopolis segment width `segment` (32, the paper's, or 64). When accepts
 * is not NULL it receives the number of accepted steps of these chains. */
int mgp_oracle_resample_subset(const float* w, int32_t n, int variant, uint32_t B, uint64_t seed,
                               uint32_t stream_id, uint32_t partition_bytes, uint32_t segment,
                               uint32_t* offsets_scratch, const int32_t* idx, int32_t count,
                               int32_t* ancestors, uint64_t* accepts)
{
    int rc = check_common(variant, n, partition_bytes);
    if (rc) return rc;
    if (segment != 32u && segment != 64u) return OR_EINVAL;
    if (variant == OR_MEGOPOLIS) {
        if (!offsets_scratch) return OR_EINVAL;
        mgp_oracle_offsets(seed, stream_id, (uint32_t)n, B, offsets_scratch);
    }
    uint32_t n_w = partition_bytes / 4u;
    if (accepts) *accepts = 0;
    for (int32_t c = 0; c < count; ++c) {
        if (idx[c] < 0 || idx[c] >= n) return OR_EINVAL;
        ancestors[c] = run_chain(w, (uint32_t)n, variant, B, seed, stream_id, n_w, segment,
                                 offsets_scratch, (uint32_t)idx[c], (uint32_t)idx[c], accepts);
    }
    return OR_OK;
}

/* The candidate indices j_0..j_{B-1} and draws u_0..u_{B-1} of particle i
 * (for tests that check the accept logic against the draws). */
int mgp_oracle_trace(int32_t n, int variant, uint32_t B, uint64_t seed, uint32_t stream_id,
                     uint32_t partition_bytes, uint32_t* offsets_scratch, int32_t i,
                     uint32_t* j_out, float* u_out)
{
    int rc = check_common(variant, n, partition_bytes);
    if (rc) return rc;
    if (i < 0 || i >= n) return OR_EINVAL;
    if (variant == OR_MEGOPOLIS) {
        if (!offsets_scratch) return OR_EINVAL;
        mgp_oracle_offsets(seed, stream_id, (uint32_t)n, B, offsets_scratch);
    }
    uint32_t n_w = partition_bytes / 4u;
    for (uint32_t b = 0; b < B; ++b) {
        j_out[b] = proposal(variant, (uint32_t)n, n_w, 32u, seed, stream_id, offsets_scratch,
                            (uint32_t)i, (uint32_t)i, b);
        u_out[b] = mgp_oracle_draw_u(seed, stream_id, (uint32_t)i, b);
    }
    return OR_OK;
}

/* Weight statistics needed by the B rule: max(w) in fp32 (exact, order-free),
 * sum(w) accumulated in fp64 in index order. Weights must be finite, >= 0,
 * and not all zero. */
int mgp_oracle_reduce(const float* w, int32_t n, float* w_max, double* w_sum)
{
    if (n < 1) return OR_EINVAL;
    float mx = 0.0f;
    double s = 0.0;
    int bad = 0;
    for (int32_t i = 0; i < n; ++i) {
        float v = w[i];
        if (!(v >= 0.0f) || isinf(v)) bad = 1;
        if (v > mx) mx = v;
        s += (double)v;
    }
    *w_max = mx;
    *w_sum = s;
    if (bad || !(mx > 0.0f)) return OR_EWEIGHTS;
    return OR_OK;
}

/* Number of iterations, eq. (proposition):
 *     B = ceil( log(eps) / log(1 - E(w) / max(w)) )
 * with E(w) the sample mean, in fp64 (log1p for the denominator). If
 * E(w) / max(w) >= 1 (all weights equal) one iteration suffices. The result
 * is at least 1 and is clamped to b_max (reported through *clamped). */
int mgp_oracle_choose_B(double w_sum, float w_max, int32_t n, double eps, uint32_t b_max,
                        uint32_t* B, double* raw_out, int* clamped)
{
    if (n < 1 || !(eps > 0.0) || !(eps <= 1.0) || b_max < 1u) return OR_EINVAL;
    double mean = w_sum / (double)n;
    double r = mean / (double)w_max;
    double raw;
    *clamped = 0;
    if (r >= 1.0) {
        raw = 1.0;
    } else {
        raw = log(eps) / log1p(-r);
    }
    if (raw_out) *raw_out = raw;
    double c = ceil(raw);
    if (c < 1.0) c = 1.0;
    if (c > (double)b_max) {
        c = (double)b_max;
        *clamped = 1;
    }
    *B = (uint32_t)c;
    return OR_OK;
}

/* x_bar_i = x_{k_i}: copy the D-dimensional state row of each ancestor. */
int mgp_oracle_gather(const float* states, int32_t n_states, int32_t d, const int32_t* ancestors,
                      int32_t n_out, float* out)
{
    if (n_states < 1 || d < 1 || n_out < 0) return OR_EINVAL;
    for (int32_t i = 0; i < n_out; ++i) {
        int32_t k = ancestors[i];
        if (k < 0 || k >= n_states) return OR_ERANGE;
        for (int32_t c = 0; c < d; ++c)
            out[(size_t)i * (size_t)d + (size_t)c] = states[(size_t)k * (size_t)d + (size_t)c];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* The SIR application of Section 7 (Algorithm 6, eqs. (predict-end2end) and */
/* (update-end2end)): x_t = x/2 + 25 x / (1 + x^2) + 8 cos(1.2 t) + v with    */
/* v ~ N(0, 10); z_t = x_t^2 / 20 + n with n ~ N(0, 1); the unnormalised      */
/* weight is the likelihood exp(-(z_t - x_t^2/20)^2 / 2).                     */
/* ------------------------------------------------------------------------ */
#define OR_TAG_SIR_NOISE 5u
#define OR_PI 3.14159265358979323846

/* Standard normal draw of particle i at step t of run `run`: Box-Muller in
 * its two-output form. Philox call (t, tag 5, run, floor(i / 4)) gives words
 * x0..x3; particles 4m and 4m+1 share the pair (x0, x1), particles 4m+2 and
 * 4m+3 the pair (x2, x3). For a pair (a, b):
 *   u1 = (a + 1) 2^-32 in (0, 1],  u2 = b 2^-32 in [0, 1),
 *   e = sqrt(-2 ln u1) cos(2 pi u2) for even i, sqrt(-2 ln u1) sin(2 pi u2)
 *   for odd i   (fp64). */
double mgp_oracle_sir_normal(uint64_t seed, uint32_t run, uint32_t i, uint32_t t)
{
    uint32_t x[4];
    draw_words(seed, OR_TAG_SIR_NOISE, run, i / 4u, t, x);
    uint32_t pair = (i / 2u) % 2u;
    double u1 = ((double)x[2u * pair] + 1.0) * 0x1p-32;
    double u2 = (double)x[2u * pair + 1u] * 0x1p-32;
    double radius = sqrt(-2.0 * log(u1));
    double angle = 2.0 * OR_PI * u2;
    return (i % 2u == 0u) ? radius * cos(angle) : radius * sin(angle);
}

/* Stage 1 of Algorithm 6 for n particles: predict from the resampled
 * particles of step t-1 and weight by the measurement z_t. Arithmetic in
 * fp64, each result rounded once to fp32. */
void mgp_oracle_sir_predict_update(const float* xbar, int32_t n, uint32_t t, double z, uint64_t seed, uint32_t run,
                                   float* x_out, float* w_out)
{
    const double sigma_v = sqrt(10.0);
    const double drift = 8.0 * cos(1.2 * (double)t);
    for (int32_t i = 0; i < n; ++i) {
        double xp = (double)xbar[i];
        double v = sigma_v * mgp_oracle_sir_normal(seed, run, (uint32_t)i, t);
        double xn = xp / 2.0 + 25.0 * xp / (1.0 + xp * xp) + drift + v;
        float xf = (float)xn;
        double xd = (double)xf;
        double r = z - xd * xd / 20.0;
        x_out[i] = xf;
        w_out[i] = (float)exp(-0.5 * r * r);
    }
}

/* Stage 3 of Algorithm 6: the estimate, the mean of the resampled particles
 * (fp64, index order). */
double mgp_oracle_mean(const float* x, int32_t n)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += (double)x[i];
    return s / (double)n;
}

/* ------------------------------------------------------------------------ */
/* Prefix-sum resamplers (the unbiased comparison methods of Section 6.5 and */
/* Table 2): multinomial resampling (Algorithm 7) and systematic resampling  */
/* (Algorithm 8). Both find, for each output i, the first input j whose      */
/* inclusive prefix sum of weights exceeds a threshold t_i: multinomial with */
/* an independent uniform t_i per output, systematic with the evenly spaced  */
/* t_i = (i + u) S / N from one uniform u. The prefix sum runs on the        */
/* weights in 64-bit fixed point, where it is exact.                         */
/* ------------------------------------------------------------------------ */
#define OR_MULTINOMIAL 0
#define OR_SYSTEMATIC 1
#define OR_TAG_MULTINOMIAL 6u
#define OR_TAG_SYSTEMATIC 7u

/* The fixed-point exponent K of n weights whose maximum is w_max > 0: with
 * w_max = m 2^E, m in [0.5, 1), K = 62 - ceil(log2 n) - E. Then every
 * q_i = floor(w_i 2^K) is below 2^(62 - ceil(log2 n)) and n of them sum to
 * less than 2^62. */
int mgp_oracle_prefix_scale(float w_max, int32_t n)
{
    int E = 0;
    frexp((double)w_max, &E);
    int L = 0;
    while (((int64_t)1 << L) < (int64_t)n) ++L;
    return 62 - L - E;
}

/* q = floor(w 2^K): exact in fp64 (a power-of-two scaling of an fp32 value
 * stays inside fp64's range for every K the scale above can give). */
uint64_t mgp_oracle_prefix_fixed(float w, int K)
{
    return (uint64_t)floor(ldexp((double)w, K));
}

/* Inclusive prefix sums incl[j] = q_0 + ... + q_j, in index order. Returns
 * OR_EWEIGHTS for invalid weights (as mgp_oracle_reduce); *K_out gets K. */
int mgp_oracle_prefix_sum(const float* w, int32_t n, uint64_t* incl, int* K_out)
{
    float w_max;
    double w_sum;
    int rc = mgp_oracle_reduce(w, n, &w_max, &w_sum);
    if (rc) return rc;
    int K = mgp_oracle_prefix_scale(w_max, n);
    uint64_t run = 0;
    for (int32_t j = 0; j < n; ++j) {
        run += mgp_oracle_prefix_fixed(w[j], K);
        incl[j] = run;
    }
    if (K_out) *K_out = K;
    return OR_OK;
}

/* The threshold t_i in [0, S) of output i, S the total of the fixed-point
 * weights.
 *   multinomial (Algorithm 7: u ~ U[0, total)): a 64-bit draw r from words 0
 *     and 1 of Philox call (0, tag 6, stream_id, i), t = floor(r S / 2^64);
 *   systematic (Algorithm 8: u = (i + u_t) / N after one draw u_t ~ U[0, 1)):
 *     u_t = (r >> 11) 2^-53 from the 64-bit draw r of call (0, tag 7,
 *     stream_id, 0), then in fp64 with the rounding of each operation
 *     c = S / N, v = (i + u_t) c, t = floor(v), and t = S - 1 should the
 *     rounding take v to S. */
uint64_t mgp_oracle_prefix_threshold(int method, uint64_t S, int32_t n, uint64_t seed, uint32_t stream_id,
                                     uint32_t i)
{
    uint32_t x[4];
    if (method == OR_MULTINOMIAL) {
        draw_words(seed, OR_TAG_MULTINOMIAL, stream_id, i, 0u, x);
        uint64_t r = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        return (uint64_t)(((unsigned __int128)r * (unsigned __int128)S) >> 64);
    }
    draw_words(seed, OR_TAG_SYSTEMATIC, stream_id, 0u, 0u, x);
    uint64_t r = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    double ut = (double)(r >> 11) * 0x1p-53;
    double c = (double)S / (double)n;
    double v = ((double)i + ut) * c;
    uint64_t t = (uint64_t)floor(v);
    return t < S ? t : S - 1u;
}

/* The first j with incl[j] > t (incl nondecreasing, incl[n-1] > t), by
 * bisection. */
static int32_t first_above(const uint64_t* incl, int32_t n, uint64_t t)
{
    int32_t lo = 0, hi = n - 1; /* the answer lies in [lo, hi] */
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (incl[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

/* Multinomial (method 0) or systematic (method 1) resampling of n weighted
 * particles: ancestors[i] = the first j with incl[j] > t_i. incl_scratch
 * holds n entries. Zero weights repeat the prefix sum and are never chosen. */
int mgp_oracle_resample_prefix(const float* w, int32_t n, int method, uint64_t seed, uint32_t stream_id,
                               uint64_t* incl_scratch, int32_t* ancestors)
{
    if (n < 1 || (method != OR_MULTINOMIAL && method != OR_SYSTEMATIC) || !incl_scratch) return OR_EINVAL;
    int rc = mgp_oracle_prefix_sum(w, n, incl_scratch, NULL);
    if (rc) return rc;
    uint64_t S = incl_scratch[n - 1];
    for (int32_t i = 0; i < n; ++i) {
        uint64_t t = mgp_oracle_prefix_threshold(method, S, n, seed, stream_id, (uint32_t)i);
        ancestors[i] = first_above(incl_scratch, n, t);
    }
    return OR_OK;
}
