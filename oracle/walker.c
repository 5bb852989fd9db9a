/*
 * Plain C random walker for the Monte Carlo NEGF estimator (oracle).
 *
 * TEST INFRASTRUCTURE ONLY: built and called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  Shares no code with the HIP library.
 *
 * The walk is the elastic linear-response procedure of Sec. II E-F of Musland, Bergli and
 * Flage-Larsen: inject at lead p (steps 3-4 with the channel marginalised), then repeat
 * step 6' (Eqs. (75), (76)) until a lead is drawn.  The estimator of Eq. (66) is
 * Tr Gamma_p A times [exit lead == q]; this file only counts exits, the caller multiplies.
 *
 * Random numbers: Philox4x32-10, written from its published definition (J. K. Salmon,
 * M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): 10 rounds of two 32x32->64 multiplications with constants 0xD2511F53 and
 * 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
 *
 * Stream layout (the HIP walker draws exactly the same words):
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   tag     = (realization << 1) | inject_lead
 *   block j of walker w at energy index k: counter = (j, w, k, tag)
 *   step n of a walk uses words (2*(n&1), 2*(n&1)+1) of block n>>1: call them (a, b)
 *
 * Two samplers:
 *   cdf   : the paper's rule (Sec. III B): u = 53-bit uniform from (a, b); cumulative sums
 *           b_j of the row normalised by the last one; the first j with b_j > u is drawn.
 *   alias : a given alias table (uint32 thresholds, int32 aliases): bucket c = (a*n)>>32
 *           with Lemire's rejection of the low word below (2^32 - n) mod n; the r-th redraw
 *           of step n takes word 0 of Philox(counter = (n, w, k, tag | 0x80000000),
 *           key = (key0, key1 ^ r)); outcome = (b < thr[c]) ? c : alias[c].
 *
 * Tallies per energy (int64, accumulated): [absorbed at L, absorbed at R, truncated,
 * sum of steps, sum of squared steps].  Injection counts as one step.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct {
    uint32_t key[2];
    uint32_t w, k, tag;
    uint32_t block_index;   /* which block is cached in words[] (UINT32_MAX: none) */
    uint32_t words[4];
} stream_t;

static void stream_init(stream_t *s, uint64_t seed, uint32_t w, uint32_t k, uint32_t tag)
{
    s->key[0] = (uint32_t)(seed & 0xffffffffu);
    s->key[1] = (uint32_t)(seed >> 32);
    s->w = w; s->k = k; s->tag = tag;
    s->block_index = 0xffffffffu;
}

static void stream_pair(stream_t *s, uint32_t n, uint32_t *a, uint32_t *b)
{
    uint32_t j = n >> 1;
    if (s->block_index != j) {
        uint32_t ctr[4] = {j, s->w, s->k, s->tag};
        oracle_philox4x32_10(ctr, s->key, s->words);
        s->block_index = j;
    }
    *a = s->words[2 * (n & 1)];
    *b = s->words[2 * (n & 1) + 1];
}

/* Lemire's bucket of step n_step from its first word a; *redraws (if not NULL) receives the
 * number of rejected words before the accepted one. */
static uint32_t lemire_bucket_count(stream_t *s, uint32_t n_step, uint32_t a, uint32_t nout,
                                    uint32_t *redraws)
{
    uint32_t r = 0;
    for (;;) {
        uint64_t m = (uint64_t)a * (uint64_t)nout;
        uint32_t lo = (uint32_t)m;
        if (lo >= nout || lo >= (uint32_t)(0u - nout) % nout) {
            if (redraws) *redraws = r;
            return (uint32_t)(m >> 32);
        }
        ++r;
        uint32_t ctr[4] = {n_step, s->w, s->k, s->tag | 0x80000000u};
        uint32_t key[2] = {s->key[0], s->key[1] ^ r};
        uint32_t out[4];
        oracle_philox4x32_10(ctr, key, out);
        a = out[0];
    }
}

static uint32_t lemire_bucket(stream_t *s, uint32_t n_step, uint32_t a, uint32_t nout)
{
    return lemire_bucket_count(s, n_step, a, nout, NULL);
}

/* Paper's step-6' sampler on a dense weight row (Sec. III B). */
static int32_t draw_cdf(const double *row, int32_t n, uint32_t a, uint32_t b)
{
    uint64_t bits = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    double u = (double)bits * (1.0 / 9007199254740992.0);
    double total = 0.0;
    for (int32_t j = 0; j < n; ++j) total += row[j];
    double cum = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        cum += row[j];
        if (cum / total > u) return j;
    }
    return n - 1;
}

/* mode 0: cdf on K [nE][n][n] row-major; mode 1: alias tables thr/alias [nE][n][pitch]. */
static int walk_impl(int mode, const double *K, const uint32_t *thr, const int32_t *alias,
                     int64_t pitch, int32_t nE, int32_t n, uint64_t seed, uint32_t realization,
                     uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                     uint32_t max_steps, int64_t *tallies)
{
    if (n < 3 || nE < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    const int32_t N = n - 2;
    const uint32_t tag = (realization << 1) | inject_lead;
    for (int32_t k = 0; k < nE; ++k) {
        int64_t cL = 0, cR = 0, tr = 0, s1 = 0, s2 = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : cL, cR, tr, s1, s2)
        for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
            uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
            stream_t st;
            stream_init(&st, seed, w, (uint32_t)k, tag);
            int32_t s = N + (int32_t)inject_lead;
            uint32_t steps = 0;
            int outcome = -1;
            while (steps < max_steps) {
                uint32_t a, b;
                stream_pair(&st, steps, &a, &b);
                int32_t next;
                if (mode == 0) {
                    next = draw_cdf(K + ((int64_t)k * n + s) * (int64_t)n, n, a, b);
                } else {
                    uint32_t c = lemire_bucket(&st, steps, a, (uint32_t)n);
                    int64_t e = ((int64_t)k * n + s) * pitch + c;
                    next = (b < thr[e]) ? (int32_t)c : alias[e];
                }
                ++steps;
                if (next >= N) { outcome = next - N; break; }
                s = next;
            }
            if (outcome == 0) ++cL;
            else if (outcome == 1) ++cR;
            else ++tr;
            s1 += steps;
            s2 += (int64_t)steps * (int64_t)steps;
        }
        tallies[5 * k + 0] += cL;
        tallies[5 * k + 1] += cR;
        tallies[5 * k + 2] += tr;
        tallies[5 * k + 3] += s1;
        tallies[5 * k + 4] += s2;
    }
    return 0;
}

int oracle_walk_cdf(const double *K, int32_t nE, int32_t n, uint64_t seed, uint32_t realization,
                    uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                    uint32_t max_steps, int64_t *tallies)
{
    return walk_impl(0, K, NULL, NULL, 0, nE, n, seed, realization, inject_lead, walker_begin,
                     n_walkers, max_steps, tallies);
}

int oracle_walk_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch, int32_t nE,
                      int32_t n, uint64_t seed, uint32_t realization, uint32_t inject_lead,
                      uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                      int64_t *tallies)
{
    if (pitch < n) return -1;
    return walk_impl(1, NULL, thr, alias, pitch, nE, n, seed, realization, inject_lead,
                     walker_begin, n_walkers, max_steps, tallies);
}

/*
 * Energy-sampled walks (Sec. II F step 2 with h(E_k) = w_k / W, W = sum_k w_k): walker w draws
 * its energy from words 0-1 of Philox(counter = (0, w, 0xFFFFFFFF, tag)) as the 53-bit
 * uniform u; with the cumulative weights c_0 = 0, c_{k+1} = c_k + w_k (index order), the
 * energy is the first k with c_{k+1} > u c_nE.  The walk itself is then the ordinary walk of
 * walker w at energy k (same counters as above), with either sampler; tallies go to the
 * drawn energy.  Negative or non-finite weights are rejected.
 */
static int32_t draw_energy(const double *cum, int32_t nE, uint64_t seed, uint32_t w, uint32_t tag)
{
    const uint32_t ctr[4] = {0u, w, 0xFFFFFFFFu, tag};
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    const uint64_t bits = (((uint64_t)x[0] << 32) | x[1]) >> 11;
    const double target = (double)bits * 0x1.0p-53 * cum[nE];
    for (int32_t k = 0; k < nE; ++k)
        if (cum[k + 1] > target) return k;
    return nE - 1;
}

static int walk_sampled_impl(int mode, const double *K, const uint32_t *thr, const int32_t *alias,
                             int64_t pitch, int32_t nE, int32_t n, const double *weights,
                             uint64_t seed, uint32_t realization, uint32_t inject_lead,
                             uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                             int64_t *tallies)
{
    if (n < 3 || nE < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    double *cum = (double *)malloc(sizeof(double) * (size_t)(nE + 1));
    if (!cum) return -1;
    cum[0] = 0.0;
    for (int32_t k = 0; k < nE; ++k) {
        if (!(weights[k] >= 0.0) || weights[k] > 1e308) { free(cum); return -1; }
        cum[k + 1] = cum[k] + weights[k];
    }
    if (!(cum[nE] > 0.0)) { free(cum); return -1; }
    const int32_t N = n - 2;
    const uint32_t tag = (realization << 1) | inject_lead;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
        uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
        const int32_t k = draw_energy(cum, nE, seed, w, tag);
        stream_t st;
        stream_init(&st, seed, w, (uint32_t)k, tag);
        int32_t s = N + (int32_t)inject_lead;
        uint32_t steps = 0;
        int outcome = -1;
        while (steps < max_steps) {
            uint32_t a, b;
            stream_pair(&st, steps, &a, &b);
            int32_t next;
            if (mode == 0) {
                next = draw_cdf(K + ((int64_t)k * n + s) * (int64_t)n, n, a, b);
            } else {
                uint32_t c = lemire_bucket(&st, steps, a, (uint32_t)n);
                int64_t e = ((int64_t)k * n + s) * pitch + c;
                next = (b < thr[e]) ? (int32_t)c : alias[e];
            }
            ++steps;
            if (next >= N) { outcome = next - N; break; }
            s = next;
        }
        int64_t *t = tallies + 5 * (int64_t)k;
        const int slot = outcome == 0 ? 0 : (outcome == 1 ? 1 : 2);
#pragma omp atomic
        t[slot] += 1;
#pragma omp atomic
        t[3] += steps;
#pragma omp atomic
        t[4] += (int64_t)steps * (int64_t)steps;
    }
    free(cum);
    return 0;
}

int oracle_walk_sampled_cdf(const double *K, int32_t nE, int32_t n, const double *weights,
                            uint64_t seed, uint32_t realization, uint32_t inject_lead,
                            uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                            int64_t *tallies)
{
    return walk_sampled_impl(0, K, NULL, NULL, 0, nE, n, weights, seed, realization,
                             inject_lead, walker_begin, n_walkers, max_steps, tallies);
}

int oracle_walk_sampled_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch,
                              int32_t nE, int32_t n, const double *weights, uint64_t seed,
                              uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                              uint64_t n_walkers, uint32_t max_steps, int64_t *tallies)
{
    if (pitch < n) return -1;
    return walk_sampled_impl(1, NULL, thr, alias, pitch, nE, n, weights, seed, realization,
                             inject_lead, walker_begin, n_walkers, max_steps, tallies);
}

/*
 * Importance-sampled walks (Sec. V A, "Improved estimator"): step 6' draws from the modified
 * rows p'_ij = p_ij b_j / rho_i, rho_i = sum_j p_ij b_j, for a non-negative bias b over the
 * outcomes, and the walker carries the likelihood ratio of its path, the product over its
 * steps i -> j of p_ij / p'_ij = rho_i / b_j.  The score of a walk that exits at the
 * collecting lead q is that product (times c_p, applied by the caller); any other walk scores
 * 0.  The stream layout is that of the plain walk, so with b = 1 the paths and counts are the
 * plain walker's.  mode 0: cumulative-sum sampler on the modified dense rows Kb [nE][n][n]
 * (any positive multiple of p'); mode 1: alias tables of the modified rows [nE][n][pitch].
 * rho and bias are [nE][n].  Tallies as above; wsum[2 k] += sum of scores, wsum[2 k + 1] +=
 * sum of squared scores at energy k.
 */
static int walk_weighted_impl(int mode, const double *Kb, const uint32_t *thr,
                              const int32_t *alias, int64_t pitch, int32_t nE, int32_t n,
                              const double *rho, const double *bias, uint64_t seed,
                              uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                              uint64_t n_walkers, uint32_t max_steps, int64_t *tallies,
                              double *wsum)
{
    if (n < 3 || nE < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    const int32_t N = n - 2;
    const int32_t q = N + 1 - (int32_t)inject_lead;
    const uint32_t tag = (realization << 1) | inject_lead;
    for (int32_t k = 0; k < nE; ++k) {
        const double *rk = rho + (int64_t)k * n;
        const double *bk = bias + (int64_t)k * n;
        int64_t cL = 0, cR = 0, tr = 0, s1 = 0, s2 = 0;
        double sx = 0.0, sx2 = 0.0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : cL, cR, tr, s1, s2, sx, sx2)
        for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
            uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
            stream_t st;
            stream_init(&st, seed, w, (uint32_t)k, tag);
            int32_t s = N + (int32_t)inject_lead;
            uint32_t steps = 0;
            int outcome = -1;
            double ratio = 1.0;
            while (steps < max_steps) {
                uint32_t a, b;
                stream_pair(&st, steps, &a, &b);
                int32_t next;
                if (mode == 0) {
                    next = draw_cdf(Kb + ((int64_t)k * n + s) * (int64_t)n, n, a, b);
                } else {
                    uint32_t c = lemire_bucket(&st, steps, a, (uint32_t)n);
                    int64_t e = ((int64_t)k * n + s) * pitch + c;
                    next = (b < thr[e]) ? (int32_t)c : alias[e];
                }
                ++steps;
                if (next < N || next == q) ratio *= rk[s] / bk[next];
                if (next >= N) { outcome = next - N; break; }
                s = next;
            }
            if (outcome == 0) ++cL;
            else if (outcome == 1) ++cR;
            else ++tr;
            s1 += steps;
            s2 += (int64_t)steps * (int64_t)steps;
            if (outcome >= 0 && N + outcome == q) {
                sx += ratio;
                sx2 += ratio * ratio;
            }
        }
        tallies[5 * k + 0] += cL;
        tallies[5 * k + 1] += cR;
        tallies[5 * k + 2] += tr;
        tallies[5 * k + 3] += s1;
        tallies[5 * k + 4] += s2;
        wsum[2 * k] += sx;
        wsum[2 * k + 1] += sx2;
    }
    return 0;
}

int oracle_walk_weighted_cdf(const double *Kb, int32_t nE, int32_t n, const double *rho,
                             const double *bias, uint64_t seed, uint32_t realization,
                             uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                             uint32_t max_steps, int64_t *tallies, double *wsum)
{
    return walk_weighted_impl(0, Kb, NULL, NULL, 0, nE, n, rho, bias, seed, realization,
                              inject_lead, walker_begin, n_walkers, max_steps, tallies, wsum);
}

int oracle_walk_weighted_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch,
                               int32_t nE, int32_t n, const double *rho, const double *bias,
                               uint64_t seed, uint32_t realization, uint32_t inject_lead,
                               uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                               int64_t *tallies, double *wsum)
{
    if (pitch < n) return -1;
    return walk_weighted_impl(1, NULL, thr, alias, pitch, nE, n, rho, bias, seed, realization,
                              inject_lead, walker_begin, n_walkers, max_steps, tallies, wsum);
}

/*
 * Transition counts of the walks that reach the collecting lead q (the data of the
 * score-function gradient of Eq. (66)): the same walks as walk_impl; every walk that exits at
 * q adds one to counts[k][o][s] for each of its steps s -> o (s a probe or the injection row
 * N + p, o a probe or q), outcome-major.  Tallies as walk_impl.  mode 0: cdf on K [nE][n][n];
 * mode 1: alias tables [nE][n][pitch].
 */
static int walk_counts_impl(int mode, const double *K, const uint32_t *thr, const int32_t *alias,
                            int64_t pitch, int32_t nE, int32_t n, uint64_t seed,
                            uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                            uint64_t n_walkers, uint32_t max_steps, int64_t *tallies,
                            int64_t *counts)
{
    if (n < 3 || nE < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    const int32_t N = n - 2;
    const int32_t q = N + 1 - (int32_t)inject_lead;
    const uint32_t tag = (realization << 1) | inject_lead;
    for (int32_t k = 0; k < nE; ++k) {
        int64_t *ck = counts + (int64_t)k * n * n;
        int64_t cL = 0, cR = 0, tr = 0, s1 = 0, s2 = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : cL, cR, tr, s1, s2)
        for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
            const uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
            int outcome = -1;
            uint32_t steps = 0;
            for (int pass = 0; pass < 2; ++pass) {  /* pass 1 replays a walk that reached q */
                stream_t st;
                stream_init(&st, seed, w, (uint32_t)k, tag);
                int32_t s = N + (int32_t)inject_lead;
                steps = 0;
                outcome = -1;
                while (steps < max_steps) {
                    uint32_t a, b;
                    stream_pair(&st, steps, &a, &b);
                    int32_t next;
                    if (mode == 0) {
                        next = draw_cdf(K + ((int64_t)k * n + s) * (int64_t)n, n, a, b);
                    } else {
                        uint32_t c = lemire_bucket(&st, steps, a, (uint32_t)n);
                        int64_t e = ((int64_t)k * n + s) * pitch + c;
                        next = (b < thr[e]) ? (int32_t)c : alias[e];
                    }
                    ++steps;
                    if (pass == 1) {
#pragma omp atomic
                        ck[(int64_t)next * n + s] += 1;
                    }
                    if (next >= N) { outcome = next - N; break; }
                    s = next;
                }
                if (pass == 0 && !(outcome >= 0 && N + outcome == q)) break;
            }
            if (outcome == 0) ++cL;
            else if (outcome == 1) ++cR;
            else ++tr;
            s1 += steps;
            s2 += (int64_t)steps * (int64_t)steps;
        }
        tallies[5 * k + 0] += cL;
        tallies[5 * k + 1] += cR;
        tallies[5 * k + 2] += tr;
        tallies[5 * k + 3] += s1;
        tallies[5 * k + 4] += s2;
    }
    return 0;
}

int oracle_walk_counts_cdf(const double *K, int32_t nE, int32_t n, uint64_t seed,
                           uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                           uint64_t n_walkers, uint32_t max_steps, int64_t *tallies,
                           int64_t *counts)
{
    return walk_counts_impl(0, K, NULL, NULL, 0, nE, n, seed, realization, inject_lead,
                            walker_begin, n_walkers, max_steps, tallies, counts);
}

int oracle_walk_counts_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch,
                             int32_t nE, int32_t n, uint64_t seed, uint32_t realization,
                             uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                             uint32_t max_steps, int64_t *tallies, int64_t *counts)
{
    if (pitch < n) return -1;
    return walk_counts_impl(1, NULL, thr, alias, pitch, nE, n, seed, realization, inject_lead,
                            walker_begin, n_walkers, max_steps, tallies, counts);
}

/*
 * Interpolated walks (Sec. V A, "Interpolation"): walker w at fine energy f walks on the
 * mixture (1 - alpha_f) p(E_lo) + alpha_f p(E_hi) of the rows of two nodes lo = lo[f] and
 * hi = lo + 1 (hi = lo for the last node), alpha_f = alpha32[f] / 2^32.  Step n uses the
 * block with counter (n, w, f | 2^31, tag): words 0 and 1 as (a, b) of the chosen sampler,
 * word 2 picks the row of E_hi when below alpha32[f], else that of E_lo.  Lemire redraws use
 * counter (n, w, f | 2^31, tag | 2^31) and key (key0, key1 ^ r).  Tallies per fine energy.
 * mode 0: cumulative-sum sampler on K [nN][n][n]; mode 1: alias tables [nN][n][pitch].
 */
static int walk_interp_impl(int mode, const double *K, const uint32_t *thr, const int32_t *alias,
                            int64_t pitch, int32_t nN, int32_t n, const int32_t *lo,
                            const uint32_t *alpha32, int32_t nF, uint64_t seed,
                            uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                            uint64_t n_walkers, uint32_t max_steps, int64_t *tallies)
{
    if (n < 3 || nN < 1 || nF < 1 || nF > 0x7FFFFFFE || inject_lead > 1 ||
        realization >= (1u << 30))
        return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    for (int32_t f = 0; f < nF; ++f)
        if (lo[f] < 0 || lo[f] >= nN) return -1;
    const int32_t N = n - 2;
    const uint32_t tag = (realization << 1) | inject_lead;
    for (int32_t f = 0; f < nF; ++f) {
        const int32_t e_lo = lo[f], e_hi = lo[f] + 1 < nN ? lo[f] + 1 : lo[f];
        const uint32_t fe = (uint32_t)f | 0x80000000u;
        int64_t cL = 0, cR = 0, tr = 0, s1 = 0, s2 = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : cL, cR, tr, s1, s2)
        for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
            const uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
            stream_t st;
            stream_init(&st, seed, w, fe, tag);
            const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
            int32_t s = N + (int32_t)inject_lead;
            uint32_t steps = 0;
            int outcome = -1;
            while (steps < max_steps) {
                const uint32_t ctr[4] = {steps, w, fe, tag};
                uint32_t x[4];
                oracle_philox4x32_10(ctr, key, x);
                const int32_t e = x[2] < alpha32[f] ? e_hi : e_lo;
                int32_t next;
                if (mode == 0) {
                    next = draw_cdf(K + ((int64_t)e * n + s) * (int64_t)n, n, x[0], x[1]);
                } else {
                    const uint32_t c = lemire_bucket(&st, steps, x[0], (uint32_t)n);
                    const int64_t at = ((int64_t)e * n + s) * pitch + c;
                    next = (x[1] < thr[at]) ? (int32_t)c : alias[at];
                }
                ++steps;
                if (next >= N) { outcome = next - N; break; }
                s = next;
            }
            if (outcome == 0) ++cL;
            else if (outcome == 1) ++cR;
            else ++tr;
            s1 += steps;
            s2 += (int64_t)steps * (int64_t)steps;
        }
        tallies[5 * f + 0] += cL;
        tallies[5 * f + 1] += cR;
        tallies[5 * f + 2] += tr;
        tallies[5 * f + 3] += s1;
        tallies[5 * f + 4] += s2;
    }
    return 0;
}

int oracle_walk_interp_cdf(const double *K, int32_t nN, int32_t n, const int32_t *lo,
                           const uint32_t *alpha32, int32_t nF, uint64_t seed,
                           uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                           uint64_t n_walkers, uint32_t max_steps, int64_t *tallies)
{
    return walk_interp_impl(0, K, NULL, NULL, 0, nN, n, lo, alpha32, nF, seed, realization,
                            inject_lead, walker_begin, n_walkers, max_steps, tallies);
}

int oracle_walk_interp_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch, int32_t nN,
                             int32_t n, const int32_t *lo, const uint32_t *alpha32, int32_t nF,
                             uint64_t seed, uint32_t realization, uint32_t inject_lead,
                             uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                             int64_t *tallies)
{
    if (pitch < n) return -1;
    return walk_interp_impl(1, NULL, thr, alias, pitch, nN, n, lo, alpha32, nF, seed,
                            realization, inject_lead, walker_begin, n_walkers, max_steps,
                            tallies);
}

/*
 * Inelastic walks (Sec. II F, step 7'): after step 6' draws a probe i at energy E_n, the walk
 * draws its next energy E_n + Delta_k, k in [0, n_off), from the table `etab` and continues
 * from probe i's row at that energy.  etab[e][i][k] (uint64) holds cumulative thresholds on the
 * 2^32 scale: the first k with r < etab[e][i][k] is drawn (k = n_off - 1 if none is).  The walk
 * keeps the random stream of its injection energy e0 (block j of the step-6' words: counter
 * (j, w, e0, tag), Lemire redraws as above); the 32-bit word r of step n is word (n & 3) of
 * Philox(counter = (n >> 2, w, e0, tag), key = (~key0, key1)).  A drawn energy outside
 * [0, nE) ends the walk as truncated and sets *bad.  Tallies per injection energy (as above);
 * hist[r][e0][e] (int64, accumulated) counts the walks injected at e0 that exit at lead r
 * with energy index e.
 * mode 0: cumulative-sum sampler on K [nE][n][n]; mode 1: alias tables [nE][n][pitch].
 */
static int walk_inelastic_impl(int mode, const double *K, const uint32_t *thr,
                               const int32_t *alias, int64_t pitch, int32_t nE, int32_t n,
                               const uint64_t *etab, const int32_t *offsets, int32_t n_off,
                               uint64_t seed, uint32_t realization, uint32_t inject_lead,
                               uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                               int64_t *tallies, int64_t *hist, int32_t *bad)
{
    if (n < 3 || nE < 1 || n_off < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (walker_begin + n_walkers > 0x100000000ull) return -1;
    const int32_t N = n - 2;
    const uint32_t tag = (realization << 1) | inject_lead;
    int32_t any_bad = 0;
    for (int32_t e0 = 0; e0 < nE; ++e0) {
        int64_t cL = 0, cR = 0, tr = 0, s1 = 0, s2 = 0;
        int64_t *hL = hist + (int64_t)e0 * nE;
        int64_t *hR = hist + ((int64_t)nE + e0) * nE;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : cL, cR, tr, s1, s2) \
    reduction(| : any_bad)
        for (int64_t i = 0; i < (int64_t)n_walkers; ++i) {
            const uint32_t w = (uint32_t)(walker_begin + (uint64_t)i);
            stream_t st;
            stream_init(&st, seed, w, (uint32_t)e0, tag);
            const uint32_t ekey[2] = {~st.key[0], st.key[1]};
            uint32_t eblock = 0xffffffffu, ewords[4];
            int32_t s = N + (int32_t)inject_lead, e = e0;
            uint32_t steps = 0;
            int outcome = -1;
            while (steps < max_steps) {
                uint32_t a, b;
                stream_pair(&st, steps, &a, &b);
                int32_t next;
                if (mode == 0) {
                    next = draw_cdf(K + ((int64_t)e * n + s) * (int64_t)n, n, a, b);
                } else {
                    uint32_t c = lemire_bucket(&st, steps, a, (uint32_t)n);
                    int64_t x = ((int64_t)e * n + s) * pitch + c;
                    next = (b < thr[x]) ? (int32_t)c : alias[x];
                }
                const uint32_t n_step = steps++;
                if (next >= N) { outcome = next - N; break; }
                /* step 7': the energy of the next row */
                if (eblock != n_step >> 2) {
                    const uint32_t ctr[4] = {n_step >> 2, w, (uint32_t)e0, tag};
                    oracle_philox4x32_10(ctr, ekey, ewords);
                    eblock = n_step >> 2;
                }
                const uint32_t r = ewords[n_step & 3];
                const uint64_t *t = etab + ((int64_t)e * N + next) * n_off;
                int32_t k = 0;
                while (k < n_off - 1 && (uint64_t)r >= t[k]) ++k;
                const int32_t en = e + offsets[k];
                if (en < 0 || en >= nE) { any_bad = 1; break; }
                e = en;
                s = next;
            }
            if (outcome == 0) {
                ++cL;
#pragma omp atomic
                hL[e] += 1;
            } else if (outcome == 1) {
                ++cR;
#pragma omp atomic
                hR[e] += 1;
            } else {
                ++tr;
            }
            s1 += steps;
            s2 += (int64_t)steps * (int64_t)steps;
        }
        tallies[5 * e0 + 0] += cL;
        tallies[5 * e0 + 1] += cR;
        tallies[5 * e0 + 2] += tr;
        tallies[5 * e0 + 3] += s1;
        tallies[5 * e0 + 4] += s2;
    }
    if (bad) *bad = any_bad;
    return 0;
}

int oracle_walk_inelastic_cdf(const double *K, int32_t nE, int32_t n, const uint64_t *etab,
                              const int32_t *offsets, int32_t n_off, uint64_t seed,
                              uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                              uint64_t n_walkers, uint32_t max_steps, int64_t *tallies,
                              int64_t *hist, int32_t *bad)
{
    return walk_inelastic_impl(0, K, NULL, NULL, 0, nE, n, etab, offsets, n_off, seed,
                               realization, inject_lead, walker_begin, n_walkers, max_steps,
                               tallies, hist, bad);
}

int oracle_walk_inelastic_alias(const uint32_t *thr, const int32_t *alias, int64_t pitch,
                                int32_t nE, int32_t n, const uint64_t *etab,
                                const int32_t *offsets, int32_t n_off, uint64_t seed,
                                uint32_t realization, uint32_t inject_lead,
                                uint64_t walker_begin, uint64_t n_walkers, uint32_t max_steps,
                                int64_t *tallies, int64_t *hist, int32_t *bad)
{
    if (pitch < n) return -1;
    return walk_inelastic_impl(1, NULL, thr, alias, pitch, nE, n, etab, offsets, n_off, seed,
                               realization, inject_lead, walker_begin, n_walkers, max_steps,
                               tallies, hist, bad);
}

/*
 * Search for rejected bucket words: walkers w of [w_begin, w_begin + count) at energy index k
 * whose draw of step n_step over nout outcomes needs at least min_redraws redraws (Lemire's
 * rejection above).  Writes up to max_out walker indices, their redraw counts and their
 * accepted buckets (in increasing walker order) and returns how many walkers qualify in all.
 */
int64_t oracle_find_redraws(uint64_t seed, uint32_t realization, uint32_t inject_lead,
                            uint32_t k, uint32_t n_step, uint32_t nout, uint64_t w_begin,
                            uint64_t count, uint32_t min_redraws, uint32_t *out_w,
                            uint32_t *out_r, uint32_t *out_c, int64_t max_out)
{
    if (nout < 1 || inject_lead > 1 || realization >= (1u << 30)) return -1;
    if (w_begin + count > 0x100000000ull) return -1;
    const uint32_t tag = (realization << 1) | inject_lead;
    const uint32_t thresh = (uint32_t)(0u - nout) % nout;
    int64_t found = 0;
    const int64_t nblk = 4096;
    const int64_t blocks = ((int64_t)count + nblk - 1) / nblk;
#pragma omp parallel for schedule(static) ordered
    for (int64_t b = 0; b < blocks; ++b) {
        uint32_t hit_w[64], hit_r[64], hit_c[64];
        int nh = 0;
        const uint64_t i0 = (uint64_t)b * nblk;
        const uint64_t i1 = i0 + nblk < count ? i0 + nblk : count;
        for (uint64_t i = i0; i < i1; ++i) {
            stream_t st;
            stream_init(&st, seed, (uint32_t)(w_begin + i), k, tag);
            uint32_t a, bb;
            stream_pair(&st, n_step, &a, &bb);
            if ((uint32_t)((uint64_t)a * nout) >= thresh) continue;
            uint32_t r = 0;
            const uint32_t c = lemire_bucket_count(&st, n_step, a, nout, &r);
            if (r >= min_redraws && nh < 64) {
                hit_w[nh] = (uint32_t)(w_begin + i);
                hit_r[nh] = r;
                hit_c[nh] = c;
                ++nh;
            }
        }
#pragma omp ordered
        for (int h = 0; h < nh; ++h) {
            if (found < max_out) {
                out_w[found] = hit_w[h];
                out_r[found] = hit_r[h];
                out_c[found] = hit_c[h];
            }
            ++found;
        }
    }
    return found;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
