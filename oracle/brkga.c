/*
 * Oracle BRKGA operators and random numbers (test infrastructure only).
 *
 * Random draws come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11): a counter-based generator, so
 * any draw is a pure function of (counter, key) and both implementations can
 * produce the same stream without sharing state.
 *
 * Draw conventions (one Philox block = 4 words):
 *   uniform fp32 in [0,1)       u = (w >> 8) * 2^-24
 *   uniform int in [0, N)        (w * N) >> 32
 *   Bernoulli(rho)               (w >> 8) < floor(rho * 2^24)
 * Counter = {word-block index, individual or slot, generation, stream tag}.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

#define TAG_MUTANT  0x4D555441u /* mutant genes */
#define TAG_PARENT  0x50415245u /* parent choice */
#define TAG_CROSS   0x43524F53u /* crossover coin flips */
#define TAG_WARM    0x5741524Du /* warm-start perturbation */
#define TAG_RANDOM  0x52414E44u /* random initial individuals */

static void mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t draw(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t tag)
{
    /* word (a % 4) of block {a / 4, b, c, tag} */
    uint32_t ctr[4] = {a >> 2, b, c, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox(ctr, key, out);
    return out[a & 3];
}

static float unit24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

typedef struct { int64_t f; int32_t i; } ranked;

static int cmp_ranked(const void* a, const void* b)
{
    const ranked* x = a;
    const ranked* y = b;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

/*
 * One generation (Section 4.4.3): rank by fitness (ties by index), copy the
 * n_elite best unchanged, add n_mutant individuals of fresh U(0,1) genes, and
 * fill the rest by biased uniform crossover between an elite parent and a
 * non-elite parent, taking each gene from the elite one with probability rho.
 * Genes are the 'genes' priorities followed, when hint != NULL, by as many
 * vehicle hints; both halves go through the same operators.
 */
void orc_brkga_evolve(int32_t Np, int32_t genes, const float* prio, const float* hint,
                      const int64_t* fitness, int32_t n_elite, int32_t n_mutant,
                      uint32_t rho_thr24, uint64_t seed, uint32_t generation,
                      float* prio_out, float* hint_out, int32_t* rank_out)
{
    ranked* r = malloc((size_t)Np * sizeof(ranked));
    for (int32_t i = 0; i < Np; ++i) { r[i].f = fitness[i]; r[i].i = i; }
    qsort(r, (size_t)Np, sizeof(ranked), cmp_ranked);
    if (rank_out)
        for (int32_t i = 0; i < Np; ++i) rank_out[i] = r[i].i;
    const int32_t G = hint ? 2 * genes : genes;
    for (int32_t i = 0; i < Np; ++i) {
        float* dp = prio_out + (size_t)i * genes;
        float* dh = hint ? hint_out + (size_t)i * genes : NULL;
        if (i < n_elite) {
            int32_t s = r[i].i;
            memcpy(dp, prio + (size_t)s * genes, (size_t)genes * sizeof(float));
            if (hint) memcpy(dh, hint + (size_t)s * genes, (size_t)genes * sizeof(float));
        } else if (i < n_elite + n_mutant) {
            for (int32_t j = 0; j < G; ++j) {
                float u = unit24(draw(seed, (uint32_t)j, (uint32_t)i, generation, TAG_MUTANT));
                if (j < genes) dp[j] = u; else dh[j - genes] = u;
            }
        } else {
            uint32_t we = draw(seed, 0, (uint32_t)i, generation, TAG_PARENT);
            uint32_t wn = draw(seed, 1, (uint32_t)i, generation, TAG_PARENT);
            int32_t e = r[(int32_t)(((uint64_t)we * (uint64_t)n_elite) >> 32)].i;
            int32_t x = r[n_elite + (int32_t)(((uint64_t)wn * (uint64_t)(Np - n_elite)) >> 32)].i;
            for (int32_t j = 0; j < G; ++j) {
                uint32_t w = draw(seed, (uint32_t)j, (uint32_t)i, generation, TAG_CROSS);
                int32_t src = ((w >> 8) < rho_thr24) ? e : x;
                if (j < genes) dp[j] = prio[(size_t)src * genes + j];
                else dh[j - genes] = hint[(size_t)src * genes + (j - genes)];
            }
        }
    }
    free(r);
}

/*
 * Warm start (Section 4.4.4).  Each source solution is encoded by the seed
 * encoding: the op at 1-based position r of a route of L_v ops gets priority
 * (r-1)/L_v, and every op of vehicle v gets hint (v + 1/2)/m (the centre of
 * the hint interval that floor(m * alpha) maps to v); ops absent from the
 * solution get 0.  Source s contributes n_var[s] variants: variant 0 as
 * encoded, variant t > 0 with every gene moved by U(-0.03, 0.03) and clamped
 * into [0, 1).  Slots [0, n_warm) cycle through the variants of all sources
 * in order (source 0's first); the remaining slots are fresh U(0,1)
 * individuals.  The perturbation of gene j in variant t of source s draws
 * from counter (j / 4, t, s, 'WARM').
 */
static void encode(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end, float* ep, float* eh)
{
    const int n = I->n, m = I->m, G = 2 * n;
    for (int o = 0; o < G; ++o) { ep[o] = 0.0f; eh[o] = 0.0f; }
    for (int v = 0, s = 0; v < m; s = rt_end[v], ++v) {
        int L = rt_end[v] - s;
        for (int j = s; j < rt_end[v]; ++j) {
            int c = ops[j] >> 1, isP = ops[j] & 1;
            int o = 2 * (c - 1) + isP;
            ep[o] = (float)((double)(j - s) / (double)L);
            eh[o] = (float)(((double)v + 0.5) / (double)m);
        }
    }
}

void orc_brkga_warm_start_multi(const orc_inst* I, int32_t n_src, const uint16_t* ops, int64_t op_stride,
                                const uint16_t* rt_end, int64_t rt_stride, const int32_t* n_var, int32_t Np,
                                int32_t n_warm, uint64_t seed, float* prio_out, float* hint_out)
{
    const int n = I->n, G = 2 * n;
    int total = 0;
    for (int s = 0; s < n_src; ++s) total += n_var[s];
    float* ep = malloc((size_t)n_src * G * sizeof(float));
    float* eh = malloc((size_t)n_src * G * sizeof(float));
    for (int s = 0; s < n_src; ++s)
        encode(I, ops + (size_t)s * op_stride, rt_end + (size_t)s * rt_stride, ep + (size_t)s * G, eh + (size_t)s * G);
    for (int32_t i = 0; i < Np; ++i) {
        float* dp = prio_out + (size_t)i * G;
        float* dh = hint_out + (size_t)i * G;
        if (i < n_warm && total > 0) {
            int q = i % total, src = 0;
            while (q >= n_var[src]) q -= n_var[src++];
            const uint32_t var = (uint32_t)q;
            for (int j = 0; j < 2 * G; ++j) {
                float g = j < G ? ep[(size_t)src * G + j] : eh[(size_t)src * G + j - G];
                if (var) {
                    double u = (double)(draw(seed, (uint32_t)j, var, (uint32_t)src, TAG_WARM) >> 8) * (1.0 / 16777216.0);
                    double x = (double)g + (u * 0.06 - 0.03);
                    if (x < 0.0) x = 0.0;
                    g = (float)x;
                    if (g >= 1.0f) g = 0.99999994f;
                }
                if (j < G) dp[j] = g; else dh[j - G] = g;
            }
        } else {
            for (int j = 0; j < 2 * G; ++j) {
                float u = unit24(draw(seed, (uint32_t)j, (uint32_t)i, 0, TAG_RANDOM));
                if (j < G) dp[j] = u; else dh[j - G] = u;
            }
        }
    }
    free(ep); free(eh);
}

void orc_brkga_warm_start(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end,
                          int32_t Np, int32_t n_warm, int32_t n_variants, uint64_t seed,
                          float* prio_out, float* hint_out)
{
    orc_brkga_warm_start_multi(I, 1, ops, 0, rt_end, 0, &n_variants, Np, n_warm, seed, prio_out, hint_out);
}
