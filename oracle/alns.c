/*
 * Oracle ALNS (test infrastructure only; see oracle.h).
 *
 * Algorithm 1 of Section 4.2 (destroy/repair, simulated annealing, adaptive
 * operator weights), with the six destroy operators of Section 4.2.2 and the
 * four repair operators of Section 4.2.3, run for several independent chains
 * in lockstep so that the periodic best-solution import (Section 4.2.1, item 1)
 * happens at well-defined points.
 *
 * Readings of points the paper leaves open (each one is also what the GPU
 * implementation does):
 *  - every repair candidate is priced by the exact evaluator (not the
 *    paper's approximate two-pass timing); a candidate must have status 0;
 *  - insertion candidates of a customer: the drop slots (vehicle, position)
 *    ranked by detour d[a][c] + d[c][b] - d[a][b] (ties: vehicle, position),
 *    the best K_D of them, and for each the best K_P pickup slots ranked the
 *    same way on the route after the drop went in; K_D = K_P = 0 means all
 *    slots.  With a per-iteration budget B of tuples and q removed customers,
 *    T_c = max(1, B / (q(q+1)/2)), K_D = max(1, floor(sqrt(T_c))),
 *    K_P = max(1, T_c / K_D);
 *  - greedy inserts the customer whose best tuple has the lowest makespan;
 *    regret-k uses per-drop-vehicle options (the best tuple with that drop
 *    vehicle), regret = sum_{h=2..k} (c_h - c_1) with a missing option priced
 *    2^40, k = 2, 3 or m; ties go to the lower best cost, then the earlier
 *    customer in the removal list; a customer with no feasible tuple makes the
 *    repair (and the iteration's candidate) fail;
 *  - worst removal: gain = z(S) - z(S without c); ranks by gain (ties: lower
 *    customer), rank r drawn with weight floor(2^60 / r^6), without
 *    replacement;
 *  - Shaw: relatedness to a random seed customer, doubled to stay integer:
 *    18 d[seed][c] + 6 |T_drop(seed) - T_drop(c)| + 5 [drop vehicles differ]
 *    + 5 [pickup vehicles differ]; the seed and the q-1 most related;
 *  - cluster: a random centre and the q-1 customers with the smallest
 *    d[centre][c];
 *  - route: a random non-empty route, its customers in order of first
 *    appearance up to q; below q_min, topped up with the customers nearest
 *    (min d from a chosen one) to those chosen;
 *  - critical path: the vehicle with the latest return (ties: lower index),
 *    its customers by descending gain up to q; below q_min, topped up with
 *    the other customers by descending gain;
 *  - SA: a candidate with z' = z goes to the annealing test and exp(0) = 1
 *    accepts it; stagnation counts iterations since the last new best, and
 *    the reheat needs both stagnation >= limit and T < gate * T_init
 *    (Section 4.2.4); weights with zero attempts in a period stay unchanged;
 *  - exp in the annealing test is a fixed Taylor evaluation (det_exp) so that
 *    two implementations reach the same decisions;
 *  - import every import_interval iterations: each chain whose best is worse
 *    than the best over all chains (ties: lower chain) takes that solution as
 *    both its current and its best.
 * Random draws: Philox4x32-10, word (a % 4) of block {a / 4, iteration, chain,
 * 'ALNS'}: a = 0 destroy roulette, 1 repair roulette, 2 q, 8 annealing,
 * 16.. destroy operator.
 */
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define TAG_ALNS 0x414C4E53u
#define BIGC (1LL << 40)
#define ND 6
#define NR 4

typedef struct {
    int L;
    uint16_t* ops;   /* capacity 2n */
    uint16_t* rt;    /* m */
} sol_t;

static uint32_t adraw(uint64_t seed, uint32_t a, uint32_t it, uint32_t chain)
{
    uint32_t ctr[4] = {a >> 2, it, chain, TAG_ALNS};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox(ctr, key, out);
    return out[a & 3];
}

static double unit_d(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }
static int uint_below(uint32_t w, int nval) { return (int)(((uint64_t)w * (uint64_t)nval) >> 32); }

double orc_det_exp(double x)
{
    /* exp(x) for x <= 0: x = k ln 2 + r, |r| <= ln2 / 2, Taylor series of
     * degree 16 for e^r, then scale by 2^k. */
    if (x < -745.0) return 0.0;
    const double LN2 = 0.6931471805599453;
    double k = floor(x / LN2 + 0.5);
    double r = x - k * LN2;
    double s = 1.0, term = 1.0;
    for (int i = 1; i <= 16; ++i) {
        term = term * (r / (double)i);
        s = s + term;
    }
    return ldexp(s, (int)k);
}

static void sol_alloc(sol_t* s, int n, int m)
{
    s->L = 0;
    s->ops = malloc((size_t)(2 * n + 2) * sizeof(uint16_t));
    s->rt = calloc((size_t)m, sizeof(uint16_t));
}
static void sol_free(sol_t* s) { free(s->ops); free(s->rt); }
static void sol_copy(sol_t* d, const sol_t* s, int m)
{
    d->L = s->L;
    memcpy(d->ops, s->ops, (size_t)s->L * sizeof(uint16_t));
    memcpy(d->rt, s->rt, (size_t)m * sizeof(uint16_t));
}
static int rstart(const sol_t* s, int v) { return v ? s->rt[v - 1] : 0; }
static int rlen(const sol_t* s, int v) { return s->rt[v] - rstart(s, v); }

static void sol_remove(const sol_t* s, const unsigned char* gone, int m, sol_t* out)
{
    int w = 0;
    for (int v = 0; v < m; ++v) {
        for (int j = rstart(s, v); j < s->rt[v]; ++j)
            if (!gone[s->ops[j] >> 1]) out->ops[w++] = s->ops[j];
        out->rt[v] = (uint16_t)w;
    }
    out->L = w;
}

static void sol_insert(const sol_t* s, const orc_tuple* t, int m, sol_t* out)
{
    int w = 0;
    uint16_t tmp[65536 / 2];
    for (int v = 0; v < m; ++v) {
        int len = 0;
        for (int j = rstart(s, v); j < s->rt[v]; ++j) tmp[len++] = s->ops[j];
        if (v == t->vD) {
            memmove(tmp + t->pD + 1, tmp + t->pD, (size_t)(len - t->pD) * sizeof(uint16_t));
            tmp[t->pD] = (uint16_t)(t->c << 1);
            ++len;
        }
        if (v == t->vP) {
            memmove(tmp + t->pP + 1, tmp + t->pP, (size_t)(len - t->pP) * sizeof(uint16_t));
            tmp[t->pP] = (uint16_t)((t->c << 1) | 1);
            ++len;
        }
        memcpy(out->ops + w, tmp, (size_t)len * sizeof(uint16_t));
        w += len;
        out->rt[v] = (uint16_t)w;
    }
    out->L = w;
}

static uint32_t sol_eval(const orc_inst* I, const sol_t* s, int32_t* mk, int64_t* times)
{
    return orc_eval(I, 1, s->ops, s->rt, mk, times);
}

/* ------------------------------------------------------------------ enumeration */
typedef struct { long long det; int v, p; } slot_t;

static int cmp_slot(const void* a, const void* b)
{
    const slot_t* x = a;
    const slot_t* y = b;
    if (x->det != y->det) return x->det < y->det ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return (x->p > y->p) - (x->p < y->p);
}

static long long detour(const orc_inst* I, int a, int c, int b)
{
    const int N1 = I->n + 1;
    return (long long)I->d[a * N1 + c] + I->d[c * N1 + b] - I->d[a * N1 + b];
}

/* Candidate tuples of customer c against partial solution s, in the order
 * described in the header.  Returns the count; tuples written to out. */
static int enumerate_tuples(const orc_inst* I, const sol_t* s, int c, int KD, int KP, orc_tuple* out,
                            slot_t* dbuf, slot_t* pbuf)
{
    const int m = I->m;
    int nd = 0;
    for (int v = 0; v < m; ++v) {
        const int s0 = rstart(s, v), len = rlen(s, v);
        for (int p = 0; p <= len; ++p) {
            int a = p > 0 ? s->ops[s0 + p - 1] >> 1 : 0;
            int b = p < len ? s->ops[s0 + p] >> 1 : 0;
            dbuf[nd].det = detour(I, a, c, b);
            dbuf[nd].v = v;
            dbuf[nd].p = p;
            ++nd;
        }
    }
    qsort(dbuf, (size_t)nd, sizeof(slot_t), cmp_slot);
    if (KD > 0 && nd > KD) nd = KD;
    int T = 0;
    for (int i = 0; i < nd; ++i) {
        const int vD = dbuf[i].v, pD = dbuf[i].p;
        int np = 0;
        for (int v = 0; v < m; ++v) {
            const int s0 = rstart(s, v), len = rlen(s, v);
            if (v == vD) {
                /* route after the drop: base[0..pD) c base[pD..len) */
                for (int p = pD + 1; p <= len + 1; ++p) {
                    int a = (p - 1 == pD) ? c : s->ops[s0 + p - 2] >> 1;
                    int b = (p <= len) ? s->ops[s0 + p - 1] >> 1 : 0;
                    pbuf[np].det = detour(I, a, c, b);
                    pbuf[np].v = v;
                    pbuf[np].p = p;
                    ++np;
                }
            } else {
                for (int p = 0; p <= len; ++p) {
                    int a = p > 0 ? s->ops[s0 + p - 1] >> 1 : 0;
                    int b = p < len ? s->ops[s0 + p] >> 1 : 0;
                    pbuf[np].det = detour(I, a, c, b);
                    pbuf[np].v = v;
                    pbuf[np].p = p;
                    ++np;
                }
            }
        }
        qsort(pbuf, (size_t)np, sizeof(slot_t), cmp_slot);
        if (KP > 0 && np > KP) np = KP;
        for (int k2 = 0; k2 < np; ++k2) {
            out[T].c = (uint16_t)c;
            out[T].vD = (uint8_t)vD;
            out[T].pD = (uint16_t)pD;
            out[T].vP = (uint8_t)pbuf[k2].v;
            out[T].pP = (uint16_t)pbuf[k2].p;
            ++T;
        }
    }
    return T;
}

/* ------------------------------------------------------------------ destroy */
typedef struct { long long key; int c; } kc_t;

static int cmp_kc(const void* a, const void* b)
{
    const kc_t* x = a;
    const kc_t* y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->c > y->c) - (x->c < y->c);
}

/* gain[c] = z(S) - z(S without c) */
static void removal_gains(const orc_inst* I, const sol_t* S, int32_t z, long long* gain, sol_t* tmp,
                          unsigned char* gone)
{
    const int n = I->n, m = I->m;
    for (int c = 1; c <= n; ++c) {
        memset(gone, 0, (size_t)n + 1);
        gone[c] = 1;
        sol_remove(S, gone, m, tmp);
        int32_t zc;
        sol_eval(I, tmp, &zc, NULL);
        gain[c] = (long long)z - zc;
    }
    memset(gone, 0, (size_t)n + 1);
}

/* Returns the number of removed customers written to rem (in order).
 * Candidate `cand` of a learned proposal draws its random words at counter
 * offsets 16 + 4096 cand + i (cand 0: the plain operator's draws). */
static int destroy(const orc_inst* I, int op, const sol_t* S, int32_t z, int q, int q_min, uint64_t seed,
                   uint32_t it, uint32_t chain, int cand, int* rem, sol_t* tmp, unsigned char* gone)
{
    const int n = I->n, m = I->m, N1 = n + 1;
    const uint32_t db = 16u + 4096u * (uint32_t)cand;
    int cnt = 0;
    if (q > n) q = n;
    if (op == 0) {                                   /* random: partial Fisher-Yates */
        int* a = malloc((size_t)n * sizeof(int));
        for (int i = 0; i < n; ++i) a[i] = i + 1;
        for (int i = 0; i < q; ++i) {
            int j = i + uint_below(adraw(seed, db + i, it, chain), n - i);
            int x = a[i]; a[i] = a[j]; a[j] = x;
            rem[cnt++] = a[i];
        }
        free(a);
    } else if (op == 1 || op == 5) {                 /* worst, critical path */
        long long* gain = malloc((size_t)(n + 1) * sizeof(long long));
        removal_gains(I, S, z, gain, tmp, gone);
        kc_t* k = malloc((size_t)n * sizeof(kc_t));
        if (op == 1) {
            for (int c = 1; c <= n; ++c) { k[c - 1].key = -gain[c]; k[c - 1].c = c; }
            qsort(k, (size_t)n, sizeof(kc_t), cmp_kc);
            /* rank r = index + 1 drawn with weight floor(2^60 / r^6) */
            unsigned long long* w = malloc((size_t)n * sizeof(unsigned long long));
            for (int i = 0; i < n; ++i) {
                unsigned long long r = (unsigned long long)(i + 1);
                w[i] = r <= 1024 ? (1ULL << 60) / (r * r * r * r * r * r) : 0ULL;
            }
            for (int s = 0; s < q; ++s) {
                unsigned long long tot = 0;
                for (int i = 0; i < n; ++i) tot += w[i];
                if (tot == 0) break;
                unsigned long long target =
                    (unsigned long long)(((unsigned __int128)adraw(seed, db + s, it, chain) * tot) >> 32);
                unsigned long long acc = 0;
                int pick = -1;
                for (int i = 0; i < n; ++i) {
                    acc += w[i];
                    if (w[i] && target < acc) { pick = i; break; }
                }
                rem[cnt++] = k[pick].c;
                w[pick] = 0;
            }
            free(w);
        } else {
            /* bottleneck vehicle: latest return */
            int32_t mk;
            int64_t* times = malloc((size_t)(S->L + 1) * sizeof(int64_t));
            sol_eval(I, S, &mk, times);
            int bv = -1;
            long long bret = -1;
            for (int v = 0; v < m; ++v) {
                if (rlen(S, v) == 0) continue;
                int last = S->rt[v] - 1;
                long long ret = times[last] + I->d[(S->ops[last] >> 1) * N1];
                if (ret > bret) { bret = ret; bv = v; }
            }
            free(times);
            unsigned char* on = calloc((size_t)n + 1, 1);
            for (int j = rstart(S, bv); j < S->rt[bv]; ++j) on[S->ops[j] >> 1] = 1;
            int nk = 0;
            for (int c = 1; c <= n; ++c)
                if (on[c]) { k[nk].key = -gain[c]; k[nk].c = c; ++nk; }
            qsort(k, (size_t)nk, sizeof(kc_t), cmp_kc);
            for (int i = 0; i < nk && cnt < q; ++i) rem[cnt++] = k[i].c;
            if (cnt < q_min) {
                nk = 0;
                for (int c = 1; c <= n; ++c)
                    if (!on[c]) { k[nk].key = -gain[c]; k[nk].c = c; ++nk; }
                qsort(k, (size_t)nk, sizeof(kc_t), cmp_kc);
                for (int i = 0; i < nk && cnt < q_min; ++i) rem[cnt++] = k[i].c;
            }
            free(on);
        }
        free(k);
        free(gain);
    } else if (op == 2) {                            /* Shaw */
        int32_t mk;
        int64_t* times = malloc((size_t)(S->L + 1) * sizeof(int64_t));
        sol_eval(I, S, &mk, times);
        long long* td = malloc((size_t)(n + 1) * sizeof(long long));
        int* dv = malloc((size_t)(n + 1) * sizeof(int));
        int* pv = malloc((size_t)(n + 1) * sizeof(int));
        for (int v = 0; v < m; ++v)
            for (int j = rstart(S, v); j < S->rt[v]; ++j) {
                int c = S->ops[j] >> 1;
                if (S->ops[j] & 1) pv[c] = v;
                else { dv[c] = v; td[c] = times[j]; }
            }
        int seedc = 1 + uint_below(adraw(seed, db, it, chain), n);
        kc_t* k = malloc((size_t)n * sizeof(kc_t));
        int nk = 0;
        for (int c = 1; c <= n; ++c) {
            if (c == seedc) continue;
            long long dt = td[seedc] - td[c];
            if (dt < 0) dt = -dt;
            k[nk].key = 18LL * I->d[seedc * N1 + c] + 6 * dt + 5 * (dv[seedc] != dv[c]) + 5 * (pv[seedc] != pv[c]);
            k[nk].c = c;
            ++nk;
        }
        qsort(k, (size_t)nk, sizeof(kc_t), cmp_kc);
        rem[cnt++] = seedc;
        for (int i = 0; i < nk && cnt < q; ++i) rem[cnt++] = k[i].c;
        free(k); free(times); free(td); free(dv); free(pv);
    } else if (op == 3) {                            /* cluster */
        int cen = 1 + uint_below(adraw(seed, db, it, chain), n);
        kc_t* k = malloc((size_t)n * sizeof(kc_t));
        int nk = 0;
        for (int c = 1; c <= n; ++c) {
            if (c == cen) continue;
            k[nk].key = I->d[cen * N1 + c];
            k[nk].c = c;
            ++nk;
        }
        qsort(k, (size_t)nk, sizeof(kc_t), cmp_kc);
        rem[cnt++] = cen;
        for (int i = 0; i < nk && cnt < q; ++i) rem[cnt++] = k[i].c;
        free(k);
    } else {                                         /* route */
        int nonempty = 0;
        for (int v = 0; v < m; ++v) nonempty += rlen(S, v) > 0;
        int pickv = uint_below(adraw(seed, db, it, chain), nonempty);
        int v = 0;
        for (int seen = -1; v < m; ++v)
            if (rlen(S, v) > 0 && ++seen == pickv) break;
        unsigned char* in = calloc((size_t)n + 1, 1);
        for (int j = rstart(S, v); j < S->rt[v] && cnt < q; ++j) {
            int c = S->ops[j] >> 1;
            if (!in[c]) { in[c] = 1; rem[cnt++] = c; }
        }
        if (cnt < q_min) {
            kc_t* k = malloc((size_t)n * sizeof(kc_t));
            int nk = 0;
            for (int c = 1; c <= n; ++c) {
                if (in[c]) continue;
                long long best = LLONG_MAX;
                for (int i = 0; i < cnt; ++i) {
                    long long x = I->d[rem[i] * N1 + c];
                    if (x < best) best = x;
                }
                k[nk].key = best;
                k[nk].c = c;
                ++nk;
            }
            qsort(k, (size_t)nk, sizeof(kc_t), cmp_kc);
            for (int i = 0; i < nk && cnt < q_min; ++i) rem[cnt++] = k[i].c;
            free(k);
        }
        free(in);
    }
    return cnt;
}

/* ------------------------------------------------------------------ local search */
#define LS_MAX_CAND 256   /* candidates per pass: the first 256 in order */
/* One pass of a periodic local search (Section 4.2.6) on the current
 * solution S.  kind 0, pickup repositioning: every pickup on a vehicle that
 * returns within 5% of the makespan (20 f_v >= 19 z), in route order, may
 * move to any pickup slot of any vehicle (after its drop on the drop's
 * vehicle).  kind 1, cross-agent relocation: every customer with an op on
 * the bottleneck vehicle (latest return, lowest index on ties), in order of
 * first appearance, may move both ops to another vehicle.  Only the first
 * 256 candidates are tried.  Candidate slots
 * are ranked by detour as in the repair (reading 22) with T = max(1, budget
 * / #candidates) tuples per candidate (relocation: K_D = max(1, floor(sqrt
 * T)) drop slots, K_P = max(1, T / K_D) pickup slots on the drop's vehicle).
 * The exactly evaluated feasible move with the lowest makespan (ties: earlier
 * candidate, then earlier tuple) replaces S if it is strictly better.
 * Returns 1 if S improved. */
static int ls_pass(const orc_inst* I, int kind, int budget, sol_t* S, int32_t* z, sol_t* base, sol_t* cand,
                   slot_t* dbuf, slot_t* pbuf, int* cands, unsigned char* gone)
{
    const int n = I->n, m = I->m;
    int64_t* times = malloc((size_t)(S->L + 1) * sizeof(int64_t));
    int32_t zz;
    sol_eval(I, S, &zz, times);
    long long fin[64];
    for (int v = 0; v < m; ++v) {
        const int e = S->rt[v];
        fin[v] = rlen(S, v) > 0 ? times[e - 1] + I->d[(S->ops[e - 1] >> 1) * (n + 1)] : 0;
    }
    free(times);
    int nc = 0, b = 0;
    for (int v = 1; v < m; ++v)
        if (fin[v] > fin[b]) b = v;
    memset(gone, 0, (size_t)n + 1);
    if (kind == 0) {
        for (int v = 0; v < m; ++v) {
            if (20 * fin[v] < 19 * (long long)zz) continue;
            for (int j = rstart(S, v); j < S->rt[v]; ++j)
                if (S->ops[j] & 1) cands[nc++] = S->ops[j] >> 1;
        }
    } else {
        for (int j = rstart(S, b); j < S->rt[b]; ++j) {
            const int c = S->ops[j] >> 1;
            if (!gone[c]) {
                gone[c] = 1;
                cands[nc++] = c;
            }
        }
        memset(gone, 0, (size_t)n + 1);
    }
    if (nc > LS_MAX_CAND) nc = LS_MAX_CAND;
    if (nc == 0) return 0;
    const long long T = budget / nc > 1 ? budget / nc : 1;
    int32_t best_mk = zz;
    int best_i = -1;
    orc_tuple best_t = {0, 0, 0, 0, 0};
    for (int i = 0; i < nc; ++i) {
        const int c = cands[i];
        gone[c] = 1;
        sol_remove(S, gone, m, base);
        gone[c] = 0;
        int cnt = 0;
        orc_tuple tl;
        tl.c = (uint16_t)c;
        if (kind == 0) {
            /* the drop keeps its vehicle and position (removing the pickup,
             * which follows it on its own route, shifts nothing before it) */
            int vD = 0, pD = 0;
            for (int v = 0; v < m; ++v)
                for (int j = rstart(S, v); j < S->rt[v]; ++j)
                    if (S->ops[j] == (uint16_t)(c << 1)) { vD = v; pD = j - rstart(S, v); }
            int np = 0;
            for (int v = 0; v < m; ++v) {
                const int s0 = rstart(base, v), len = rlen(base, v);
                if (v == vD) {
                    for (int p = pD + 1; p <= len + 1; ++p) {
                        int a = (p - 1 == pD) ? c : base->ops[s0 + p - 2] >> 1;
                        int bb = (p <= len) ? base->ops[s0 + p - 1] >> 1 : 0;
                        pbuf[np].det = detour(I, a, c, bb); pbuf[np].v = v; pbuf[np].p = p; ++np;
                    }
                } else {
                    for (int p = 0; p <= len; ++p) {
                        int a = p > 0 ? base->ops[s0 + p - 1] >> 1 : 0;
                        int bb = p < len ? base->ops[s0 + p] >> 1 : 0;
                        pbuf[np].det = detour(I, a, c, bb); pbuf[np].v = v; pbuf[np].p = p; ++np;
                    }
                }
            }
            qsort(pbuf, (size_t)np, sizeof(slot_t), cmp_slot);
            if (np > T) np = (int)T;
            for (int k = 0; k < np; ++k, ++cnt) {
                tl.vD = (uint8_t)vD; tl.pD = (uint16_t)pD; tl.vP = (uint8_t)pbuf[k].v; tl.pP = (uint16_t)pbuf[k].p;
                sol_insert(base, &tl, m, cand);
                int32_t mk;
                if (sol_eval(I, cand, &mk, NULL) == 0 && mk < best_mk) { best_mk = mk; best_i = i; best_t = tl; }
            }
        } else {
            int KD = (int)floor(sqrt((double)T));
            if (KD < 1) KD = 1;
            int KP = (int)(T / KD);
            if (KP < 1) KP = 1;
            int nd = 0;
            for (int v = 0; v < m; ++v) {
                if (v == b) continue;
                const int s0 = rstart(base, v), len = rlen(base, v);
                for (int p = 0; p <= len; ++p) {
                    int a = p > 0 ? base->ops[s0 + p - 1] >> 1 : 0;
                    int bb = p < len ? base->ops[s0 + p] >> 1 : 0;
                    dbuf[nd].det = detour(I, a, c, bb); dbuf[nd].v = v; dbuf[nd].p = p; ++nd;
                }
            }
            qsort(dbuf, (size_t)nd, sizeof(slot_t), cmp_slot);
            if (nd > KD) nd = KD;
            for (int di = 0; di < nd; ++di) {
                const int vD = dbuf[di].v, pD = dbuf[di].p;
                const int s0 = rstart(base, vD), len = rlen(base, vD);
                int np = 0;
                for (int p = pD + 1; p <= len + 1; ++p) {
                    int a = (p - 1 == pD) ? c : base->ops[s0 + p - 2] >> 1;
                    int bb = (p <= len) ? base->ops[s0 + p - 1] >> 1 : 0;
                    pbuf[np].det = detour(I, a, c, bb); pbuf[np].v = vD; pbuf[np].p = p; ++np;
                }
                qsort(pbuf, (size_t)np, sizeof(slot_t), cmp_slot);
                if (np > KP) np = KP;
                for (int k = 0; k < np; ++k, ++cnt) {
                    tl.vD = (uint8_t)vD; tl.pD = (uint16_t)pD; tl.vP = (uint8_t)vD; tl.pP = (uint16_t)pbuf[k].p;
                    sol_insert(base, &tl, m, cand);
                    int32_t mk;
                    if (sol_eval(I, cand, &mk, NULL) == 0 && mk < best_mk) { best_mk = mk; best_i = i; best_t = tl; }
                }
            }
        }
        (void)cnt;
    }
    if (best_i < 0) return 0;
    gone[cands[best_i]] = 1;
    sol_remove(S, gone, m, base);
    gone[cands[best_i]] = 0;
    sol_insert(base, &best_t, m, S);
    *z = best_mk;
    return 1;
}

/* Up to three passes of one kind; returns 1 if S improved. */
static int local_search(const orc_inst* I, int kind, int budget, sol_t* S, int32_t* z, sol_t* base, sol_t* cand,
                        slot_t* dbuf, slot_t* pbuf, int* cands, unsigned char* gone)
{
    int any = 0;
    for (int pass = 0; pass < 3; ++pass) {
        if (!ls_pass(I, kind, budget, S, z, base, cand, dbuf, pbuf, cands, gone)) break;
        any = 1;
    }
    return any;
}

/* ------------------------------------------------------------------ repair */
/* Returns 1 on success (S complete), 0 if some customer had no feasible tuple. */
static int repair(const orc_inst* I, int op, sol_t* S, const int* rem, int nrem, int KD, int KP,
                  orc_tuple* tbuf, slot_t* dbuf, slot_t* pbuf, sol_t* tmp, int32_t* zout, int* order)
{
    const int m = I->m;
    int kreg = op == 1 ? 2 : op == 2 ? 3 : m;
    int* left = malloc((size_t)nrem * sizeof(int));
    memcpy(left, rem, (size_t)nrem * sizeof(int));
    int nleft = nrem;
    long long* opt = malloc((size_t)m * sizeof(long long));
    int ok = 1;
    while (nleft > 0) {
        int best_i = -1;
        long long best_c1 = 0, best_reg = 0;
        orc_tuple best_t;
        memset(&best_t, 0, sizeof best_t);
        for (int i = 0; i < nleft; ++i) {
            int c = left[i];
            int T = enumerate_tuples(I, S, c, KD, KP, tbuf, dbuf, pbuf);
            long long c1 = LLONG_MAX;
            int t1 = -1;
            for (int v = 0; v < m; ++v) opt[v] = BIGC;
            for (int t = 0; t < T; ++t) {
                sol_insert(S, &tbuf[t], m, tmp);
                int32_t mk;
                uint32_t st = sol_eval(I, tmp, &mk, NULL);
                if (st != 0) continue;
                if (mk < c1) { c1 = mk; t1 = t; }
                if (mk < opt[tbuf[t].vD]) opt[tbuf[t].vD] = mk;
            }
            if (t1 < 0) { ok = 0; break; }
            long long reg = 0;
            if (op != 0) {
                /* sort per-vehicle options ascending (m is small) */
                for (int a = 1; a < m; ++a)
                    for (int b = a; b > 0 && opt[b] < opt[b - 1]; --b) {
                        long long x = opt[b]; opt[b] = opt[b - 1]; opt[b - 1] = x;
                    }
                for (int h = 1; h < kreg && h < m; ++h) reg += opt[h] - opt[0];
                for (int h = m; h < kreg; ++h) reg += BIGC - opt[0];
            }
            int better;
            if (best_i < 0) better = 1;
            else if (op == 0) better = c1 < best_c1;
            else better = reg > best_reg || (reg == best_reg && c1 < best_c1);
            if (better) { best_i = i; best_c1 = c1; best_reg = reg; best_t = tbuf[t1]; }
        }
        if (!ok) break;
        sol_insert(S, &best_t, m, tmp);
        sol_copy(S, tmp, m);
        *zout = (int32_t)best_c1;
        if (order) order[nrem - nleft] = left[best_i];
        /* keep the removal-list order of the customers still waiting */
        memmove(left + best_i, left + best_i + 1, (size_t)(nleft - best_i - 1) * sizeof(int));
        --nleft;
    }
    free(left);
    free(opt);
    return ok;
}

/* ------------------------------------------------------------------ driver */
static int roulette(const double* w, int nops, uint32_t mask, double u)
{
    double tot = 0.0;
    for (int i = 0; i < nops; ++i)
        if (mask & (1u << i)) tot = tot + w[i];
    const double target = u * tot;
    double acc = 0.0;
    int last = -1;
    for (int i = 0; i < nops; ++i) {
        if (!(mask & (1u << i))) continue;
        acc = acc + w[i];
        last = i;
        if (target < acc) return i;
    }
    return last;
}

/* Slots per removed customer under a budget of tuples per iteration:
 * T_c = max(1, B / (q(q+1)/2)) tuples for each of the q(q+1)/2 customer
 * evaluations of a repair, K_D = max(1, floor(sqrt(T_c))) drop slots and
 * K_P = max(1, T_c / K_D) pickup slots per drop; B = 0 means every slot. */
static void budget_split(int budget, int nrem, int* KD, int* KP)
{
    *KD = 0;
    *KP = 0;
    if (budget <= 0) return;
    long long tc = (long long)budget / ((long long)nrem * (nrem + 1) / 2);
    if (tc < 1) tc = 1;
    *KD = (int)floor(sqrt((double)tc));
    if (*KD < 1) *KD = 1;
    *KP = (int)(tc / *KD);
    if (*KP < 1) *KP = 1;
}

void orc_alns_qrange(int n, int* q_min, int* q_max)
{
    int qmax = n / 20;              /* floor(0.05 n) */
    if (qmax < 4) qmax = 4;
    int qmin = qmax / 2;
    if (qmin < 4) qmin = 4;
    *q_min = qmin;
    *q_max = qmax;
}

typedef struct {
    sol_t S, B;
    orc_alns_chain k;   /* the scalars Algorithm 1 keeps per chain */
} chain_t;

/* Algorithm 1 after the repair of iteration it (0-based) of one chain:
 * attempts of the two chosen operators, the acceptance test (an improving
 * candidate always, a new best with the extra sigma1 - sigma2, otherwise
 * annealing with probability exp(-(z' - z) / T) against the uniform u in
 * [0, 1)), cooling, the stagnation counter and the gated reheat
 * (Section 4.2.4), and the weight update every tau iterations (Section 4.2.1,
 * adaptive scoring): w = max(w_min, (1 - r) w + r s / a), unchanged when an
 * operator had no attempt.  A failed repair (repaired = 0) is not accepted.
 * Returns 0 rejected, 1 improving, 2 new best, 3 accepted by annealing. */
int32_t orc_alns_update(const orc_alns_params* P, orc_alns_chain* c, int32_t di, int32_t ri, int32_t repaired,
                        int32_t zn, double u, int64_t it)
{
    int accepted = 0;
    c->aD[di]++;
    c->aR[ri]++;
    if (repaired) {
        if (zn < c->z) {
            c->z = zn;
            c->sD[di] += P->sigma2;
            c->sR[ri] += P->sigma2;
            accepted = 1;
            if (zn < c->zb) {
                c->zb = zn;
                c->sD[di] += P->sigma1 - P->sigma2;
                c->sR[ri] += P->sigma1 - P->sigma2;
                c->stag = 0;
                accepted = 2;
            }
        } else {
            const double pacc = orc_det_exp(-((double)zn - (double)c->z) / c->T);
            if (u < pacc) {
                c->z = zn;
                c->sD[di] += P->sigma3;
                c->sR[ri] += P->sigma3;
                accepted = 3;
            }
        }
    }
    c->T = P->alpha * c->T;
    c->stag += 1;
    if (c->stag >= P->stag_limit && c->T < P->gate * c->T_init) {
        c->T = P->reheat * P->T0 * (double)c->zb;
        c->stag = 0;
    }
    if ((it + 1) % P->tau == 0) {
        for (int i = 0; i < ND; ++i) {
            if (c->aD[i] > 0) {
                double w = (1.0 - P->r) * c->wD[i] + P->r * ((double)c->sD[i] / (double)c->aD[i]);
                c->wD[i] = w > P->w_min ? w : P->w_min;
            }
            c->sD[i] = 0;
            c->aD[i] = 0;
        }
        for (int i = 0; i < NR; ++i) {
            if (c->aR[i] > 0) {
                double w = (1.0 - P->r) * c->wR[i] + P->r * ((double)c->sR[i] / (double)c->aR[i]);
                c->wR[i] = w > P->w_min ? w : P->w_min;
            }
            c->sR[i] = 0;
            c->aR[i] = 0;
        }
    }
    return accepted;
}

/* chain0: the first chain's index in the random-draw counters (chains of
 * one instance in a state that holds several instances are numbered on from
 * the earlier instances' chains). */
int32_t orc_alns_run_ex(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                        uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                        uint16_t* best_rt, int32_t* best_mk, int64_t* trace, uint32_t chain0, int32_t* cur_mk,
                        double* fstate)
{
    const int n = I->n, m = I->m;
    int q_min = P->q_min, q_max = P->q_max;
    if (q_min <= 0 || q_max <= 0) orc_alns_qrange(n, &q_min, &q_max);
    if (q_max > n) q_max = n;
    if (q_min > q_max) q_min = q_max;
    chain_t* C = calloc((size_t)chains, sizeof(chain_t));
    sol_t work, tmp, tmp2;
    sol_alloc(&work, n, m);
    sol_alloc(&tmp, n, m);
    sol_alloc(&tmp2, n, m);
    const int maxslots = 2 * n + m + 2;
    slot_t* dbuf = malloc((size_t)maxslots * sizeof(slot_t));
    slot_t* pbuf = malloc((size_t)maxslots * sizeof(slot_t));
    orc_tuple* tbuf = malloc((size_t)maxslots * (size_t)maxslots * sizeof(orc_tuple) > (1u << 28)
                                 ? (size_t)maxslots * 64 * sizeof(orc_tuple)
                                 : (size_t)maxslots * (size_t)maxslots * sizeof(orc_tuple));
    int* rem = malloc((size_t)(n + 1) * sizeof(int));
    unsigned char* gone = calloc((size_t)n + 1, 1);
    const uint32_t dmask = P->op_mask & 0x3Fu, rmask = (P->op_mask >> 8) & 0xFu;
    for (int ch = 0; ch < chains; ++ch) {
        chain_t* c = &C[ch];
        sol_alloc(&c->S, n, m);
        sol_alloc(&c->B, n, m);
        c->S.L = init_rt[m - 1];
        memcpy(c->S.ops, init_ops, (size_t)c->S.L * sizeof(uint16_t));
        memcpy(c->S.rt, init_rt, (size_t)m * sizeof(uint16_t));
        sol_copy(&c->B, &c->S, m);
        sol_eval(I, &c->S, &c->k.z, NULL);
        c->k.zb = c->k.z;
        c->k.T = P->T0 * (double)c->k.zb;
        c->k.T_init = c->k.T;
        for (int i = 0; i < ND; ++i) c->k.wD[i] = 1.0;
        for (int i = 0; i < NR; ++i) c->k.wR[i] = 1.0;
    }
    for (int64_t it = 0; it < iterations; ++it) {
        for (int ch = 0; ch < chains; ++ch) {
            chain_t* c = &C[ch];
            const uint32_t u_it = (uint32_t)it, u_ch = chain0 + (uint32_t)ch;
            const int di = roulette(c->k.wD, ND, dmask, unit_d(adraw(seed, 0, u_it, u_ch)));
            const int ri = roulette(c->k.wR, NR, rmask, unit_d(adraw(seed, 1, u_it, u_ch)));
            const int q = q_min + uint_below(adraw(seed, 2, u_it, u_ch), q_max - q_min + 1);
            int nrem = destroy(I, di, &c->S, c->k.z, q, q_min, seed, u_it, u_ch, 0, rem, &tmp, gone);
            memset(gone, 0, (size_t)n + 1);
            for (int i = 0; i < nrem; ++i) gone[rem[i]] = 1;
            sol_remove(&c->S, gone, m, &work);
            memset(gone, 0, (size_t)n + 1);
            int KD, KP;
            budget_split(P->tuple_budget, nrem, &KD, &KP);
            int32_t zn = INT32_MAX;
            int okr = repair(I, ri, &work, rem, nrem, KD, KP, tbuf, dbuf, pbuf, &tmp2, &zn, NULL);
            const double u = unit_d(adraw(seed, 8, u_it, u_ch));
            const int accepted = orc_alns_update(P, &c->k, di, ri, okr, zn, u, it);
            if (accepted) sol_copy(&c->S, &work, m);
            if (accepted == 2) sol_copy(&c->B, &work, m);
            if (trace) {
                int64_t* tr = trace + ((size_t)ch * (size_t)iterations + (size_t)it) * 4;
                tr[0] = okr ? zn : INT32_MAX;
                tr[1] = c->k.z;
                tr[2] = c->k.zb;
                tr[3] = di | (ri << 8) | (accepted << 16) | ((int64_t)nrem << 24);
            }
            /* periodic local search on the current solution (Section 4.2.6):
             * repositioning before relocation when both fall due */
            int ls_any = 0;
            if (P->ls_repos_interval > 0 && (it + 1) % P->ls_repos_interval == 0)
                ls_any |= local_search(I, 0, P->ls_budget, &c->S, &c->k.z, &tmp, &tmp2, dbuf, pbuf, rem, gone);
            if (P->ls_reloc_interval > 0 && (it + 1) % P->ls_reloc_interval == 0)
                ls_any |= local_search(I, 1, P->ls_budget, &c->S, &c->k.z, &tmp, &tmp2, dbuf, pbuf, rem, gone);
            if (ls_any && c->k.z < c->k.zb) {
                sol_copy(&c->B, &c->S, m);
                c->k.zb = c->k.z;
                c->k.stag = 0;
            }
            memset(gone, 0, (size_t)n + 1);
        }
        if (P->import_interval > 0 && (it + 1) % P->import_interval == 0) {
            int bc = 0;
            for (int ch = 1; ch < chains; ++ch)
                if (C[ch].k.zb < C[bc].k.zb) bc = ch;
            for (int ch = 0; ch < chains; ++ch) {
                if (C[ch].k.zb > C[bc].k.zb) {
                    sol_copy(&C[ch].B, &C[bc].B, m);
                    C[ch].k.zb = C[bc].k.zb;
                    sol_copy(&C[ch].S, &C[bc].B, m);
                    C[ch].k.z = C[bc].k.zb;
                }
            }
        }
    }
    int32_t best = INT32_MAX;
    for (int ch = 0; ch < chains; ++ch) {
        if (best_ops) memcpy(best_ops + (size_t)ch * 2 * n, C[ch].B.ops, (size_t)C[ch].B.L * sizeof(uint16_t));
        if (best_rt) memcpy(best_rt + (size_t)ch * m, C[ch].B.rt, (size_t)m * sizeof(uint16_t));
        if (best_mk) best_mk[ch] = C[ch].k.zb;
        if (cur_mk) cur_mk[ch] = C[ch].k.z;
        if (fstate) {   /* final temperature and operator weights */
            double* f = fstate + (size_t)ch * (1 + ND + NR);
            f[0] = C[ch].k.T;
            for (int i = 0; i < ND; ++i) f[1 + i] = C[ch].k.wD[i];
            for (int i = 0; i < NR; ++i) f[1 + ND + i] = C[ch].k.wR[i];
        }
        if (C[ch].k.zb < best) best = C[ch].k.zb;
        sol_free(&C[ch].S);
        sol_free(&C[ch].B);
    }
    free(C); sol_free(&work); sol_free(&tmp); sol_free(&tmp2);
    free(dbuf); free(pbuf); free(tbuf); free(rem); free(gone);
    return best;
}


int32_t orc_alns_run_from(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                          uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                          uint16_t* best_rt, int32_t* best_mk, int64_t* trace, uint32_t chain0)
{
    return orc_alns_run_ex(I, P, chains, iterations, seed, init_ops, init_rt, best_ops, best_rt, best_mk, trace,
                           chain0, NULL, NULL);
}

int32_t orc_alns_run(const orc_inst* I, const orc_alns_params* P, int32_t chains, int64_t iterations,
                     uint64_t seed, const uint16_t* init_ops, const uint16_t* init_rt, uint16_t* best_ops,
                     uint16_t* best_rt, int32_t* best_mk, int64_t* trace)
{
    return orc_alns_run_from(I, P, chains, iterations, seed, init_ops, init_rt, best_ops, best_rt, best_mk, trace, 0);
}

/* One destroy operator applied to a complete solution (ops / rt_end) as
 * iteration `it` of chain `chain` would apply it, candidate `cand`; writes
 * the removed customers to rem (up to q) and returns their number, or -1 if
 * the solution is not feasible. */
int32_t orc_alns_destroy(const orc_inst* I, int32_t op, const uint16_t* ops, const uint16_t* rt_end, int32_t q,
                         int32_t q_min, uint64_t seed, uint32_t it, uint32_t chain, int32_t cand, int32_t* rem)
{
    const int n = I->n, m = I->m;
    sol_t S, tmp;
    sol_alloc(&S, n, m);
    sol_alloc(&tmp, n, m);
    S.L = rt_end[m - 1];
    memcpy(S.ops, ops, (size_t)S.L * sizeof(uint16_t));
    memcpy(S.rt, rt_end, (size_t)m * sizeof(uint16_t));
    int32_t z;
    int rc = -1;
    if (sol_eval(I, &S, &z, NULL) == 0) {
        unsigned char* gone = calloc((size_t)n + 1, 1);
        int* r = malloc((size_t)(n + 1) * sizeof(int));
        rc = destroy(I, op, &S, z, q, q_min, seed, it, chain, cand, r, &tmp, gone);
        for (int i = 0; i < rc; ++i) rem[i] = r[i];
        free(r);
        free(gone);
    }
    sol_free(&S);
    sol_free(&tmp);
    return rc;
}


/* Periodic local search (kind 0 pickup repositioning, 1 cross-agent
 * relocation) on a complete feasible solution, up to `passes` passes;
 * writes the result to out_ops / out_rt and its makespan to *z.  Returns the
 * number of improving passes, or -1 if the solution is not feasible. */
int32_t orc_alns_local_search(const orc_inst* I, int32_t kind, int32_t budget, int32_t passes, const uint16_t* ops,
                              const uint16_t* rt_end, uint16_t* out_ops, uint16_t* out_rt, int32_t* z)
{
    const int n = I->n, m = I->m;
    sol_t S, base, cand;
    sol_alloc(&S, n, m);
    sol_alloc(&base, n, m);
    sol_alloc(&cand, n, m);
    S.L = rt_end[m - 1];
    memcpy(S.ops, ops, (size_t)S.L * sizeof(uint16_t));
    memcpy(S.rt, rt_end, (size_t)m * sizeof(uint16_t));
    int rc = -1;
    if (sol_eval(I, &S, z, NULL) == 0) {
        const int maxslots = 2 * n + m + 2;
        slot_t* dbuf = malloc((size_t)maxslots * sizeof(slot_t));
        slot_t* pbuf = malloc((size_t)maxslots * sizeof(slot_t));
        int* cands = malloc((size_t)(n + 1) * sizeof(int));
        unsigned char* gone = calloc((size_t)n + 1, 1);
        rc = 0;
        for (int p = 0; p < passes; ++p) {
            if (!ls_pass(I, kind, budget, &S, z, &base, &cand, dbuf, pbuf, cands, gone)) break;
            ++rc;
        }
        free(dbuf); free(pbuf); free(cands); free(gone);
    }
    memcpy(out_ops, S.ops, (size_t)S.L * sizeof(uint16_t));
    memcpy(out_rt, S.rt, (size_t)m * sizeof(uint16_t));
    sol_free(&S); sol_free(&base); sol_free(&cand);
    return rc;
}


static void sol_load(sol_t* S, const uint16_t* ops, const uint16_t* rt_end, int m)
{
    S->L = m > 0 ? rt_end[m - 1] : 0;
    memcpy(S->ops, ops, (size_t)S->L * sizeof(uint16_t));
    memcpy(S->rt, rt_end, (size_t)m * sizeof(uint16_t));
}

/* Insertion candidates of customer c against a partial solution, in ranked
 * order (drop slots by detour, then for each the pickup slots by detour on
 * the route after the drop went in); K_D = K_P = 0 lists every slot pair.
 * Writes the tuples to out (capacity (2n+m+2)^2 when unbounded) and returns
 * their number. */
int32_t orc_alns_enumerate(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end, int32_t c, int32_t KD,
                           int32_t KP, orc_tuple* out)
{
    const int n = I->n, m = I->m;
    sol_t S;
    sol_alloc(&S, n, m);
    sol_load(&S, ops, rt_end, m);
    const int maxslots = 2 * n + m + 2;
    slot_t* dbuf = malloc((size_t)maxslots * sizeof(slot_t));
    slot_t* pbuf = malloc((size_t)maxslots * sizeof(slot_t));
    const int T = enumerate_tuples(I, &S, c, KD, KP, out, dbuf, pbuf);
    free(dbuf);
    free(pbuf);
    sol_free(&S);
    return T;
}

/* One repair (op 0 greedy, 1 regret-2, 2 regret-3, 3 regret-m) of a partial
 * solution missing the nrem customers of rem (in removal order), with K_D /
 * K_P slots per customer (0: all).  Writes the completed solution, its
 * makespan and the customers in the order they were inserted (nullable).
 * Returns 1, or 0 when some customer had no feasible insertion. */
int32_t orc_alns_repair(const orc_inst* I, int32_t op, const uint16_t* ops, const uint16_t* rt_end, const int32_t* rem,
                        int32_t nrem, int32_t KD, int32_t KP, uint16_t* out_ops, uint16_t* out_rt, int32_t* z,
                        int32_t* order)
{
    const int n = I->n, m = I->m;
    sol_t S, tmp;
    sol_alloc(&S, n, m);
    sol_alloc(&tmp, n, m);
    sol_load(&S, ops, rt_end, m);
    const int maxslots = 2 * n + m + 2;
    slot_t* dbuf = malloc((size_t)maxslots * sizeof(slot_t));
    slot_t* pbuf = malloc((size_t)maxslots * sizeof(slot_t));
    orc_tuple* tbuf = malloc((size_t)maxslots * (size_t)maxslots * sizeof(orc_tuple));
    int* rr = malloc((size_t)(nrem + 1) * sizeof(int));
    int* oo = malloc((size_t)(nrem + 1) * sizeof(int));
    for (int i = 0; i < nrem; ++i) rr[i] = rem[i];
    *z = INT32_MAX;
    const int ok = repair(I, op, &S, rr, nrem, KD, KP, tbuf, dbuf, pbuf, &tmp, z, oo);
    if (order)
        for (int i = 0; i < nrem; ++i) order[i] = ok ? oo[i] : 0;
    memcpy(out_ops, S.ops, (size_t)S.L * sizeof(uint16_t));
    memcpy(out_rt, S.rt, (size_t)m * sizeof(uint16_t));
    free(dbuf); free(pbuf); free(tbuf); free(rr); free(oo);
    sol_free(&S);
    sol_free(&tmp);
    return ok;
}

/* Slot counts of the budget split (see budget_split). */
void orc_alns_budget_split(int32_t budget, int32_t nrem, int32_t* KD, int32_t* KP)
{
    int a, b;
    budget_split(budget, nrem, &a, &b);
    *KD = a;
    *KP = b;
}
