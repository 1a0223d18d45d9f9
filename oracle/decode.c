/*
 * Oracle multi-pass decoder (test infrastructure only; see oracle.h).
 *
 * Follows Section 4.4.2 (Algorithm 2 and the SelectVehicle rule) with these
 * readings of points the text leaves open:
 *  - keys must lie in [0, 1) (Section 4.4.1); -0.0 counts as 0.0, anything
 *    else (NaN, negative, >= 1) marks the chromosome BAD_KEY;
 *  - the argsort is stable: equal priorities keep op-index order;
 *  - a pickup is feasible once its drop is scheduled and some vehicle has
 *    room; the chosen vehicle waits for the resource (Eq. 9) instead of the
 *    pickup being refused until some clock passes the ready time;
 *  - SelectVehicle minimises the op's completion time (arrival for a drop,
 *    max(arrival, ready) for a pickup); ties go to the vehicle first reached
 *    when counting cyclically from the hint vehicle floor(m * alpha_o);
 *  - with ORC_DECODE_HINT_FIRST the hint vehicle takes the op whenever it can
 *    (Section 4.4.1: the hint maps to vehicle floor(m * alpha_o) and is
 *    overridden only for feasibility; Section 4.4.4: the ALNS encoding then
 *    decodes to the ALNS solution); SelectVehicle as above chooses only when
 *    the hint vehicle cannot take it;
 *  - initial loads follow the instance's load model (FULL_START: q = k as in
 *    Algorithm 2; MIN_PRELOAD: a vehicle takes one more resource from the
 *    depot only when a drop needs it, within k and the fleet total R).
 */
#include "oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { float key; int o; } keyed;

static int cmp_keyed(const void* a, const void* b)
{
    const keyed* x = a;
    const keyed* y = b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->o > y->o) - (x->o < y->o);
}

static int canon_key(float x, float* out)
{
    if (x == 0.0f) x = 0.0f; /* -0.0 -> +0.0 */
    if (!(x >= 0.0f && x < 1.0f)) return 0;
    *out = x;
    return 1;
}

uint32_t orc_decode_ex(const orc_inst* I, const float* prio, const float* hint,
                       int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                       uint16_t* ops_out, uint16_t* rt_end_out, int32_t flags)
{
    const int hint_first = (flags & ORC_DECODE_HINT_FIRST) != 0;
    const int n = I->n, m = I->m, k = I->k, N1 = n + 1, O = 2 * n;
    const int minpre = I->load_model != ORC_FULL_START;
    keyed* ord = malloc((size_t)O * sizeof(keyed));
    float* alpha = malloc((size_t)O * sizeof(float));
    int bad = 0;
    for (int o = 0; o < O; ++o) {
        ord[o].o = o;
        if (!canon_key(prio[o], &ord[o].key)) bad = 1;
        alpha[o] = 0.0f;
        if (hint && !canon_key(hint[o], &alpha[o])) bad = 1;
    }
    if (bad) {
        *fitness = INT64_MAX;
        *makespan = INT32_MAX;
        *unscheduled = O;
        if (rt_end_out) memset(rt_end_out, 0, (size_t)m * sizeof(uint16_t));
        free(ord); free(alpha);
        return ORC_BAD_KEY;
    }
    qsort(ord, (size_t)O, sizeof(keyed), cmp_keyed);

    long long* t = calloc((size_t)m, sizeof(long long));
    int* loc = calloc((size_t)m, sizeof(int));
    int* q = malloc((size_t)m * sizeof(int));
    int* M = calloc((size_t)m, sizeof(int));      /* highest load reached so far */
    int* len = calloc((size_t)m, sizeof(int));
    uint16_t* seq = malloc((size_t)m * O * sizeof(uint16_t));
    unsigned char* sched = calloc((size_t)O, 1);
    long long* ready = calloc((size_t)N1, sizeof(long long));
    long long Lsum = 0;
    for (int v = 0; v < m; ++v) q[v] = minpre ? 0 : k;

    int nsched = 0;
    for (int pass = 1; pass <= O; ++pass) {
        int progressed = 0;
        for (int i = 0; i < O; ++i) {
            const int o = ord[i].o;
            if (sched[o]) continue;
            const int c = o / 2 + 1, isP = o & 1;
            if (isP && !sched[o - 1]) continue;     /* drop not yet scheduled */
            int h = 0;
            if (hint) {
                float prod = (float)m * alpha[o];
                h = (int)floorf(prod);
                if (h > m - 1) h = m - 1;
            }
            int bv = -1, brot = 0;
            long long bkey = 0;
            for (int v = 0; v < m; ++v) {
                long long arr = t[v] + I->d[loc[v] * N1 + c];
                long long key;
                int cand;
                if (!isP) {
                    cand = q[v] > 0 || (minpre && M[v] < k && Lsum < I->R);
                    key = arr;
                } else {
                    cand = q[v] < k;
                    key = arr > ready[c] ? arr : ready[c];
                }
                if (!cand) continue;
                if (hint_first && v == h) {   /* the hint vehicle can take it: it does */
                    bv = v; bkey = key;
                    break;
                }
                int rot = (v - h + m) % m;
                if (bv < 0 || key < bkey || (key == bkey && rot < brot)) {
                    bv = v; bkey = key; brot = rot;
                }
            }
            if (bv < 0) continue;
            const int v = bv;
            if (!isP) {
                if (q[v] == 0) { M[v]++; Lsum++; q[v]++; }   /* take one more from the depot */
                q[v]--;
                t[v] = bkey;
                ready[c] = bkey + I->p[c];
            } else {
                q[v]++;
                if (q[v] > M[v]) M[v] = q[v];
                t[v] = bkey;
            }
            loc[v] = c;
            seq[(size_t)v * O + len[v]++] = (uint16_t)((c << 1) | isP);
            sched[o] = 1;
            ++nsched;
            progressed = 1;
        }
        if (nsched == O || !progressed) break;
    }
    long long z = 0;
    for (int v = 0; v < m; ++v) {
        if (!len[v]) continue;
        long long r = t[v] + I->d[loc[v] * N1];
        if (r > z) z = r;
    }
    *makespan = (int32_t)z;
    *unscheduled = O - nsched;
    *fitness = z + 1000000LL * (O - nsched);
    if (ops_out && rt_end_out) {
        int e = 0;
        for (int v = 0; v < m; ++v) {
            memcpy(ops_out + e, seq + (size_t)v * O, (size_t)len[v] * sizeof(uint16_t));
            e += len[v];
            rt_end_out[v] = (uint16_t)e;
        }
    }
    uint32_t st = 0;
    if (!minpre && (long long)m * k > I->R) st |= ORC_RES;
    free(t); free(loc); free(q); free(M); free(len); free(seq); free(sched); free(ready);
    free(ord); free(alpha);
    return st;
}


uint32_t orc_decode(const orc_inst* I, const float* prio, const float* hint,
                    int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                    uint16_t* ops_out, uint16_t* rt_end_out)
{
    return orc_decode_ex(I, prio, hint, fitness, makespan, unscheduled, ops_out, rt_end_out, 0);
}
