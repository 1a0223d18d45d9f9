/*
 * Oracle insertion scan (test infrastructure only; see oracle.h).
 *
 * The repair operators of Section 4.2.3 price each way of putting a removed
 * customer back: its drop into some (vehicle, position) and its pickup into
 * some (vehicle, position), possibly on different vehicles, costed by the
 * resulting makespan.  This oracle builds each modified solution in full and
 * evaluates it with the definition (orc_eval); nothing is incremental.
 */
#include "oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

static int tuple_valid(const orc_inst* I, const uint16_t* ops, const uint16_t* rt, const orc_tuple* t)
{
    const int n = I->n, m = I->m;
    if (t->c < 1 || t->c > n || t->vD >= m || t->vP >= m) return 0;
    const int L = rt[m - 1];
    for (int j = 0; j < L; ++j)
        if ((ops[j] >> 1) == t->c) return 0;       /* customer already served */
    int lenD = rt[t->vD] - (t->vD ? rt[t->vD - 1] : 0);
    int lenP = rt[t->vP] - (t->vP ? rt[t->vP - 1] : 0);
    if (t->pD > lenD) return 0;
    if (t->vP == t->vD) return t->pP >= t->pD + 1 && t->pP <= lenD + 1;
    return t->pP <= lenP;
}

/* Positions: D_c goes before index pD of route vD; P_c before index pP of
 * route vP, counted after the drop was inserted. */
static void build(const orc_inst* I, const uint16_t* ops, const uint16_t* rt, const orc_tuple* t,
                  uint16_t* out_ops, uint16_t* out_rt)
{
    const int m = I->m;
    int w = 0;
    uint16_t* tmp = malloc(((size_t)rt[m - 1] + 2) * sizeof(uint16_t));
    for (int v = 0, s = 0; v < m; s = rt[v], ++v) {
        int len = 0;
        for (int j = s; j < rt[v]; ++j) tmp[len++] = ops[j];
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
        memcpy(out_ops + w, tmp, (size_t)len * sizeof(uint16_t));
        w += len;
        out_rt[v] = (uint16_t)w;
    }
    free(tmp);
}

void orc_insert_scan(const orc_inst* I, const uint16_t* base_ops, const uint16_t* base_rt,
                     int64_t T, const orc_tuple* tuples, int32_t S, const int64_t* seg_off,
                     int32_t* mk_out, uint32_t* st_out, int64_t* seg_top3)
{
    const int m = I->m;
    uint16_t* ops = malloc(((size_t)base_rt[m - 1] + 2 + 2 * (size_t)m) * sizeof(uint16_t));
    uint16_t* rt = malloc((size_t)m * sizeof(uint16_t));
    int32_t* mk = malloc((size_t)(T ? T : 1) * sizeof(int32_t));
    uint32_t* st = malloc((size_t)(T ? T : 1) * sizeof(uint32_t));
    /* positions are only defined against a valid route-end table */
    int rt_ok = 1;
    for (int v = 0, prev = 0; v < m; prev = base_rt[v], ++v)
        if (base_rt[v] < prev) rt_ok = 0;
    if (base_rt[m - 1] > 2 * I->n) rt_ok = 0;
    for (int64_t i = 0; i < T; ++i) {
        if (!rt_ok) {
            mk[i] = INT32_MAX;
            st[i] = ORC_BAD_COVER;
            continue;
        }
        if (!tuple_valid(I, base_ops, base_rt, &tuples[i])) {
            mk[i] = INT32_MAX;
            st[i] = ORC_BAD_TUPLE;
            continue;
        }
        build(I, base_ops, base_rt, &tuples[i], ops, rt);
        st[i] = orc_eval(I, 1, ops, rt, &mk[i], NULL);
    }
    if (mk_out) memcpy(mk_out, mk, (size_t)T * sizeof(int32_t));
    if (st_out) memcpy(st_out, st, (size_t)T * sizeof(uint32_t));
    for (int32_t s = 0; s < S; ++s) {
        int64_t best[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        for (int64_t i = seg_off[s]; i < seg_off[s + 1]; ++i) {
            if (st[i] != 0) continue;
            int64_t key = ((int64_t)mk[i] << 32) | (int64_t)(uint32_t)i;
            if (key < best[2]) {
                best[2] = key;
                if (best[2] < best[1]) { int64_t x = best[1]; best[1] = best[2]; best[2] = x; }
                if (best[1] < best[0]) { int64_t x = best[0]; best[0] = best[1]; best[1] = x; }
            }
        }
        seg_top3[3 * s + 0] = best[0];
        seg_top3[3 * s + 1] = best[1];
        seg_top3[3 * s + 2] = best[2];
    }
    free(ops); free(rt); free(mk); free(st);
}
