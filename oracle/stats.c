/*
 * Oracle solution statistics (test infrastructure only; see oracle.h).
 *
 * The two coordination measures of Section 5.2 (the processing-time
 * hypothesis): Cross-Agent, the customers whose drop and pickup are done by
 * different vehicles, and Interleaved, the customers for which a vehicle
 * does other work between their drop and their pickup.
 *
 * Reading of "Interleaved" (the paper defines it in words only): the vehicle
 * that drops c does another operation between the drop and the pickup of c.
 * When the same vehicle picks c up, that is an operation between the two in
 * its route; when another vehicle does, it is the drop vehicle's next
 * operation after the drop, if its time (the evaluator's op time: arrival
 * for a drop, departure for a pickup) is before the pickup time of c.
 * Counts are taken on the earliest-start schedule of the sequences.
 */
#include <stdlib.h>

#include "oracle.h"

/* Returns 0 and the two counts, or -1 (counts untouched) when the cover is
 * incomplete or the schedule deadlocks. */
int32_t orc_solution_stats(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end, int32_t* cross,
                           int32_t* interleaved)
{
    const int n = I->n, m = I->m;
    const int L = rt_end[m - 1];
    int32_t mk;
    int64_t* t = malloc((size_t)(L + 1) * sizeof(int64_t));
    const uint32_t st = orc_eval(I, 0, ops, rt_end, &mk, t);
    if (st & (ORC_BAD_COVER | ORC_DEADLOCK)) {
        free(t);
        return -1;
    }
    int* posD = malloc((size_t)(n + 1) * sizeof(int));
    int* posP = malloc((size_t)(n + 1) * sizeof(int));
    int* veh = malloc((size_t)L * sizeof(int));
    int* end = malloc((size_t)m * sizeof(int));
    for (int v = 0, s = 0; v < m; s = rt_end[v], ++v) {
        end[v] = rt_end[v];
        for (int j = s; j < rt_end[v]; ++j) {
            veh[j] = v;
            if (ops[j] & 1) posP[ops[j] >> 1] = j;
            else posD[ops[j] >> 1] = j;
        }
    }
    int nc = 0, ni = 0;
    for (int c = 1; c <= n; ++c) {
        const int jd = posD[c], jp = posP[c];
        const int vd = veh[jd], vp = veh[jp];
        if (vd != vp) {
            ++nc;
            if (jd + 1 < end[vd] && t[jd + 1] < t[jp]) ++ni;
        } else if (jp != jd + 1) {
            ++ni;
        }
    }
    *cross = nc;
    *interleaved = ni;
    free(t); free(posD); free(posP); free(veh); free(end);
    return 0;
}
