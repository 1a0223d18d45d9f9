/*
 * Oracle evaluators (test infrastructure only; see oracle.h).
 *
 * orc_eval     the definition: cover, load and the earliest-start timing sweep.
 * orc_eval_dag an independent longest-path evaluation of the same timing model.
 */
#include "oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

#define UNSET (-1LL)

static int route_ends_ok(int n, int m, const uint16_t* rt_end)
{
    int prev = 0;
    for (int v = 0; v < m; ++v) {
        if ((int)rt_end[v] < prev) return 0;
        prev = rt_end[v];
    }
    return prev <= 2 * n;
}

/*
 * Eq. (1): every customer receives exactly one drop and exactly one pickup.
 * Under allow_partial a customer may instead be absent altogether (neither op
 * present), which is how a destroyed solution is represented.
 */
static int cover_ok(int n, int allow_partial, const uint16_t* ops, int L)
{
    int ok = 1;
    unsigned char* nd = calloc((size_t)n + 1, 1);
    unsigned char* np = calloc((size_t)n + 1, 1);
    for (int j = 0; j < L && ok; ++j) {
        int c = ops[j] >> 1;
        if (c < 1 || c > n) { ok = 0; break; }
        if (ops[j] & 1) { if (np[c]++) ok = 0; }
        else            { if (nd[c]++) ok = 0; }
    }
    for (int c = 1; c <= n && ok; ++c) {
        if (nd[c] != np[c]) ok = 0;
        else if (!allow_partial && nd[c] == 0) ok = 0;
    }
    free(nd);
    free(np);
    return ok;
}

/*
 * Capacity, Eq. (13)-(18).  Let w_j be the number of drops minus pickups a
 * vehicle has done after its j-th op (w_0 = 0).
 *  FULL_START (the MILP as printed, q_0 = k): the load after op j is k - w_j,
 *    so 0 <= k - w_j <= k for every j; every vehicle holds k resources, so
 *    the fleet needs m*k of the R resources.
 *  MIN_PRELOAD: the vehicle leaves with the least load its route needs,
 *    L_v = max_j w_j, and its load k_j = L_v - w_j stays in [0, k]; the preloads
 *    together may not exceed the R resources available.
 */
static uint32_t load_status(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end)
{
    uint32_t st = 0;
    long long Lsum = 0;
    int s = 0;
    for (int v = 0; v < I->m; ++v) {
        int e = rt_end[v];
        long long w = 0, wmax = 0, wmin = 0;
        for (int j = s; j < e; ++j) {
            w += (ops[j] & 1) ? -1 : 1;
            if (w > wmax) wmax = w;
            if (w < wmin) wmin = w;
        }
        if (I->load_model == ORC_FULL_START) {
            if (wmin < 0 || wmax > I->k) st |= ORC_LOAD;
        } else {
            if (wmax - wmin > I->k) st |= ORC_LOAD;
            Lsum += wmax;
        }
        s = e;
    }
    if (I->load_model == ORC_FULL_START) {
        if ((long long)I->m * I->k > I->R) st |= ORC_RES;
    } else if (Lsum > I->R) {
        st |= ORC_RES;
    }
    return st;
}

uint32_t orc_eval(const orc_inst* I, int allow_partial, const uint16_t* ops,
                  const uint16_t* rt_end, int32_t* makespan, int64_t* op_time)
{
    const int n = I->n, m = I->m;
    const int32_t* d = I->d;
    const int N1 = n + 1;
    *makespan = INT32_MAX;
    if (!route_ends_ok(n, m, rt_end)) return ORC_BAD_COVER;
    const int L = rt_end[m - 1];
    if (!cover_ok(n, allow_partial, ops, L)) return ORC_BAD_COVER;

    uint32_t status = load_status(I, ops, rt_end);

    /*
     * Timing, Eq. (7)-(12): a drop happens on arrival, a pickup at departure,
     * and departure waits until the drop time plus p_c (Eq. 9), whichever
     * vehicle made the drop.  Each vehicle advances along its route while it
     * can; a pickup whose drop has not happened yet holds its vehicle.  When a
     * full round moves no vehicle the waits form a cycle (deadlock).
     */
    long long* t = calloc((size_t)m, sizeof(long long));
    int* loc = calloc((size_t)m, sizeof(int));
    int* ptr = malloc((size_t)m * sizeof(int));
    int* end = malloc((size_t)m * sizeof(int));
    long long* ready = malloc((size_t)N1 * sizeof(long long));
    for (int c = 0; c < N1; ++c) ready[c] = UNSET;
    for (int v = 0; v < m; ++v) {
        ptr[v] = v ? rt_end[v - 1] : 0;
        end[v] = rt_end[v];
    }
    for (;;) {
        int progressed = 0, done = 1;
        for (int v = 0; v < m; ++v) {
            while (ptr[v] < end[v]) {
                int j = ptr[v];
                int c = ops[j] >> 1;
                long long arr = t[v] + d[loc[v] * N1 + c];
                if (!(ops[j] & 1)) {            /* drop: at arrival (Eq. 7) */
                    t[v] = arr;
                    ready[c] = arr + I->p[c];
                } else {                        /* pickup (Eq. 8-10) */
                    if (ready[c] == UNSET) break;
                    t[v] = arr > ready[c] ? arr : ready[c];
                }
                if (op_time) op_time[j] = t[v];
                loc[v] = c;
                ptr[v]++;
                progressed = 1;
            }
            if (ptr[v] < end[v]) done = 0;
        }
        if (done) break;
        if (!progressed) { status |= ORC_DEADLOCK; break; }
    }
    if (!(status & ORC_DEADLOCK)) {
        /* Eq. (21)-(22): makespan = latest return to the depot; an unused
         * vehicle never leaves and contributes 0. */
        long long z = 0;
        for (int v = 0; v < m; ++v) {
            int s = v ? rt_end[v - 1] : 0;
            if (rt_end[v] == s) continue;
            long long r = t[v] + d[loc[v] * N1 + 0];
            if (r > z) z = r;
        }
        *makespan = z > INT32_MAX - 1 ? INT32_MAX - 1 : (int32_t)z;
    }
    free(t); free(loc); free(ptr); free(end); free(ready);
    return status;
}

/*
 * The same timing model as a graph: one node per op, a route edge from each op
 * to the next op of its vehicle (weight = travel time), and a cross edge from
 * D_c to P_c (weight p_c).  A node's time is the longest path into it
 * (earliest start); a cycle means some pickup waits on itself.
 */
uint32_t orc_eval_dag(const orc_inst* I, const uint16_t* ops, const uint16_t* rt_end,
                      int32_t* makespan, int64_t* op_time)
{
    const int n = I->n, m = I->m, N1 = n + 1;
    const int L = rt_end[m - 1];
    *makespan = INT32_MAX;
    int* route_of = malloc((size_t)(L + 1) * sizeof(int));
    int* first = malloc((size_t)(L + 1) * sizeof(int));
    int* pick_at = malloc((size_t)N1 * sizeof(int));
    int* indeg = calloc((size_t)(L + 1), sizeof(int));
    long long* T = calloc((size_t)(L + 1), sizeof(long long));
    int* queue = malloc((size_t)(L + 1) * sizeof(int));
    for (int c = 0; c < N1; ++c) pick_at[c] = -1;
    for (int v = 0, s = 0; v < m; s = rt_end[v], ++v)
        for (int j = s; j < rt_end[v]; ++j) { route_of[j] = v; first[j] = (j == s); }
    for (int j = 0; j < L; ++j)
        if (ops[j] & 1) pick_at[ops[j] >> 1] = j;
    for (int j = 0; j < L; ++j) {
        indeg[j] = !first[j];
        if (ops[j] & 1) indeg[j] += 1;
        /* a node with no predecessor starts from the depot at time 0 */
        T[j] = first[j] ? I->d[ops[j] >> 1] : 0;
    }
    int head = 0, tail = 0, done = 0;
    for (int j = 0; j < L; ++j)
        if (indeg[j] == 0) queue[tail++] = j;
    while (head < tail) {
        int j = queue[head++];
        ++done;
        if (op_time) op_time[j] = T[j];
        int c = ops[j] >> 1;
        /* route successor */
        if (j + 1 < L && !first[j + 1] && route_of[j + 1] == route_of[j]) {
            int k2 = j + 1;
            long long cand = T[j] + I->d[c * N1 + (ops[k2] >> 1)];
            if (cand > T[k2]) T[k2] = cand;
            if (--indeg[k2] == 0) queue[tail++] = k2;
        }
        /* cross successor: the pickup of the customer this node drops */
        if (!(ops[j] & 1) && pick_at[c] >= 0) {
            int k2 = pick_at[c];
            long long cand = T[j] + I->p[c];
            if (cand > T[k2]) T[k2] = cand;
            if (--indeg[k2] == 0) queue[tail++] = k2;
        }
    }
    uint32_t st = 0;
    if (done < L) {
        st = ORC_DEADLOCK;
    } else {
        long long z = 0;
        for (int v = 0, s = 0; v < m; s = rt_end[v], ++v) {
            if (rt_end[v] == s) continue;
            int last = rt_end[v] - 1;
            long long r = T[last] + I->d[(ops[last] >> 1) * N1];
            if (r > z) z = r;
        }
        *makespan = (int32_t)z;
    }
    free(route_of); free(first); free(pick_at); free(indeg); free(T); free(queue);
    return st;
}

void orc_eval_batch(const orc_inst* I, int allow_partial, int64_t B, const int64_t* op_off,
                    const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end,
                    int32_t* makespan, uint32_t* status)
{
    for (int64_t b = 0; b < B; ++b) {
        const uint16_t* o = ops + (op_off ? op_off[b] : b * 2 * (int64_t)I->n);
        const uint16_t* r = rt_end + (rt_off ? rt_off[b] : b * (int64_t)I->m);
        status[b] = orc_eval(I, allow_partial, o, r, &makespan[b], NULL);
    }
}
