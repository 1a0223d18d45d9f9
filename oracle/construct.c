/*
 * Oracle construction heuristics (test infrastructure only; see oracle.h).
 *
 * 1. The initial solution of Section 4.2 ("Initial Solution Construction"),
 *    its first three phases: sweep clustering by a pseudo-angle computed
 *    from the distance matrix alone, load balancing of the sectors by the
 *    workload estimate w_c = 2 d(0,c) + p_c, and a nearest-neighbour route
 *    per vehicle.  The fourth phase (refinement by relocation and pickup
 *    reassignment until nothing improves) is the local search of Section
 *    4.2.6 run to a fixed point; oracle/__init__.py composes it.
 * 2. The three construction seeds of the BRKGA warm start (Section 4.4.4):
 *    nearest neighbour, load balanced, shortest processing time.
 *
 * Readings (the paper names the phases and their goals, not the formulas):
 *  - pseudo-angle: the depot is the origin, the customer r farthest from it
 *    (lowest index on ties) fixes the direction of angle 0, and the law of
 *    cosines gives every customer's coordinate along that axis,
 *    x_c = X_c / (2b) with X_c = a_c^2 + b^2 - d(r,c)^2, a_c = d(0,c),
 *    b = d(0,r).  The sign of the other coordinate comes from a second
 *    reference r2, the customer farthest from the axis (largest
 *    4 a^2 b^2 - X^2, lowest index on ties), placed on the positive side:
 *    sign(y_c) = sign(2 b^2 (a_c^2 + a_r2^2 - d(r2,c)^2) - X_c X_r2).
 *    Angles run from 0 towards r2's side; the angle order is the order of
 *    (half, cosine) with the cosine X_c / (2 a_c b) taken as the integer
 *    quotient trunc(X_c 2^30 / (2 a_c b)) clamped to [-2^30, 2^30], ties by
 *    customer index.  All of this is exact 64-bit integer arithmetic on
 *    distances shifted right until the largest is below 2^14 (no shift on
 *    distances below 2^14);
 *  - sectors: m' = m vehicles under FULL_START, m' = max(1, min(m, R))
 *    under MIN_PRELOAD; the angle order is cut into m' contiguous runs, the
 *    first n mod m' of length floor(n/m') + 1, the rest floor(n/m');
 *  - balancing: while the heaviest sector v_max (lowest index on ties)
 *    exceeds the lightest v_min by 10% of the heaviest or more
 *    (10 (W_max - W_min) >= W_max), move from v_max to v_min the customer
 *    with 0 < w_c < W_max - W_min closest to half the gap (least
 *    |W_max - W_min - 2 w_c|, lowest index on ties); stop when no customer
 *    qualifies.  Every move lowers sum W_v^2, so the loop ends (no move
 *    limit: the passage gives only the 10% stopping rule);
 *  - per-vehicle nearest neighbour: vehicle v serves its sector alone,
 *    starting at the depot at time 0 with at most cap_v resources out at a
 *    time (cap_v = k under FULL_START; under MIN_PRELOAD R is split as
 *    evenly as possible over the m' vehicles, the first R mod m' getting
 *    one more, and cap_v = min(k, share)).  Each step takes the op with the
 *    earliest completion: a drop completes at arrival, a pickup at
 *    max(arrival, drop time + p_c); drops only while fewer than cap_v
 *    resources are out.  Ties by op index o = 2(c-1) + isPickup;
 *  - LB (load balanced) assigns whole customers, heaviest workload w_c
 *    first (ties by index), each to the vehicle of least assigned workload
 *    so far among the m' above (ties by index), then builds the routes as
 *    the per-vehicle nearest neighbour above;
 *  - NN and SPT are one dispatch loop over all m vehicles with the
 *    decoder's load rules (Algorithm 2 with the library's load model): a
 *    drop needs a resource on board or, under MIN_PRELOAD, room to preload
 *    one more (the vehicle's peak load below k and fewer than R preloaded in
 *    all); a pickup needs its drop done and the vehicle below k.  Each step
 *    places one (vehicle, op) pair:
 *      NN  the vehicle free earliest (least current time, ties by index)
 *          among those with a feasible op takes its nearest one (least
 *          d(loc_v, c), ties by op);
 *      SPT drops only in ascending (p_c, c) order: the candidates are the
 *          first undropped customer's drop and every pending pickup on
 *          every vehicle that may take it, and the pair of earliest
 *          completion wins (ties by op, then vehicle).
 *    The loop stops when every op is placed, or when nothing is feasible
 *    (possible only with R = 0); ops never placed are left out.
 */
#include <limits.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CONS_SWEEP 0
#define CONS_NN 1
#define CONS_LB 2
#define CONS_SPT 3

static int64_t dd(const orc_inst* I, int a, int b) { return I->d[(size_t)a * (I->n + 1) + b]; }

int32_t orc_cons_vehicles(const orc_inst* I)
{
    if (I->load_model == ORC_FULL_START) return I->m;
    int mv = I->m < I->R ? I->m : I->R;
    return mv < 1 ? 1 : mv;
}

/* Customers 1..n in pseudo-angle order. */
void orc_cons_angle_order(const orc_inst* I, int32_t* order)
{
    const int n = I->n;
    int64_t dmax = 0;
    for (int c = 0; c <= n; ++c) {
        if (dd(I, 0, c) > dmax) dmax = dd(I, 0, c);
        for (int x = 1; x <= n; ++x)
            if (dd(I, x, c) > dmax) dmax = dd(I, x, c);
    }
    int s = 0;
    while ((dmax >> s) >= (1 << 14)) ++s;
    int r = 1;
    for (int c = 2; c <= n; ++c)
        if ((dd(I, 0, c) >> s) > (dd(I, 0, r) >> s)) r = c;
    const int64_t b = dd(I, 0, r) >> s;
    int64_t* X = malloc((size_t)(n + 1) * sizeof(int64_t));
    uint64_t* key = malloc((size_t)n * sizeof(uint64_t));
    for (int c = 1; c <= n; ++c) {
        const int64_t a = dd(I, 0, c) >> s, e = dd(I, r, c) >> s;
        X[c] = a * a + b * b - e * e;
    }
    int r2 = 1;
    int64_t hbest = INT64_MIN;
    for (int c = 1; c <= n; ++c) {
        const int64_t a = dd(I, 0, c) >> s;
        const int64_t h = 4 * a * a * b * b - X[c] * X[c];
        if (h > hbest) { hbest = h; r2 = c; }
    }
    const int64_t a2 = dd(I, 0, r2) >> s;
    for (int c = 1; c <= n; ++c) {
        const int64_t a = dd(I, 0, c) >> s, e2 = dd(I, r2, c) >> s;
        int side = 0;
        if (hbest > 0) {
            const int64_t t = 2 * b * b * (a * a + a2 * a2 - e2 * e2) - X[c] * X[r2];
            side = t > 0 ? 1 : (t < 0 ? -1 : 0);
        }
        int64_t q;
        if (a == 0 || b == 0) {
            q = (int64_t)1 << 30;
        } else {
            q = X[c] * ((int64_t)1 << 30) / (2 * a * b);
            if (q > ((int64_t)1 << 30)) q = (int64_t)1 << 30;
            if (q < -((int64_t)1 << 30)) q = -((int64_t)1 << 30);
        }
        const int half = side < 0 || (side == 0 && X[c] < 0);
        const uint64_t u = half ? (uint64_t)(q + ((int64_t)1 << 30)) : (uint64_t)(((int64_t)1 << 30) - q);
        key[c - 1] = ((uint64_t)half << 47) | (u << 15) | (uint64_t)c;
    }
    /* insertion sort: plain and small enough for the oracle's sizes */
    for (int i = 1; i < n; ++i) {
        const uint64_t x = key[i];
        int j = i - 1;
        while (j >= 0 && key[j] > x) { key[j + 1] = key[j]; --j; }
        key[j + 1] = x;
    }
    for (int i = 0; i < n; ++i) order[i] = (int32_t)(key[i] & 0x7FFF);
    free(X);
    free(key);
}

/* Sector of every customer (sector[0] unused): before balancing in sector0
 * (nullable), after it in sector.  Returns the number of moves. */
int32_t orc_cons_sectors(const orc_inst* I, int32_t* sector0, int32_t* sector)
{
    const int n = I->n, mv = orc_cons_vehicles(I);
    int32_t* order = malloc((size_t)n * sizeof(int32_t));
    orc_cons_angle_order(I, order);
    const int base = n / mv, extra = n % mv;
    for (int v = 0, i = 0; v < mv; ++v) {
        const int len = base + (v < extra);
        for (int j = 0; j < len; ++j, ++i) sector[order[i]] = v;
    }
    sector[0] = -1;
    if (sector0) memcpy(sector0, sector, (size_t)(n + 1) * sizeof(int32_t));
    int64_t W[64];
    for (int v = 0; v < mv; ++v) W[v] = 0;
    for (int c = 1; c <= n; ++c) W[sector[c]] += 2 * dd(I, 0, c) + I->p[c];
    /* Each move takes w with 0 < w < gap from the heaviest to the lightest
     * sector, so the sum of squared workloads falls by 2 w (gap - w) > 0: an
     * integer that falls at every move, hence the loop ends by itself. */
    int moves = 0;
    for (;;) {
        int hi = 0, lo = 0;
        for (int v = 1; v < mv; ++v) {
            if (W[v] > W[hi]) hi = v;
            if (W[v] < W[lo]) lo = v;
        }
        const int64_t gap = W[hi] - W[lo];
        if (10 * gap < W[hi]) break;
        int best = 0;
        int64_t bdev = INT64_MAX;
        for (int c = 1; c <= n; ++c) {
            if (sector[c] != hi) continue;
            const int64_t w = 2 * dd(I, 0, c) + I->p[c];
            if (w <= 0 || w >= gap) continue;
            const int64_t dev = gap - 2 * w >= 0 ? gap - 2 * w : 2 * w - gap;
            if (dev < bdev) { bdev = dev; best = c; }
        }
        if (!best) break;
        const int64_t w = 2 * dd(I, 0, best) + I->p[best];
        sector[best] = lo;
        W[hi] -= w;
        W[lo] += w;
        ++moves;
    }
    free(order);
    return moves;
}

/* LB: whole customers to the least loaded vehicle, heaviest first. */
static void lb_sectors(const orc_inst* I, int32_t* sector)
{
    const int n = I->n, mv = orc_cons_vehicles(I);
    int32_t* cs = malloc((size_t)n * sizeof(int32_t));
    for (int i = 0; i < n; ++i) cs[i] = i + 1;
    for (int i = 1; i < n; ++i) {   /* insertion sort by (-w, c) */
        const int x = cs[i];
        const int64_t wx = 2 * dd(I, 0, x) + I->p[x];
        int j = i - 1;
        while (j >= 0) {
            const int64_t wj = 2 * dd(I, 0, cs[j]) + I->p[cs[j]];
            if (wj > wx || (wj == wx && cs[j] < x)) break;
            cs[j + 1] = cs[j];
            --j;
        }
        cs[j + 1] = x;
    }
    int64_t W[64];
    for (int v = 0; v < mv; ++v) W[v] = 0;
    for (int i = 0; i < n; ++i) {
        int lo = 0;
        for (int v = 1; v < mv; ++v)
            if (W[v] < W[lo]) lo = v;
        sector[cs[i]] = lo;
        W[lo] += 2 * dd(I, 0, cs[i]) + I->p[cs[i]];
    }
    sector[0] = -1;
    free(cs);
}

/* Appends the placed (vehicle, op) pairs in placement order to routes. */
static void to_routes(int m, int cnt, const int32_t* seq_v, const int32_t* seq_o, uint16_t* ops, uint16_t* rt_end)
{
    int pos = 0;
    for (int v = 0; v < m; ++v) {
        for (int i = 0; i < cnt; ++i)
            if (seq_v[i] == v) ops[pos++] = (uint16_t)(((seq_o[i] >> 1) + 1) << 1 | (seq_o[i] & 1));
        rt_end[v] = (uint16_t)pos;
    }
}

/* Phase 3: each vehicle's route over its own sector. */
static int sweep_routes(const orc_inst* I, const int32_t* sector, int32_t* seq_v, int32_t* seq_o)
{
    const int n = I->n, mv = orc_cons_vehicles(I);
    int64_t* ready = malloc((size_t)(n + 1) * sizeof(int64_t));
    unsigned char* st = calloc((size_t)n + 1, 1);   /* 0 waiting, 1 dropped, 2 picked */
    int cnt = 0;
    for (int v = 0; v < mv; ++v) {
        int cap = I->k;
        if (I->load_model != ORC_FULL_START) {
            const int share = I->R / mv + (v < I->R % mv);
            cap = share < I->k ? share : I->k;
        }
        int64_t t = 0;
        int loc = 0, out = 0;
        for (;;) {
            int64_t bk = INT64_MAX;
            int bo = -1;
            for (int c = 1; c <= n; ++c) {
                if (sector[c] != v || st[c] == 2) continue;
                const int64_t arr = t + dd(I, loc, c);
                if (st[c] == 0) {
                    if (out >= cap) continue;
                    if (arr < bk || (arr == bk && 2 * (c - 1) < bo)) { bk = arr; bo = 2 * (c - 1); }
                } else {
                    const int64_t k = arr > ready[c] ? arr : ready[c];
                    if (k < bk || (k == bk && 2 * (c - 1) + 1 < bo)) { bk = k; bo = 2 * (c - 1) + 1; }
                }
            }
            if (bo < 0) break;
            const int c = bo / 2 + 1;
            t = bk;
            loc = c;
            if (bo & 1) { st[c] = 2; --out; }
            else { st[c] = 1; ready[c] = t + I->p[c]; ++out; }
            seq_v[cnt] = v;
            seq_o[cnt] = bo;
            ++cnt;
        }
    }
    free(ready);
    free(st);
    return cnt;
}

/* The seeds' dispatch loop (NN, SPT). */
static int dispatch(const orc_inst* I, int rule, int32_t* seq_v, int32_t* seq_o)
{
    const int n = I->n, m = I->m, k = I->k, full = I->load_model == ORC_FULL_START;
    int64_t t[64];
    int loc[64], q[64], M[64];
    int Lsum = 0;
    for (int v = 0; v < m; ++v) { t[v] = 0; loc[v] = 0; q[v] = full ? k : 0; M[v] = full ? k : 0; }
    int64_t* ready = malloc((size_t)(n + 1) * sizeof(int64_t));
    unsigned char* st = calloc((size_t)n + 1, 1);
    int32_t* spt = malloc((size_t)n * sizeof(int32_t));
    for (int i = 0; i < n; ++i) spt[i] = i + 1;
    for (int i = 1; i < n; ++i) {   /* insertion sort by (p, c) */
        const int x = spt[i];
        int j = i - 1;
        while (j >= 0 && (I->p[spt[j]] > I->p[x] || (I->p[spt[j]] == I->p[x] && spt[j] > x))) { spt[j + 1] = spt[j]; --j; }
        spt[j + 1] = x;
    }
    int spt_next = 0, cnt = 0, undropped = n, pending = 0;
    for (;;) {
        while (spt_next < n && st[spt[spt_next]] != 0) ++spt_next;
        int bv = -1, bo = -1;
        int64_t bk1 = INT64_MAX, bk2 = INT64_MAX;
        int nn_v = -1;
        if (rule == CONS_NN) {
            for (int v = 0; v < m; ++v) {
                const int canD = q[v] > 0 || (!full && M[v] < k && Lsum < I->R);
                const int canP = q[v] < k;
                if (!((canD && undropped > 0) || (canP && pending > 0))) continue;
                if (nn_v < 0 || t[v] < t[nn_v]) nn_v = v;
            }
            if (nn_v < 0) break;
        }
        for (int v = 0; v < m; ++v) {
            if (rule == CONS_NN && v != nn_v) continue;
            const int canD = q[v] > 0 || (!full && M[v] < k && Lsum < I->R);
            const int canP = q[v] < k;
            for (int c = 1; c <= n; ++c) {
                if (st[c] == 2) continue;
                const int isP = st[c] == 1;
                if (isP ? !canP : !canD) continue;
                if (!isP && rule == CONS_SPT && c != spt[spt_next]) continue;
                const int o = 2 * (c - 1) + isP;
                const int64_t arr = t[v] + dd(I, loc[v], c);
                const int64_t comp = isP && ready[c] > arr ? ready[c] : arr;
                const int64_t k1 = rule == CONS_NN ? dd(I, loc[v], c) : comp;
                /* NN: one vehicle, (distance, op); SPT: (completion, op, vehicle) */
                if (k1 < bk1 || (k1 == bk1 && (o < bo || (o == bo && v < bv)))) { bk1 = k1; bk2 = comp; bo = o; bv = v; }
            }
        }
        if (bo < 0) break;
        const int c = bo / 2 + 1, v = bv;
        t[v] = bk2;
        loc[v] = c;
        if (bo & 1) {
            st[c] = 2;
            ++q[v];
            if (q[v] > M[v]) M[v] = q[v];
            --pending;
        } else {
            if (q[v] == 0) { ++M[v]; ++Lsum; ++q[v]; }
            --q[v];
            st[c] = 1;
            ready[c] = t[v] + I->p[c];
            --undropped;
            ++pending;
        }
        seq_v[cnt] = v;
        seq_o[cnt] = bo;
        ++cnt;
    }
    free(ready);
    free(st);
    free(spt);
    return cnt;
}

/* One construction: ops (2n) and rt_end (m); seq_v / seq_o (nullable, 2n)
 * receive the placement order.  Returns the number of ops placed. */
int32_t orc_construct(const orc_inst* I, int32_t heuristic, uint16_t* ops, uint16_t* rt_end, int32_t* seq_v_out,
                      int32_t* seq_o_out)
{
    const int n = I->n;
    int32_t* seq_v = malloc((size_t)2 * n * sizeof(int32_t));
    int32_t* seq_o = malloc((size_t)2 * n * sizeof(int32_t));
    int cnt;
    if (heuristic == CONS_SWEEP || heuristic == CONS_LB) {
        int32_t* sector = malloc((size_t)(n + 1) * sizeof(int32_t));
        if (heuristic == CONS_SWEEP) orc_cons_sectors(I, NULL, sector);
        else lb_sectors(I, sector);
        cnt = sweep_routes(I, sector, seq_v, seq_o);
        free(sector);
    } else {
        cnt = dispatch(I, heuristic, seq_v, seq_o);
    }
    to_routes(I->m, cnt, seq_v, seq_o, ops, rt_end);
    if (seq_v_out) memcpy(seq_v_out, seq_v, (size_t)cnt * sizeof(int32_t));
    if (seq_o_out) memcpy(seq_o_out, seq_o, (size_t)cnt * sizeof(int32_t));
    free(seq_v);
    free(seq_o);
    return cnt;
}
