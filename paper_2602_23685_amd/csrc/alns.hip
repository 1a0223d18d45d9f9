// alns_step: Algorithm 1 of Section 4.2 for many chains on one device.
//
// Every chain (an independent ALNS instance of Section 4.2.1, item 1) keeps
// its current solution S, its best S*, temperature, operator weights, scores
// and attempt counts in device memory.  One iteration is a fixed sequence of
// launches over all chains at once:
//   begin    roulette selection of the destroy / repair operators, q
//   gains    z(S) - z(S without c) for every customer (worst and critical-
//            path removal only), one sweep per customer, many blocks per chain
//   destroy  the removal list and the partial solution W = S minus it
//   rounds   (q_max times) enumerate candidate tuples of every waiting
//            customer, price them all exactly with the insertion scan, and
//            insert the customer the repair operator picks
//   accept   simulated annealing, scores, cooling, reheat, weight update
// and every import_interval iterations the chains of an instance adopt the
// best solution among them.  The operator and tie-breaking rules follow the
// readings stated in the header of vrprpd.h's alns section.
#include <climits>
#include <cmath>
#include <cstring>

#include "common.h"
#include "philox.h"
#include "scan.h"
#include "sweep.h"
#include "ckpt.h"

namespace vrprpd {

constexpr uint32_t kTagAlns = 0x414C4E53u;
constexpr int kND = 6, kNR = 4;
constexpr long long kBigC = 1LL << 40;
constexpr int kAlnsStep = 4;
// Insertion-scan workgroups take about this many tuples of a segment each:
// more, smaller workgroups spread a round's few thousand tuples over the CUs
// (each stages the base solution once).
constexpr int kScanTuplesPerBlock = 16;
constexpr int kGainWaves = 4;   // gains kernel: 4 waves of 16-lane groups (m <= 16)
constexpr int kGainGroups = 16;

struct AlnsDev {
    // problem
    const InstDev* inst_tab;
    const void* dist;
    const int32_t* proc;
    const int32_t* chain_inst;   // [C]
    int32_t C, N, M, Q, TPC;     // chains, n_max, m_max, q_max, tuples per customer slot
    alns_params prm;
    uint64_t seed;
    // solutions (stride 2N ops, M route ends per chain)
    uint16_t *S_ops, *S_rt, *B_ops, *B_rt, *W_ops, *W_rt;   // W: two buffers per chain
    int32_t* W_cur;
    int32_t *z, *zb, *zn;
    double *T, *T_init, *wD, *wR;
    long long *sD, *sR;
    int32_t *aD, *aR, *stag;
    // per-iteration scratch
    int32_t *di, *ri, *q, *nrem, *nleft, *KD, *KP, *rstate;   // rstate: 0 running, 1 done, 2 failed
    int32_t *rem, *left;           // [C][Q]
    long long* gains;              // [C][N+1]
    vrprpd_tuple* tuples;          // [C][Q][TPC]
    int32_t *tmk, *seg_cnt, *seg_base;
    uint32_t* tst;
    int64_t *seg_off, *seg_top3;
    int64_t *base_op_off, *base_rt_off;   // [C] offsets of the current W buffers
    int64_t* trace;                // [C][trace_cap][4] or null
    int64_t trace_cap, trace_base; // capacity; iteration of trace row 0
    uint32_t* it_dev;              // iteration counter (advanced by k_tick at the end of an iteration)
    unsigned long long* evals;     // exact evaluations performed (tuples and removal gains)
    // learned destroy proposal (Section 7.4 names learned operators as future
    // work; this library's form): K candidate removal sets per chain, scored
    // by the network from per-customer features
    int32_t K;                     // candidates per chain (1: the plain operator's set only)
    int32_t learn_on;              // features (and gains for every chain) each iteration
    double eps;                    // probability of keeping the plain operator's set
    uint16_t* feat;                // [C][N][64] bf16 features of S's customers (row cust - 1)
    float* fstat;                  // [C][N + 1][2] static features of the chain's instance
    int32_t* dbar;                 // [C]
    float* score;                  // [C][N] network scores
    int32_t *cand_rem, *cand_cnt;  // [C][K][Q], [C][K]
    int32_t* chosen;               // [C] candidate taken this iteration
    // (state, removal set, makespan change) records
    uint16_t* rec_x;               // [rec_cap][Q][64]
    float* rec_t;                  // [rec_cap] (z' - z) / z
    int32_t* rec_n;                // [rec_cap] removed customers
    int64_t rec_cap, rec_base;     // capacity in sets; iteration of the first record
    // periodic local search (Section 4.2.6); buffers exist when ls_budget > 0
    int32_t LQ;                    // candidates per pass at most
    int64_t LB;                    // tuple slots per chain
    uint16_t *ls_ops, *ls_rt;      // [C][LQ][2N], [C][LQ][M]: bases S without one candidate
    int32_t *ls_cand, *ls_pd;      // [C][LQ]: customer; its drop's (vehicle << 16 | position) in S
    int32_t *ls_nc, *ls_T, *ls_KD, *ls_KP, *ls_b, *ls_active, *ls_any;   // [C]
    int32_t* ls_stop;              // [C] refinement: the chain's last round improved nothing
    int32_t *ls_base_inst, *ls_seg_base, *ls_seg_cnt, *ls_tmk;          // [C][LQ] / [C][LB]
    uint32_t* ls_tst;
    int64_t *ls_seg_off, *ls_base_off, *ls_rt_off, *ls_top3;            // [C][LQ] (top3: x3)
    vrprpd_tuple* ls_tuples;       // [C][LB]
};

__device__ __forceinline__ uint32_t adraw(uint64_t seed, uint32_t a, uint32_t it, uint32_t chain)
{
    return philox_word(seed, a, it, chain, kTagAlns);
}
__device__ __forceinline__ double unit_d(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }
__device__ __forceinline__ int uint_below(uint32_t w, int nval) { return (int)(((uint64_t)w * (uint64_t)nval) >> 32); }

// exp(x) for x <= 0 by range reduction to |r| <= ln2/2 and a degree-16 Taylor
// series: a fixed sequence of IEEE operations, so every implementation that
// performs the same steps makes the same annealing decisions.
__device__ __forceinline__ double det_exp(double x)
{
    if (x < -745.0) return 0.0;
    const double LN2 = 0.6931471805599453;
    const double k = floor(x / LN2 + 0.5);
    const double r = x - k * LN2;
    double s = 1.0, term = 1.0;
    for (int i = 1; i <= 16; ++i) {
        term = term * (r / (double)i);
        s = s + term;
    }
    return ldexp(s, (int)k);
}

__device__ __forceinline__ int roulette(const double* w, int nops, uint32_t mask, double u)
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


// Sequential carving of dynamic LDS into 16-byte aligned arrays; the host
// sizes the allocation with the same rounding (LdsSize).
struct Carve {
    unsigned char* p;
    template <typename T>
    __device__ T* take(size_t count)
    {
        T* r = reinterpret_cast<T*>(p);
        p += (count * sizeof(T) + 15) & ~(size_t)15;
        return r;
    }
};
struct LdsSize {
    size_t bytes = 0;
    template <typename T>
    void take(size_t count) { bytes += (count * sizeof(T) + 15) & ~(size_t)15; }
};

// ---------------------------------------------------------------- begin
__global__ void k_begin(AlnsDev a)
{
    const uint32_t it = *a.it_dev;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    int qmin = a.prm.q_min, qmax = a.prm.q_max;
    if (qmin <= 0 || qmax <= 0) {
        qmax = I.n / 20;
        if (qmax < 4) qmax = 4;
        qmin = qmax / 2;
        if (qmin < 4) qmin = 4;
    }
    if (qmax > I.n) qmax = I.n;
    if (qmin > qmax) qmin = qmax;
    const uint32_t dmask = a.prm.op_mask & 0x3Fu, rmask = (a.prm.op_mask >> 8) & 0xFu;
    const int di = roulette(a.wD + kND * c, kND, dmask, unit_d(adraw(a.seed, 0, it, (uint32_t)c + (uint32_t)a.prm.chain_base)));
    const int ri = roulette(a.wR + kNR * c, kNR, rmask, unit_d(adraw(a.seed, 1, it, (uint32_t)c + (uint32_t)a.prm.chain_base)));
    const int q = qmin + uint_below(adraw(a.seed, 2, it, (uint32_t)c + (uint32_t)a.prm.chain_base), qmax - qmin + 1);
    a.di[c] = di;
    a.ri[c] = ri;
    a.q[c] = q;
    a.aD[kND * c + di] += 1;
    a.aR[kNR * c + ri] += 1;
    a.rstate[c] = 0;
    a.nleft[c] = 0;
    a.nrem[c] = qmin;   // q_min of this chain, read by destroy
}

// Stages a chain's solution (ops + legs) in LDS.  Returns the op count.
template <typename DT>
__device__ int stage_solution(OpStore<DT>& S, const uint16_t* ops, const uint16_t* rt, int m, const DT* D, int N1,
                              int* rs, int* re)
{
    if (threadIdx.x < m) {
        rs[threadIdx.x] = threadIdx.x ? rt[threadIdx.x - 1] : 0;
        re[threadIdx.x] = rt[threadIdx.x];
    }
    __syncthreads();
    const int L = re[m - 1];
    for (int j = threadIdx.x; j < L; j += blockDim.x) S.set_code(j, ops[j]);
    // padding past the last route for the sweeps' unguarded fetches
    for (int j = L + threadIdx.x; j < L + kAlnsStep; j += blockDim.x) S.set(j, 0u, 0);
    __syncthreads();
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const int c = (int)(S.code(j) >> 1);
        const int pc = j > 0 ? (int)(S.code(j - 1) >> 1) : 0;
        S.set_leg(j, (int)D[pc * N1 + c]);
    }
    __syncthreads();
    if (threadIdx.x < m && rs[threadIdx.x] < re[threadIdx.x])
        S.set_leg(rs[threadIdx.x], (int)D[(int)(S.code(rs[threadIdx.x]) >> 1)]);
    __syncthreads();
    return L;
}

// Lane v's view of route v of the staged solution with customer `cust`'s ops
// taken out (cust = 0: nothing removed).  Returns the route and its return leg.
template <typename DT, bool kRec>
__device__ DelRouteT<DT, kRec> del_route(const OpStore<DT>& S, const int* rs, const int* re, int lane, int m,
                                         const uint16_t* posD, const uint16_t* posP, int cust, const DT* D, int N1,
                                         int* times, int& ret)
{
    DelRouteT<DT, kRec> R;
    R.S = &S;
    R.times = times;
    R.y1 = R.y2 = kNoPos;
    R.lb1 = R.lb2 = 0;
    R.bs = 0;
    R.vlen = 0;
    ret = 0;
    if (lane >= m) return R;
    const int s = rs[lane], e = re[lane];
    R.bs = s;
    int r[2], nr = 0;
    if (cust) {
        const int a = posD[cust], b = posP[cust];
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        if (lo >= s && lo < e) r[nr++] = lo - s;
        if (hi >= s && hi < e) r[nr++] = hi - s;
    }
    const int len = e - s;
    R.vlen = len - nr;
    auto cust_at = [&](int rel) { return (int)(S.code(s + rel) >> 1); };
    if (nr >= 1) {
        R.y1 = r[0];
        if (nr == 2) R.y2 = r[1] - 1;
        // legs into the first kept op after each removed one
        const int prev1 = r[0] > 0 ? cust_at(r[0] - 1) : 0;
        if (nr == 2 && r[1] == r[0] + 1) {
            if (r[1] + 1 < len) R.lb2 = (int)D[prev1 * N1 + cust_at(r[1] + 1)];
        } else {
            if (r[0] + 1 < len) R.lb1 = (int)D[prev1 * N1 + cust_at(r[0] + 1)];
            if (nr == 2 && r[1] + 1 < len) R.lb2 = (int)D[cust_at(r[1] - 1) * N1 + cust_at(r[1] + 1)];
        }
    }
    // return leg from the last kept op
    int last = len - 1;
    while (last >= 0 && ((nr >= 1 && last == r[0]) || (nr == 2 && last == r[1]))) --last;
    ret = last >= 0 ? (int)D[cust_at(last) * N1] : 0;
    return R;
}

// ---------------------------------------------------------------- gains
// Block (chain, chunk): z(S without c) for the chunk's customers, one sweep
// per customer per group.  Only chains drawing worst or critical-path removal.
template <typename DT, int GL, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_gains(AlnsDev a, int per_block)
{
    constexpr int G = 64 / GL;
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x;
    const int di = a.di[c];
    if (!a.learn_on && di != 1 && di != 5) return;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1;
    const int c0 = 1 + blockIdx.y * per_block;
    if (c0 > n) return;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane % GL, gidx = wave * G + lane / GL;
    Carve cv{smem};
    int* pblk = cv.take<int>(a.N + 1);
    uint16_t* posD = cv.take<uint16_t>(a.N + 2);
    uint16_t* posP = cv.take<uint16_t>(a.N + 2);
    int* rs = cv.take<int>(kMaxM);
    int* re = cv.take<int>(kMaxM);
    unsigned char* ops_base = cv.take<unsigned char>((size_t)OpStore<DT>::kBytesPerOp * (2 * a.N + kAlnsStep));
    int* ready = cv.take<int>((size_t)WPB * G * (a.N + 1)) + gidx * (a.N + 1);
    OpStore<DT> S;
    S.init(ops_base, 2 * a.N + kAlnsStep);
    for (int x = threadIdx.x; x <= n; x += blockDim.x) pblk[x] = x ? P[x] : 0;
    const uint16_t* sops = a.S_ops + (int64_t)c * 2 * a.N;
    const int L = stage_solution(S, sops, a.S_rt + (int64_t)c * a.M, m, D, N1, rs, re);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const uint32_t cd = S.code(j);
        if (cd & 1u) posP[cd >> 1] = (uint16_t)j;
        else posD[cd >> 1] = (uint16_t)j;
    }
    for (int x = li; x <= n; x += GL) ready[x] = -1;
    __syncthreads();
    int pol = 0;
    const int zS = a.z[c];
    const int c1 = min(n, c0 + per_block - 1);
    int prev = 0;
    for (int cust = c0 + gidx; cust <= c1; cust += WPB * G) {
        // the customer left out last time is back: its entry is stale
        if (li == 0 && prev) ready[prev] = pol ? 0 : -1;
        wave_lds_fence();
        prev = cust;
        int ret;
        const auto R = del_route<DT, false>(S, rs, re, li, m, posD, posP, cust, D, N1, nullptr, ret);
        const SweepOut o = sweep_route<kAlnsStep, GL>(R, ready, pblk, pol);
        pol ^= 1;
        const int rv = (li < m && R.vlen > 0) ? o.t + ret : 0;
        const int zc = group_max<GL>(rv);
        if (li == 0) a.gains[(int64_t)c * (a.N + 1) + cust] = (long long)zS - zc;
    }
    if (threadIdx.x == 0) atomicAdd(a.evals, (unsigned long long)(c1 - c0 + 1));
}

// ---------------------------------------------------------------- destroy
template <typename DT>
__global__ __launch_bounds__(256) void k_destroy(AlnsDev a)
{
    const uint32_t it = *a.it_dev;
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x;
    const int cand = blockIdx.y;                        // candidate: draws at 16 + 4096 cand + i
    const uint32_t db = 16u + 4096u * (uint32_t)cand;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const int di = a.di[c];
    const int q_min = a.nrem[c];
    int q = a.q[c];
    if (q > n) q = n;
    const int npow = pow2_ge(n);
    Carve cv{smem};
    unsigned long long* key = cv.take<unsigned long long>(pow2_ge(a.N));
    int* times = cv.take<int>(2 * a.N + kAlnsStep);
    int* pblk = cv.take<int>(a.N + 1);
    uint16_t* posD = cv.take<uint16_t>(a.N + 2);
    uint16_t* posP = cv.take<uint16_t>(a.N + 2);
    unsigned char* flag = cv.take<unsigned char>(a.N + 1);
    int* rs = cv.take<int>(kMaxM);
    int* re = cv.take<int>(kMaxM);
    int* rem = cv.take<int>(a.Q);
    int* ready = cv.take<int>(a.N + 1);
    unsigned char* ops_base = cv.take<unsigned char>((size_t)OpStore<DT>::kBytesPerOp * (2 * a.N + kAlnsStep));
    __shared__ int sh_cnt;
    OpStore<DT> S;
    S.init(ops_base, 2 * a.N + kAlnsStep);
    const uint16_t* sops = a.S_ops + (int64_t)c * 2 * a.N;
    const uint16_t* srt = a.S_rt + (int64_t)c * a.M;
    const int L = stage_solution(S, sops, srt, m, D, N1, rs, re);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const uint32_t cd = S.code(j);
        if (cd & 1u) posP[cd >> 1] = (uint16_t)j;
        else posD[cd >> 1] = (uint16_t)j;
    }
    for (int x = threadIdx.x; x <= n; x += blockDim.x) {
        pblk[x] = x ? P[x] : 0;
        flag[x] = 0;
        ready[x] = -1;
    }
    if (threadIdx.x == 0) sh_cnt = 0;
    __syncthreads();

    // times of every op of S (Shaw needs drop times, critical path the returns)
    if (di == 2 || di == 5) {
        if (threadIdx.x < 64) {
            int ret;
            const auto R = del_route<DT, true>(S, rs, re, threadIdx.x, m, posD, posP, 0, D, N1, times, ret);
            (void)sweep_route<kAlnsStep, 64>(R, ready, pblk, 0);
        }
    }
    __syncthreads();
    const long long* gain = a.gains + (int64_t)c * (a.N + 1);
    const uint32_t uc = (uint32_t)c + (uint32_t)a.prm.chain_base;
    if (di == 0) {                                   // random: partial Fisher-Yates
        int* perm = reinterpret_cast<int*>(key);
        for (int x = threadIdx.x; x < n; x += blockDim.x) perm[x] = x + 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < q; ++i) {
                const int j = i + uint_below(adraw(a.seed, db + i, it, uc), n - i);
                const int x = perm[i];
                perm[i] = perm[j];
                perm[j] = x;
                rem[i] = perm[i];
            }
            sh_cnt = q;
        }
    } else if (di == 1) {                            // worst: rank by gain, weight 2^60 / r^6
        for (int x = threadIdx.x; x < npow; x += blockDim.x)
            key[x] = x < n ? (((unsigned long long)((1LL << 34) - gain[x + 1]) << 16) | (unsigned)(x + 1)) : ~0ull;
        __syncthreads();
        block_sort_u64(key, npow);
        // rank weights floor(2^60 / r^6) for ranks r <= min(n, 1024) (the
        // times[] space is free for this operator) and their total: integer
        // sums, so summing in parallel gives the same value
        const int nw = n < 1024 ? n : 1024;
        unsigned long long* wt = reinterpret_cast<unsigned long long*>(times);
        __shared__ unsigned long long wtot;
        if (threadIdx.x == 0) wtot = 0;
        __syncthreads();
        {
            unsigned long long part = 0;
            for (int i = threadIdx.x; i < nw; i += blockDim.x) {
                const unsigned long long r = (unsigned long long)(i + 1);
                wt[i] = (1ULL << 60) / (r * r * r * r * r * r);
                part += wt[i];
            }
            atomicAdd(&wtot, part);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            // Roulette over the unflagged ranks, one wave: the first rank
            // whose running weight sum exceeds the draw, found 64 ranks at a
            // time by a wave prefix sum.
            const int lane = threadIdx.x;
            unsigned long long tot = wtot;
            int cnt = 0;
            for (int s2 = 0; s2 < q; ++s2) {
                if (tot == 0) break;
                const unsigned long long w32 = adraw(a.seed, db + s2, it, uc);
                const unsigned long long hi = (w32 * (tot >> 32)) + ((w32 * (tot & 0xFFFFFFFFull)) >> 32);
                unsigned long long base = 0;
                int pick = -1;
                for (int i0 = 0; i0 < nw && pick < 0; i0 += 64) {
                    const int i = i0 + lane;
                    const unsigned long long w = (i < nw && !flag[i]) ? wt[i] : 0ULL;
                    unsigned long long x = w;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const unsigned long long y = __shfl_up(x, o, 64);
                        if (lane >= o) x += y;
                    }
                    const unsigned long long hit = __ballot(w != 0ULL && hi < base + x);
                    if (hit) pick = i0 + __ffsll((long long)hit) - 1;
                    base += __shfl(x, 63, 64);
                }
                tot -= wt[pick];
                if (lane == 0) {
                    flag[pick] = 1;
                    rem[cnt] = (int)(key[pick] & 0xFFFFu);
                }
                ++cnt;
                wave_lds_fence();
            }
            if (lane == 0) sh_cnt = cnt;
        }
    } else if (di == 2 || di == 3) {                 // Shaw, cluster
        const int cen = 1 + uint_below(adraw(a.seed, db, it, uc), n);
        for (int x = threadIdx.x; x < npow; x += blockDim.x) {
            unsigned long long k = ~0ull;
            const int cc = x + 1;
            if (x < n && cc != cen) {
                long long rel;
                if (di == 3) {
                    rel = (long long)D[cen * N1 + cc];
                } else {
                    long long dt = (long long)times[posD[cen]] - times[posD[cc]];
                    dt = dt < 0 ? -dt : dt;
                    auto veh_of = [&](int pos) {
                        int v = 0;
                        while (v < m - 1 && pos >= re[v]) ++v;
                        return v;
                    };
                    rel = 18LL * D[cen * N1 + cc] + 6 * dt + 5 * (veh_of(posD[cen]) != veh_of(posD[cc])) +
                          5 * (veh_of(posP[cen]) != veh_of(posP[cc]));
                }
                k = ((unsigned long long)rel << 16) | (unsigned)cc;
            }
            key[x] = k;
        }
        __syncthreads();
        block_sort_u64(key, npow);
        if (threadIdx.x == 0) {
            int cnt = 0;
            rem[cnt++] = cen;
            for (int i = 0; i < n - 1 && cnt < q; ++i) rem[cnt++] = (int)(key[i] & 0xFFFFu);
            sh_cnt = cnt;
        }
    } else if (di == 4) {                            // route
        if (threadIdx.x == 0) {
            int nonempty = 0;
            for (int v = 0; v < m; ++v) nonempty += re[v] > rs[v];
            const int pickv = uint_below(adraw(a.seed, db, it, uc), nonempty);
            int v = 0;
            for (int seen = -1; v < m; ++v)
                if (re[v] > rs[v] && ++seen == pickv) break;
            int cnt = 0;
            for (int j = rs[v]; j < re[v] && cnt < q; ++j) {
                const int cc = (int)(S.code(j) >> 1);
                if (!flag[cc]) {
                    flag[cc] = 1;
                    rem[cnt++] = cc;
                }
            }
            sh_cnt = cnt;
        }
        __syncthreads();
        const int cnt0 = sh_cnt;
        if (cnt0 < q_min) {
            for (int x = threadIdx.x; x < npow; x += blockDim.x) {
                unsigned long long k = ~0ull;
                const int cc = x + 1;
                if (x < n && !flag[cc]) {
                    long long best = 0x7FFFFFFFFFFFLL;
                    for (int i = 0; i < cnt0; ++i) {
                        const long long dd = (long long)D[rem[i] * N1 + cc];
                        best = dd < best ? dd : best;
                    }
                    k = ((unsigned long long)best << 16) | (unsigned)cc;
                }
                key[x] = k;
            }
            __syncthreads();
            block_sort_u64(key, npow);
            if (threadIdx.x == 0) {
                int cnt = cnt0;
                for (int i = 0; i < n && cnt < q_min && key[i] != ~0ull; ++i) rem[cnt++] = (int)(key[i] & 0xFFFFu);
                sh_cnt = cnt;
            }
        }
    } else {                                         // critical path
        if (threadIdx.x == 0) {
            int bv = -1;
            long long bret = -1;
            for (int v = 0; v < m; ++v) {
                if (re[v] == rs[v]) continue;
                const int last = re[v] - 1;
                const long long r = (long long)times[last] + D[(int)(S.code(last) >> 1) * N1];
                if (r > bret) { bret = r; bv = v; }
            }
            for (int j = rs[bv]; j < re[bv]; ++j) flag[S.code(j) >> 1] = 1;
        }
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int x = threadIdx.x; x < npow; x += blockDim.x) {
                unsigned long long k = ~0ull;
                const int cc = x + 1;
                if (x < n && (flag[cc] != 0) == (pass == 0))
                    k = ((unsigned long long)((1LL << 34) - gain[cc]) << 16) | (unsigned)cc;
                key[x] = k;
            }
            __syncthreads();
            block_sort_u64(key, npow);
            if (threadIdx.x == 0) {
                int cnt = pass == 0 ? 0 : sh_cnt;
                const int lim = pass == 0 ? q : q_min;
                for (int i = 0; i < n && cnt < lim && key[i] != ~0ull; ++i) rem[cnt++] = (int)(key[i] & 0xFFFFu);
                sh_cnt = cnt;
            }
            __syncthreads();
            if (pass == 0 && sh_cnt >= q_min) break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nrem = sh_cnt;
        int32_t* out = a.cand_rem + ((int64_t)c * a.K + cand) * a.Q;
        for (int i = 0; i < nrem; ++i) out[i] = rem[i];
        a.cand_cnt[(int64_t)c * a.K + cand] = nrem;
    }
}

// ---------------------------------------------------------------- apply
// Block per chain: takes one candidate removal set (the plain operator's,
// candidate 0, unless the network picked another) and builds the partial
// solution W = S without it.
template <typename DT>
__global__ __launch_bounds__(256) void k_apply(AlnsDev a, int use_scores)
{
    const uint32_t it = *a.it_dev;
    const int c = blockIdx.x;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int m = I.m, n = I.n;
    __shared__ int pick;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* flag = smem;
    if (threadIdx.x == 0) {
        int k = 0;
        if (use_scores && a.K > 1 && !(unit_d(adraw(a.seed, 3, it, (uint32_t)c + (uint32_t)a.prm.chain_base)) < a.eps)) {
            // lowest predicted makespan change; ties to the lower index
            float best = 0.f;
            for (int j = 0; j < a.K; ++j) {
                const int cnt = a.cand_cnt[(int64_t)c * a.K + j];
                const int32_t* r = a.cand_rem + ((int64_t)c * a.K + j) * a.Q;
                float sc = 0.f;
                for (int i = 0; i < cnt; ++i) sc += a.score[(int64_t)c * a.N + r[i] - 1];
                if (j == 0 || sc < best) {
                    best = sc;
                    k = j;
                }
            }
        }
        pick = k;
        a.chosen[c] = k;
    }
    for (int x = threadIdx.x; x <= n; x += blockDim.x) flag[x] = 0;
    __syncthreads();
    const int k = pick;
    const int nrem = a.cand_cnt[(int64_t)c * a.K + k];
    const int32_t* rem = a.cand_rem + ((int64_t)c * a.K + k) * a.Q;
    for (int i = threadIdx.x; i < nrem; i += blockDim.x) flag[rem[i]] = 1;
    __syncthreads();
    uint16_t* wops = a.W_ops + ((int64_t)2 * c + 0) * 2 * a.N;
    uint16_t* wrt = a.W_rt + ((int64_t)2 * c + 0) * a.M;
    const uint16_t* sops = a.S_ops + (int64_t)c * 2 * a.N;
    const uint16_t* srt = a.S_rt + (int64_t)c * a.M;
    // W = S without the removed customers: kept-op counts per thread chunk,
    // an exclusive scan over the chunks, then every thread copies its chunk
    __shared__ int part[256];
    const int L = srt[m - 1];
    const int per = (L + (int)blockDim.x - 1) / (int)blockDim.x;
    const int j0 = threadIdx.x * per, j1 = min(L, j0 + per);
    int kept = 0;
    for (int j = j0; j < j1; ++j) kept += flag[sops[j] >> 1] ? 0 : 1;
    part[threadIdx.x] = kept;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const int v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int w = part[threadIdx.x] - kept;
    for (int j = j0; j < j1; ++j) {
        const uint16_t x = sops[j];
        if (!flag[x >> 1]) wops[w++] = x;
    }
    if (threadIdx.x < m) {
        // kept ops before route end srt[v]
        const int e = srt[threadIdx.x];
        const int t = per > 0 ? min(e / per, (int)blockDim.x - 1) : 0;
        int cntv = (t > 0 ? part[t - 1] : 0);
        for (int j = t * per; j < e; ++j) cntv += flag[sops[j] >> 1] ? 0 : 1;
        wrt[threadIdx.x] = (uint16_t)cntv;
    }
    if (threadIdx.x == 0) {
        a.W_cur[c] = 0;
        a.base_op_off[c] = ((int64_t)2 * c + 0) * 2 * a.N;
        a.base_rt_off[c] = ((int64_t)2 * c + 0) * a.M;
        a.nrem[c] = nrem;
        a.nleft[c] = nrem;
        for (int i = 0; i < nrem; ++i) {
            a.left[c * a.Q + i] = rem[i];
            a.rem[c * a.Q + i] = rem[i];
        }
        int KD = 0, KP = 0;
        if (a.prm.tuple_budget > 0) {
            long long tc = (long long)a.prm.tuple_budget / ((long long)nrem * (nrem + 1) / 2);
            if (tc < 1) tc = 1;
            KD = (int)floor(sqrt((double)tc));
            if (KD < 1) KD = 1;
            KP = (int)(tc / KD);
            if (KP < 1) KP = 1;
        }
        a.KD[c] = KD;
        a.KP[c] = KP;
        a.rstate[c] = nrem > 0 ? 0 : 1;
    }
}

// ---------------------------------------------------------------- features
// Per-customer features of the learned destroy proposal (the feature list is
// in vrprpd.h).  Every feature is one correctly rounded fp32 division of two
// integers converted once to fp32, then rounded to bfloat16.
__device__ __forceinline__ float fdiv(long long a, long long b) { return __fdiv_rn((float)a, (float)b); }

// Block per chain, once: dbar and the two static features of every customer
// (distance to the nearest other node, mean of the four nearest).
template <typename DT>
__global__ __launch_bounds__(256) void k_static(AlnsDev a)
{
    const int c = blockIdx.x;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    __shared__ long long part[256];
    long long sum = 0;
    for (int x = 1 + threadIdx.x; x <= n; x += blockDim.x) sum += (long long)D[x];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        const long long db = t / n;
        part[0] = db > 1 ? db : 1;
        a.dbar[c] = (int32_t)part[0];
    }
    __syncthreads();
    const long long db = part[0];
    for (int cust = 1 + threadIdx.x; cust <= n; cust += blockDim.x) {
        long long best[4] = {LLONG_MAX, LLONG_MAX, LLONG_MAX, LLONG_MAX};
        for (int j = 0; j <= n; ++j) {
            if (j == cust) continue;
            long long v = (long long)D[(int64_t)cust * N1 + j];
            for (int r = 0; r < 4; ++r) {
                if (v < best[r]) {
                    const long long t = best[r];
                    best[r] = v;
                    v = t;
                }
            }
        }
        const int cnt = n < 4 ? n : 4;    // n other nodes (the depot included)
        long long s4 = 0;
        for (int r = 0; r < cnt; ++r) s4 += best[r];
        float* f = a.fstat + ((int64_t)c * (a.N + 1) + cust) * 2;
        f[0] = fdiv(best[0], db);
        f[1] = fdiv(s4, (long long)cnt * db);
    }
}

// Block per chain: the schedule of S (one recorded sweep), then one thread
// per customer.
template <typename DT>
__global__ __launch_bounds__(256) void k_features(AlnsDev a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1, k = I.k;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    Carve cv{smem};
    int* times = cv.take<int>(2 * a.N + kAlnsStep);
    int* walk = cv.take<int>(2 * a.N + kAlnsStep);
    int* pblk = cv.take<int>(a.N + 1);
    uint16_t* posD = cv.take<uint16_t>(a.N + 2);
    uint16_t* posP = cv.take<uint16_t>(a.N + 2);
    int* rs = cv.take<int>(kMaxM);
    int* re = cv.take<int>(kMaxM);
    int* fin = cv.take<int>(kMaxM);
    int* ready = cv.take<int>(a.N + 1);
    unsigned char* ops_base = cv.take<unsigned char>((size_t)OpStore<DT>::kBytesPerOp * (2 * a.N + kAlnsStep));
    OpStore<DT> S;
    S.init(ops_base, 2 * a.N + kAlnsStep);
    const int L = stage_solution(S, a.S_ops + (int64_t)c * 2 * a.N, a.S_rt + (int64_t)c * a.M, m, D, N1, rs, re);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const uint32_t cd = S.code(j);
        if (cd & 1u) posP[cd >> 1] = (uint16_t)j;
        else posD[cd >> 1] = (uint16_t)j;
    }
    for (int x = threadIdx.x; x <= n; x += blockDim.x) {
        pblk[x] = x ? P[x] : 0;
        ready[x] = -1;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        int ret;
        const auto R = del_route<DT, true>(S, rs, re, threadIdx.x, m, posD, posP, 0, D, N1, times, ret);
        (void)sweep_route<kAlnsStep, 64>(R, ready, pblk, 0);
    }
    __syncthreads();
    if (threadIdx.x < m) {
        const int v = threadIdx.x;
        int w = 0;
        for (int j = rs[v]; j < re[v]; ++j) {
            w += (S.code(j) & 1u) ? -1 : 1;
            walk[j] = w;
        }
        fin[v] = re[v] > rs[v] ? times[re[v] - 1] + (int)D[(int)(S.code(re[v] - 1) >> 1) * N1] : 0;
    }
    __syncthreads();
    const long long z = a.z[c];
    const long long db = a.dbar[c];
    uint16_t* out = a.feat + (int64_t)c * a.N * 64;
    for (int cust = 1 + threadIdx.x; cust <= n; cust += blockDim.x) {
        const int jD = posD[cust], jP = posP[cust];
        int vD = 0, vP = 0;
        while (vD < m - 1 && jD >= re[vD]) ++vD;
        while (vP < m - 1 && jP >= re[vP]) ++vP;
        const int sD = rs[vD], sP = rs[vP];
        const int LD = re[vD] - sD, LP = re[vP] - sP;
        const int iD = jD - sD, iP = jP - sP;
        const int prevD = iD > 0 ? (int)(S.code(jD - 1) >> 1) : 0;
        const int nextD = iD + 1 < LD ? (int)(S.code(jD + 1) >> 1) : 0;
        const int prevP = iP > 0 ? (int)(S.code(jP - 1) >> 1) : 0;
        const int nextP = iP + 1 < LP ? (int)(S.code(jP + 1) >> 1) : 0;
        const long long tD = times[jD], tP = times[jP];
        const long long aP = (iP > 0 ? (long long)times[jP - 1] : 0) + (long long)D[prevP * N1 + cust];
        const long long fD = fin[vD], fP = fin[vP];
        const long long pc = P[cust];
        const long long g = a.gains[(int64_t)c * (a.N + 1) + cust];
        const bool same = vD == vP;
        const long long dpc_D = D[prevD * N1 + cust], dcn_D = D[cust * N1 + nextD];
        const long long dpc_P = D[prevP * N1 + cust], dcn_P = D[cust * N1 + nextP];
        float b[32];
        b[0] = 1.f;
        b[1] = fdiv(D[cust], db);
        b[2] = fdiv(pc, db);
        b[3] = fdiv(tD, z);
        b[4] = fdiv(tP, z);
        b[5] = fdiv(tP - tD - pc, z);
        b[6] = fdiv(tP - aP, z);
        b[7] = same ? 1.f : 0.f;
        b[8] = fdiv(iD, LD);
        b[9] = fdiv(iP, LP);
        b[10] = fdiv(fD, z);
        b[11] = fdiv(fP, z);
        b[12] = fD == z ? 1.f : 0.f;
        b[13] = fP == z ? 1.f : 0.f;
        b[14] = fdiv(dpc_D + dcn_D - (long long)D[prevD * N1 + nextD], db);
        b[15] = fdiv(dpc_P + dcn_P - (long long)D[prevP * N1 + nextP], db);
        b[16] = fdiv(dpc_D, db);
        b[17] = fdiv(dcn_D, db);
        b[18] = fdiv(dpc_P, db);
        b[19] = fdiv(dcn_P, db);
        b[20] = fdiv(g, z);
        b[21] = fdiv(walk[jD], k);
        b[22] = fdiv(walk[jP], k);
        b[23] = fdiv((long long)LD * m, 2LL * n);
        b[24] = fdiv((long long)LP * m, 2LL * n);
        b[25] = same ? fdiv(iP - iD, LD) : 0.f;
        const float* fs = a.fstat + ((int64_t)c * (a.N + 1) + cust) * 2;
        b[26] = fs[0];
        b[27] = fs[1];
        b[28] = fdiv(z - fD, z);
        b[29] = fdiv(z - fP, z);
        b[30] = g > 0 ? 1.f : 0.f;
        b[31] = tP > tD ? fdiv(pc, tP - tD) : 1.f;
        const float gate = (fD == z || fP == z) ? 1.f : 0.f;
        uint16_t* row = out + (int64_t)(cust - 1) * 64;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            row[i] = f2bf(b[i]);
            row[32 + i] = f2bf(b[i] * gate);
        }
    }
}

// ---------------------------------------------------------------- enumerate
// Block (chain, slot i): candidate tuples of the i-th waiting customer
// against the chain's partial solution W, in this order: the drop slots
// ranked by (detour, vehicle, position), the best K_D; for each, the pickup
// slots ranked the same way on the route after the drop went in, the best K_P.
__device__ __forceinline__ unsigned long long slot_key(long long det, int v, int p)
{
    return ((unsigned long long)(det + (1LL << 31)) << 22) | ((unsigned long long)v << 16) | (unsigned)p;
}

template <typename DT>
__global__ __launch_bounds__(256) void k_enum(AlnsDev a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x, slot = blockIdx.y;
    const int sidx = c * a.Q + slot;
    if (threadIdx.x < 3) a.seg_top3[3 * (int64_t)sidx + threadIdx.x] = INT64_MAX;   // the scan merges into it
    if (a.rstate[c] != 0 || slot >= a.nleft[c]) {
        if (threadIdx.x == 0) a.seg_cnt[sidx] = 0;
        return;
    }
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int cust = a.left[c * a.Q + slot];
    const int wb = a.W_cur[c];
    const uint16_t* wops = a.W_ops + ((int64_t)2 * c + wb) * 2 * a.N;
    const uint16_t* wrt = a.W_rt + ((int64_t)2 * c + wb) * a.M;
    __shared__ int rs[kMaxM], re[kMaxM], cum[kMaxM + 1];
    if (threadIdx.x < m) {
        rs[threadIdx.x] = threadIdx.x ? wrt[threadIdx.x - 1] : 0;
        re[threadIdx.x] = wrt[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cum[0] = 0;
        for (int v = 0; v < m; ++v) cum[v + 1] = cum[v] + (re[v] - rs[v]) + 1;
    }
    __syncthreads();
    const int L = re[m - 1];
    const int nslots = L + m;            // drop slots
    const int npow = pow2_ge(nslots + 1);
    unsigned long long* key = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* dsel = key + npow;
    auto cust_at = [&](int j) { return (int)(wops[j] >> 1); };
    auto det = [&](int x, int y) { return (long long)D[x * N1 + cust] + D[cust * N1 + y] - D[x * N1 + y]; };
    for (int k = threadIdx.x; k < npow; k += blockDim.x) {
        unsigned long long kv = ~0ull;
        if (k < nslots) {
            int v = 0;
            while (cum[v + 1] <= k) ++v;
            const int p = k - cum[v], len = re[v] - rs[v];
            const int x = p > 0 ? cust_at(rs[v] + p - 1) : 0;
            const int y = p < len ? cust_at(rs[v] + p) : 0;
            kv = slot_key(det(x, y), v, p);
        }
        key[k] = kv;
    }
    __syncthreads();
    block_sort_u64(key, npow);
    const int KD = a.KD[c], KP = a.KP[c];
    const int nd = (KD > 0 && KD < nslots) ? KD : nslots;
    // Pickup slots after the drop went in at (vD, pD): every other route's
    // slots keep their drop-slot keys; route vD offers the slot right after
    // the drop (detour 0) and its old slots p >= pD + 1, now at p + 1.  A
    // uniform shift of p inside route vD keeps the (detour, vehicle,
    // position) order, so each drop's ranked pickup list is the sorted
    // drop-slot list with route vD's entries p <= pD dropped, the others of
    // vD renumbered, and the new slot merged in: no sort per drop.  There are
    // nslots - pD such slots.
    int* tstart = reinterpret_cast<int*>(dsel);
    for (int di = threadIdx.x; di < nd; di += blockDim.x) {
        const int pD = (int)(key[di] & 0xFFFFu);
        const int cnt = nslots - pD;
        tstart[di] = (KP > 0 && KP < cnt) ? KP : cnt;
    }
    __syncthreads();
    __shared__ int total;
    if (threadIdx.x == 0) {
        int t = 0;
        for (int di = 0; di < nd; ++di) {
            const int np = tstart[di];
            tstart[di] = t;
            t += np;
        }
        total = t;
    }
    __syncthreads();
    vrprpd_tuple* out = a.tuples + (int64_t)sidx * a.TPC;
    for (int di = threadIdx.x; di < nd; di += blockDim.x) {
        const unsigned long long kd = key[di];
        const int vD = (int)((kd >> 16) & 0x3Fu), pD = (int)(kd & 0xFFFFu);
        const int t0 = tstart[di];
        const int np = (di + 1 < nd ? tstart[di + 1] : total) - t0;
        const unsigned long long kw = slot_key(0, vD, pD + 1);
        bool wait_out = false;
        int k = 0;
        for (int got = 0; got < np; ++got) {
            unsigned long long kv = ~0ull;          // next slot of the sorted list that stays a pickup slot
            while (k < nslots) {
                const unsigned long long x = key[k];
                const int v = (int)((x >> 16) & 0x3Fu), p = (int)(x & 0xFFFFu);
                if (v != vD) {
                    kv = x;
                    break;
                }
                if (p > pD) {
                    kv = x + 1;                     // renumbered: position p + 1 (no carry: p < 2^16 - 1)
                    break;
                }
                ++k;                                // at or before the drop: not a pickup slot
            }
            unsigned long long pick;
            if (!wait_out && kw < kv) {
                pick = kw;
                wait_out = true;
            } else {
                pick = kv;
                ++k;
            }
            if (pick == ~0ull) break;
            if (t0 + got < a.TPC) {
                vrprpd_tuple t;
                t.c = (uint16_t)cust;
                t.vD = (uint8_t)vD;
                t.pD = (uint16_t)pD;
                t.vP = (uint8_t)((pick >> 16) & 0x3Fu);
                t.pP = (uint16_t)(pick & 0xFFFFu);
                out[t0 + got] = t;
            }
        }
    }
    const int T = total;
    if (threadIdx.x == 0) a.seg_cnt[sidx] = T < a.TPC ? T : a.TPC;
}

// dst = src with the tuple's drop and pickup spliced in (the insertion the
// scan priced).  Called by every thread of a block.
__device__ void splice_tuple(const uint16_t* src, const uint16_t* srt, int m, const vrprpd_tuple tp, uint16_t* dst,
                             uint16_t* drt)
{
    __shared__ int nstart[kMaxM + 1], sstart[kMaxM];
    __syncthreads();
    if (threadIdx.x == 0) {
        int w = 0;
        for (int v = 0; v < m; ++v) {
            nstart[v] = w;
            sstart[v] = v ? srt[v - 1] : 0;
            const int len = srt[v] - sstart[v];
            w += len + (v == tp.vD) + (v == tp.vP);
            drt[v] = (uint16_t)w;
        }
        nstart[m] = w;
    }
    __syncthreads();
    // every output position at once: its route v, the virtual index i on it,
    // and the inserted ops at virtual positions x1 < x2 of that route
    const int total = nstart[m];
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        int v = 0;
        while (nstart[v + 1] <= p) ++v;
        const int i = p - nstart[v];
        int x1 = kNoPos, x2 = kNoPos;
        uint16_t k1 = 0, k2 = 0;
        if (v == tp.vD && v == tp.vP) { x1 = tp.pD; k1 = (uint16_t)(tp.c << 1); x2 = tp.pP; k2 = (uint16_t)((tp.c << 1) | 1); }
        else if (v == tp.vD) { x1 = tp.pD; k1 = (uint16_t)(tp.c << 1); }
        else if (v == tp.vP) { x1 = tp.pP; k1 = (uint16_t)((tp.c << 1) | 1); }
        dst[p] = i == x1 ? k1 : (i == x2 ? k2 : src[sstart[v] + i - (i > x1) - (i > x2)]);
    }
}

// ---------------------------------------------------------------- select
// Block per chain: price every waiting customer from the scan results, pick
// one by the repair operator's rule, insert it into W.
__global__ __launch_bounds__(256) void k_select(AlnsDev a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x;
    if (a.rstate[c] != 0) return;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int m = I.m;
    const int nl = a.nleft[c], ri = a.ri[c];
    const int kreg = ri == 1 ? 2 : ri == 2 ? 3 : m;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    // per waiting customer: its best makespan c1 and regret (LDS, [Q] each)
    long long* c1s = reinterpret_cast<long long*>(smem);
    long long* regs = c1s + a.Q;
    __shared__ long long opt[4][kMaxM];
    __shared__ unsigned long long evals;
    __shared__ int best_i, fail;
    __shared__ long long best_key;
    if (threadIdx.x == 0) {
        fail = 0;
        evals = 0;
    }
    __syncthreads();
    {
        unsigned long long part = 0;
        for (int i = threadIdx.x; i < nl; i += blockDim.x) part += (unsigned long long)a.seg_cnt[c * a.Q + i];
        atomicAdd(&evals, part);
    }
    // One wave per customer: the best tuple of each drop vehicle (for the
    // regret), then the regret over the kreg best vehicles.
    for (int i = wave; i < nl; i += nw) {
        const int sidx = c * a.Q + i;
        const long long key0 = a.seg_top3[3 * sidx];
        if (key0 == INT64_MAX) {
            if (lane == 0) fail = 1;
            continue;
        }
        c1s[i] = key0 >> 32;
        if (ri == 0) continue;
        long long* o = opt[wave];
        if (lane < m) o[lane] = kBigC;
        wave_lds_fence();
        const int cnt = a.seg_cnt[sidx];
        const int64_t t0 = a.seg_off[sidx];
        for (int k = lane; k < cnt; k += 64) {
            if (a.tst[t0 + k] != 0) continue;
            atomicMin((unsigned long long*)&o[a.tuples[t0 + k].vD], (unsigned long long)a.tmk[t0 + k]);
        }
        wave_lds_fence();
        // regret = sum over the kreg best vehicles (kBigC past m) of their
        // best minus the overall best: the kk = min(kreg, m) smallest of
        // o[0..m) by rank, summed across the wave
        {
            const long long ov = lane < m ? o[lane] : 0;
            int rank = 0;
            if (lane < m)
                for (int u = 0; u < m; ++u) {
                    const long long x = o[u];
                    rank += (x < ov || (x == ov && u < lane)) ? 1 : 0;
                }
            const int kk = kreg < m ? kreg : m;
            long long sum = (lane < m && rank < kk) ? ov : 0;
            long long mn = lane < m ? ov : LLONG_MAX;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                sum += __shfl_xor(sum, off, 64);
                const long long y = __shfl_xor(mn, off, 64);
                mn = y < mn ? y : mn;
            }
            if (lane == 0) regs[i] = sum - (long long)kk * mn + (long long)(kreg > m ? kreg - m : 0) * (kBigC - mn);
        }
        wave_lds_fence();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(a.evals, evals);
        // greedy: the lowest best makespan; regret: the largest regret, then
        // the lower best makespan; ties to the earlier customer
        int bi = -1;
        for (int i = 0; i < nl && !fail; ++i) {
            bool better;
            if (bi < 0) better = true;
            else if (ri == 0) better = c1s[i] < c1s[bi];
            else better = regs[i] > regs[bi] || (regs[i] == regs[bi] && c1s[i] < c1s[bi]);
            if (better) bi = i;
        }
        best_i = bi;
        if (bi >= 0) best_key = a.seg_top3[3 * (c * a.Q + bi)];
    }
    __syncthreads();
    if (fail) {
        if (threadIdx.x == 0) {
            a.rstate[c] = 2;
            a.zn[c] = INT32_MAX;
        }
        return;
    }
    // insert the chosen tuple into the other W buffer
    const vrprpd_tuple tp = a.tuples[(uint32_t)(best_key & 0xFFFFFFFFll)];
    const int wb = a.W_cur[c];
    splice_tuple(a.W_ops + ((int64_t)2 * c + wb) * 2 * a.N, a.W_rt + ((int64_t)2 * c + wb) * a.M, m, tp,
                 a.W_ops + ((int64_t)2 * c + (wb ^ 1)) * 2 * a.N, a.W_rt + ((int64_t)2 * c + (wb ^ 1)) * a.M);
    __syncthreads();
    if (threadIdx.x == 0) {
        a.W_cur[c] = wb ^ 1;
        a.base_op_off[c] = ((int64_t)2 * c + (wb ^ 1)) * 2 * a.N;
        a.base_rt_off[c] = ((int64_t)2 * c + (wb ^ 1)) * a.M;
        a.zn[c] = (int)(best_key >> 32);
        int* lf = a.left + c * a.Q;
        for (int i = best_i; i + 1 < nl; ++i) lf[i] = lf[i + 1];
        a.nleft[c] = nl - 1;
        if (nl - 1 == 0) a.rstate[c] = 1;
    }
}

// ---------------------------------------------------------------- local search
// Periodic local search on each chain's current solution (Section 4.2.6):
// kind 0 pickup repositioning, kind 1 cross-agent relocation.  A pass is
// setup (schedule, candidates, one base S without the candidate per
// candidate), enumeration of ranked tuples per candidate, the insertion scan
// over all (chain, candidate) segments, and apply (the best strictly
// improving move replaces S).  A chain whose pass finds nothing stops.
constexpr int kLsMaxCand = 256;

__global__ void k_ls_begin(AlnsDev a, int reset_any, int use_stop)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    a.ls_active[c] = use_stop ? !a.ls_stop[c] : 1;
    if (reset_any) a.ls_any[c] = 0;
}

// Refinement (the construction's last phase): a chain whose round improved
// nothing stops; every chain starts its annealing at T0 times the refined
// makespan.
__global__ void k_refine_round_end(AlnsDev a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    if (!a.ls_any[c]) a.ls_stop[c] = 1;
}

__global__ void k_refine_temperature(AlnsDev a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const double T = a.prm.T0 * (double)a.z[c];
    a.T[c] = T;
    a.T_init[c] = T;
}

template <typename DT>
__global__ __launch_bounds__(256) void k_ls_setup(AlnsDev a, int kind)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x;
    if (!a.ls_active[c]) {              // nothing to scan for this chain
        for (int i = threadIdx.x; i < a.LQ; i += blockDim.x) a.ls_seg_cnt[(int64_t)c * a.LQ + i] = 0;
        return;
    }
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    Carve cv{smem};
    int* times = cv.take<int>(2 * a.N + kAlnsStep);
    int* pblk = cv.take<int>(a.N + 1);
    uint16_t* posD = cv.take<uint16_t>(a.N + 2);
    uint16_t* posP = cv.take<uint16_t>(a.N + 2);
    int* rs = cv.take<int>(kMaxM);
    int* re = cv.take<int>(kMaxM);
    long long* fin = cv.take<long long>(kMaxM);
    int* ready = cv.take<int>(a.N + 1);
    unsigned char* seen = cv.take<unsigned char>(a.N + 1);
    int* cand = cv.take<int>(kLsMaxCand);
    unsigned char* ops_base = cv.take<unsigned char>((size_t)OpStore<DT>::kBytesPerOp * (2 * a.N + kAlnsStep));
    __shared__ int sh_nc;
    OpStore<DT> S;
    S.init(ops_base, 2 * a.N + kAlnsStep);
    const int L = stage_solution(S, a.S_ops + (int64_t)c * 2 * a.N, a.S_rt + (int64_t)c * a.M, m, D, N1, rs, re);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const uint32_t cd = S.code(j);
        if (cd & 1u) posP[cd >> 1] = (uint16_t)j;
        else posD[cd >> 1] = (uint16_t)j;
    }
    for (int x = threadIdx.x; x <= n; x += blockDim.x) {
        pblk[x] = x ? P[x] : 0;
        ready[x] = -1;
        seen[x] = 0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        int ret;
        const auto R = del_route<DT, true>(S, rs, re, threadIdx.x, m, posD, posP, 0, D, N1, times, ret);
        (void)sweep_route<kAlnsStep, 64>(R, ready, pblk, 0);
    }
    __syncthreads();
    if (threadIdx.x < m) {
        const int v = threadIdx.x;
        fin[v] = re[v] > rs[v] ? (long long)times[re[v] - 1] + (long long)D[(int)(S.code(re[v] - 1) >> 1) * N1] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long z = 0;
        int b = 0;
        for (int v = 0; v < m; ++v) {
            if (fin[v] > z) z = fin[v];
            if (fin[v] > fin[b]) b = v;
        }
        int nc = 0;
        if (kind == 0) {
            for (int v = 0; v < m && nc < kLsMaxCand; ++v) {
                if (20 * fin[v] < 19 * z) continue;
                for (int j = rs[v]; j < re[v] && nc < kLsMaxCand; ++j)
                    if (S.code(j) & 1u) cand[nc++] = (int)(S.code(j) >> 1);
            }
        } else {
            for (int j = rs[b]; j < re[b] && nc < kLsMaxCand; ++j) {
                const int cu = (int)(S.code(j) >> 1);
                if (!seen[cu]) {
                    seen[cu] = 1;
                    cand[nc++] = cu;
                }
            }
        }
        sh_nc = nc;
        a.ls_nc[c] = nc;
        a.ls_b[c] = b;
        if (nc == 0) {
            a.ls_active[c] = 0;
        } else {
            long long T = (long long)a.prm.ls_budget / nc;
            if (T < 1) T = 1;
            int KD = (int)floor(sqrt((double)T));
            if (KD < 1) KD = 1;
            int KP = (int)(T / KD);
            if (KP < 1) KP = 1;
            a.ls_T[c] = (int)T;
            a.ls_KD[c] = KD;
            a.ls_KP[c] = KP;
        }
    }
    __syncthreads();
    const int nc = sh_nc;
    const int T = nc ? a.ls_T[c] : 0;
    for (int i = 0; i < a.LQ; ++i) {
        const int64_t idx = (int64_t)c * a.LQ + i;
        if (i >= nc) {
            if (threadIdx.x == 0) {
                a.ls_seg_cnt[idx] = 0;
                a.ls_seg_off[idx] = (int64_t)c * a.LB;
            }
            continue;
        }
        const int cu = cand[i];
        const int jd = posD[cu], jp = posP[cu];
        const int lo = jd < jp ? jd : jp, hi = jd < jp ? jp : jd;
        uint16_t* bo = a.ls_ops + idx * 2 * a.N;
        uint16_t* br = a.ls_rt + idx * a.M;
        for (int j = threadIdx.x; j < L - 2; j += blockDim.x) {
            const int src = j + (j >= lo) + (j >= hi - 1);
            bo[j] = (uint16_t)S.code(src);
        }
        if (threadIdx.x < m) {
            const int e = re[threadIdx.x];
            br[threadIdx.x] = (uint16_t)(e - (lo < e) - (hi < e));
        }
        if (threadIdx.x == 0) {
            int vD = 0;
            while (vD < m - 1 && jd >= re[vD]) ++vD;
            a.ls_cand[idx] = cu;
            a.ls_pd[idx] = (vD << 16) | (jd - rs[vD]);
            a.ls_seg_off[idx] = (int64_t)c * a.LB + (int64_t)i * T;
            a.ls_base_off[idx] = idx * 2 * a.N;
            a.ls_rt_off[idx] = idx * a.M;
            a.ls_base_inst[idx] = a.chain_inst[c];
        }
    }
}

// Block (chain, candidate): the candidate's ranked tuples against its base.
template <typename DT>
__global__ __launch_bounds__(256) void k_ls_enum(AlnsDev a, int kind)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x, i = blockIdx.y;
    const int64_t idx = (int64_t)c * a.LQ + i;
    if (threadIdx.x < 3) a.ls_top3[3 * idx + threadIdx.x] = INT64_MAX;   // the scan merges into it
    if (!a.ls_active[c] || i >= a.ls_nc[c]) return;   // ls_seg_cnt is 0 there (setup)
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int cust = a.ls_cand[idx];
    const uint16_t* wops = a.ls_ops + idx * 2 * a.N;
    const uint16_t* wrt = a.ls_rt + idx * a.M;
    const int T = a.ls_T[c], KD = a.ls_KD[c], KP = a.ls_KP[c], bveh = a.ls_b[c];
    __shared__ int rs[kMaxM], re[kMaxM], cum[kMaxM + 1];
    if (threadIdx.x < m) {
        rs[threadIdx.x] = threadIdx.x ? wrt[threadIdx.x - 1] : 0;
        re[threadIdx.x] = wrt[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cum[0] = 0;
        for (int v = 0; v < m; ++v) cum[v + 1] = cum[v] + (re[v] - rs[v]) + 1;
    }
    __syncthreads();
    const int L = re[m - 1];
    const int nslots = L + m;
    const int npow = pow2_ge(nslots + 1);
    unsigned long long* key = reinterpret_cast<unsigned long long*>(smem);
    int* dl = reinterpret_cast<int*>(key + npow);     // chosen drop slots (index into key[])
    int* tstart = dl + npow;
    auto cust_at = [&](int j) { return (int)(wops[j] >> 1); };
    auto det = [&](int x, int y) { return (long long)D[x * N1 + cust] + D[cust * N1 + y] - D[x * N1 + y]; };
    for (int k = threadIdx.x; k < npow; k += blockDim.x) {
        unsigned long long kv = ~0ull;
        if (k < nslots) {
            int v = 0;
            while (cum[v + 1] <= k) ++v;
            const int p = k - cum[v], len = re[v] - rs[v];
            const int x = p > 0 ? cust_at(rs[v] + p - 1) : 0;
            const int y = p < len ? cust_at(rs[v] + p) : 0;
            kv = slot_key(det(x, y), v, p);
        }
        key[k] = kv;
    }
    __syncthreads();
    block_sort_u64(key, npow);
    __shared__ int nd, total;
    __shared__ unsigned long long fixed_drop;
    if (threadIdx.x == 0) {
        if (kind == 0) {
            const int pd = a.ls_pd[idx];
            fixed_drop = slot_key(0, pd >> 16, pd & 0xFFFF);   // only (vehicle, position) are read
            nd = 1;
        } else {
            int cnt = 0;
            for (int k = 0; k < nslots && cnt < KD; ++k)
                if ((int)((key[k] >> 16) & 0x3Fu) != bveh) dl[cnt++] = k;
            nd = cnt;
        }
        // tuples per drop, then their offsets
        int t = 0;
        for (int di = 0; di < nd; ++di) {
            const unsigned long long kd = kind == 0 ? fixed_drop : key[dl[di]];
            const int vD = (int)((kd >> 16) & 0x3Fu), pD = (int)(kd & 0xFFFFu);
            int cnt;
            if (kind == 0) {
                cnt = nslots - pD;
                if (cnt > T) cnt = T;
            } else {
                cnt = (re[vD] - rs[vD]) + 1 - pD;   // slots after the drop on its own route
                if (cnt > KP) cnt = KP;
            }
            tstart[di] = t;
            t += cnt;
        }
        total = t;
    }
    __syncthreads();
    vrprpd_tuple* out = a.ls_tuples + a.ls_seg_off[idx];
    for (int di = threadIdx.x; di < nd; di += blockDim.x) {
        const unsigned long long kd = kind == 0 ? fixed_drop : key[dl[di]];
        const int vD = (int)((kd >> 16) & 0x3Fu), pD = (int)(kd & 0xFFFFu);
        const int t0 = tstart[di];
        const int np = (di + 1 < nd ? tstart[di + 1] : total) - t0;
        const unsigned long long kw = slot_key(0, vD, pD + 1);
        bool wait_out = false;
        int k = 0;
        for (int got = 0; got < np; ++got) {
            unsigned long long kv = ~0ull;
            while (k < nslots) {
                const unsigned long long x = key[k];
                const int v = (int)((x >> 16) & 0x3Fu), p = (int)(x & 0xFFFFu);
                if (v != vD) {
                    if (kind == 0) {
                        kv = x;
                        break;
                    }
                } else if (p > pD) {
                    kv = x + 1;
                    break;
                }
                ++k;
            }
            unsigned long long pick;
            if (!wait_out && kw < kv) {
                pick = kw;
                wait_out = true;
            } else {
                pick = kv;
                ++k;
            }
            if (pick == ~0ull) break;
            vrprpd_tuple tt;
            tt.c = (uint16_t)cust;
            tt.vD = (uint8_t)vD;
            tt.pD = (uint16_t)pD;
            tt.vP = (uint8_t)((pick >> 16) & 0x3Fu);
            tt.pP = (uint16_t)(pick & 0xFFFFu);
            out[t0 + got] = tt;
        }
    }
    if (threadIdx.x == 0) a.ls_seg_cnt[idx] = total;
}

// Block per chain: the best strictly improving move of the pass replaces S.
__global__ __launch_bounds__(256) void k_ls_apply(AlnsDev a)
{
    const int c = blockIdx.x;
    if (!a.ls_active[c]) return;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int m = I.m;
    __shared__ long long best;
    __shared__ int take;
    if (threadIdx.x == 0) {
        const int nc = a.ls_nc[c];
        long long b = INT64_MAX;
        unsigned long long tot = 0;
        for (int i = 0; i < nc; ++i) {
            const int64_t idx = (int64_t)c * a.LQ + i;
            const long long k0 = a.ls_top3[3 * idx];
            b = k0 < b ? k0 : b;
            tot += (unsigned long long)a.ls_seg_cnt[idx];
        }
        atomicAdd(a.evals, tot);
        take = b != INT64_MAX && (b >> 32) < (long long)a.z[c];
        best = b;
        if (!take) a.ls_active[c] = 0;
    }
    __syncthreads();
    if (!take) return;
    const int64_t t = best & 0xFFFFFFFFll;
    const int i = (int)((t - (int64_t)c * a.LB) / a.ls_T[c]);
    const int64_t idx = (int64_t)c * a.LQ + i;
    const vrprpd_tuple tp = a.ls_tuples[t];
    splice_tuple(a.ls_ops + idx * 2 * a.N, a.ls_rt + idx * a.M, m, tp, a.S_ops + (int64_t)c * 2 * a.N,
                 a.S_rt + (int64_t)c * a.M);
    if (threadIdx.x == 0) {
        a.z[c] = (int)(best >> 32);
        a.ls_any[c] = 1;
    }
}

// Block per chain: a local search that produced a new best keeps it.
__global__ __launch_bounds__(256) void k_ls_finish(AlnsDev a)
{
    const int c = blockIdx.x;
    if (!a.ls_any[c] || a.z[c] >= a.zb[c]) return;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int m = I.m;
    const int L = a.S_rt[(int64_t)c * a.M + m - 1];
    for (int j = threadIdx.x; j < L; j += blockDim.x) a.B_ops[(int64_t)c * 2 * a.N + j] = a.S_ops[(int64_t)c * 2 * a.N + j];
    for (int v = threadIdx.x; v < m; v += blockDim.x) a.B_rt[(int64_t)c * a.M + v] = a.S_rt[(int64_t)c * a.M + v];
    __syncthreads();
    if (threadIdx.x == 0) {
        a.zb[c] = a.z[c];
        a.stag[c] = 0;
    }
}

// ---------------------------------------------------------------- accept
__global__ __launch_bounds__(256) void k_accept(AlnsDev a)
{
    const uint32_t it = *a.it_dev;
    const int64_t trace_it = a.trace ? (int64_t)it - a.trace_base : -1;
    const int c = blockIdx.x;
    const InstDev I = a.inst_tab[a.chain_inst[c]];
    const int m = I.m;
    __shared__ int copyS, copyB;
    __shared__ int64_t rec_slot;
    if (threadIdx.x == 0) {
        const alns_params& P = a.prm;
        const int di = a.di[c], ri = a.ri[c];
        const bool ok = a.rstate[c] == 1;
        const int z_before = a.z[c];
        const int zn = ok ? a.zn[c] : INT32_MAX;
        int accepted = 0;
        copyS = copyB = 0;
        double* T = a.T + c;
        if (ok) {
            if (zn < a.z[c]) {
                a.z[c] = zn;
                a.sD[kND * c + di] += P.sigma2;
                a.sR[kNR * c + ri] += P.sigma2;
                accepted = 1;
                copyS = 1;
                if (zn < a.zb[c]) {
                    a.zb[c] = zn;
                    a.sD[kND * c + di] += P.sigma1 - P.sigma2;
                    a.sR[kNR * c + ri] += P.sigma1 - P.sigma2;
                    a.stag[c] = 0;
                    accepted = 2;
                    copyB = 1;
                }
            } else {
                const double u = unit_d(adraw(a.seed, 8, it, (uint32_t)c + (uint32_t)a.prm.chain_base));
                const double pacc = det_exp(-((double)zn - (double)a.z[c]) / *T);
                if (u < pacc) {
                    a.z[c] = zn;
                    a.sD[kND * c + di] += P.sigma3;
                    a.sR[kNR * c + ri] += P.sigma3;
                    accepted = 3;
                    copyS = 1;
                }
            }
        }
        *T = P.alpha * *T;
        a.stag[c] += 1;
        if (a.stag[c] >= P.stag_limit && *T < P.gate * a.T_init[c]) {
            *T = P.reheat * P.T0 * (double)a.zb[c];
            a.stag[c] = 0;
        }
        if ((it + 1) % (uint32_t)P.tau == 0) {
            for (int i = 0; i < kND; ++i) {
                const int k = kND * c + i;
                if (a.aD[k] > 0) {
                    const double w = (1.0 - P.r) * a.wD[k] + P.r * ((double)a.sD[k] / (double)a.aD[k]);
                    a.wD[k] = w > P.w_min ? w : P.w_min;
                }
                a.sD[k] = 0;
                a.aD[k] = 0;
            }
            for (int i = 0; i < kNR; ++i) {
                const int k = kNR * c + i;
                if (a.aR[k] > 0) {
                    const double w = (1.0 - P.r) * a.wR[k] + P.r * ((double)a.sR[k] / (double)a.aR[k]);
                    a.wR[k] = w > P.w_min ? w : P.w_min;
                }
                a.sR[k] = 0;
                a.aR[k] = 0;
            }
        }
        rec_slot = -1;
        if (a.rec_x) {
            const int64_t slot = ((int64_t)it - a.rec_base) * a.C + c;
            if (slot >= 0 && slot < a.rec_cap) {
                rec_slot = slot;
                const int nr = ok ? a.nrem[c] : 0;
                a.rec_n[slot] = nr;
                a.rec_t[slot] = ok ? (float)(((double)zn - (double)z_before) / (double)z_before) : 0.f;
            }
        }
        if (a.trace && trace_it >= 0 && trace_it < a.trace_cap) {
            int64_t* tr = a.trace + ((int64_t)c * a.trace_cap + trace_it) * 4;
            tr[0] = zn;
            tr[1] = a.z[c];
            tr[2] = a.zb[c];
            tr[3] = (int64_t)di | ((int64_t)ri << 8) | ((int64_t)accepted << 16) | ((int64_t)a.nrem[c] << 24);
        }
    }
    __syncthreads();
    if (rec_slot >= 0) {
        // the removed customers' feature rows, as they were before the destroy
        const int nr = a.rec_n[rec_slot];
        uint16_t* dst = a.rec_x + rec_slot * a.Q * 64;
        for (int e = threadIdx.x; e < nr * 64; e += blockDim.x) {
            const int cust = a.rem[c * a.Q + e / 64];
            dst[e] = a.feat[((int64_t)c * a.N + cust - 1) * 64 + (e & 63)];
        }
    }
    if (copyS || copyB) {
        const int wb = a.W_cur[c];
        const uint16_t* wops = a.W_ops + ((int64_t)2 * c + wb) * 2 * a.N;
        const uint16_t* wrt = a.W_rt + ((int64_t)2 * c + wb) * a.M;
        const int L = wrt[m - 1];
        for (int j = threadIdx.x; j < L; j += blockDim.x) {
            if (copyS) a.S_ops[(int64_t)c * 2 * a.N + j] = wops[j];
            if (copyB) a.B_ops[(int64_t)c * 2 * a.N + j] = wops[j];
        }
        for (int v = threadIdx.x; v < m; v += blockDim.x) {
            if (copyS) a.S_rt[(int64_t)c * a.M + v] = wrt[v];
            if (copyB) a.B_rt[(int64_t)c * a.M + v] = wrt[v];
        }
    }
}

// ---------------------------------------------------------------- import
// Block per instance: chains [c0, c0 + cpi) adopt the best of them.
__global__ __launch_bounds__(256) void k_import(AlnsDev a, int cpi)
{
    if (a.prm.import_interval <= 0 || (*a.it_dev + 1) % (uint32_t)a.prm.import_interval != 0) return;
    const int c0 = blockIdx.x * cpi;
    __shared__ int bc;
    if (threadIdx.x == 0) {
        bc = c0;
        for (int c = c0 + 1; c < c0 + cpi; ++c)
            if (a.zb[c] < a.zb[bc]) bc = c;
    }
    __syncthreads();
    const InstDev I = a.inst_tab[a.chain_inst[c0]];
    const int m = I.m;
    const int L = a.B_rt[(int64_t)bc * a.M + m - 1];
    for (int c = c0; c < c0 + cpi; ++c) {
        if (a.zb[c] <= a.zb[bc]) continue;
        for (int j = threadIdx.x; j < L; j += blockDim.x) {
            const uint16_t x = a.B_ops[(int64_t)bc * 2 * a.N + j];
            a.B_ops[(int64_t)c * 2 * a.N + j] = x;
            a.S_ops[(int64_t)c * 2 * a.N + j] = x;
        }
        for (int v = threadIdx.x; v < m; v += blockDim.x) {
            const uint16_t x = a.B_rt[(int64_t)bc * a.M + v];
            a.B_rt[(int64_t)c * a.M + v] = x;
            a.S_rt[(int64_t)c * a.M + v] = x;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.zb[c] = a.zb[bc];
            a.z[c] = a.zb[bc];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- records
constexpr uint32_t kTagBatch = 0x42544348u;

__device__ __forceinline__ int64_t batch_slot(uint64_t seed, int i, int64_t count)
{
    const uint64_t w = ((uint64_t)philox_word(seed, (uint32_t)i, 1, 0, kTagBatch) << 32) |
                       philox_word(seed, (uint32_t)i, 0, 0, kTagBatch);
    return (int64_t)(w % (uint64_t)count);
}

// One block: set i of the batch is record slot batch_slot(i) (uniform, with
// replacement); its rows start at seg_off[i].
__global__ __launch_bounds__(1024) void k_batch_index(AlnsDev a, int S, uint64_t seed, int64_t count, int64_t* seg_off,
                                                      float* target)
{
    __shared__ int64_t carry;
    __shared__ int64_t part[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < S; base += 1024) {
        const int i = base + threadIdx.x;
        int64_t nr = 0;
        if (i < S) {
            const int64_t slot = batch_slot(seed, i, count);
            nr = a.rec_n[slot];
            target[i] = a.rec_t[slot];
        }
        part[threadIdx.x] = nr;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < S) seg_off[i] = carry + part[threadIdx.x] - nr;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) seg_off[S] = carry;
}

__global__ __launch_bounds__(256) void k_batch_rows(AlnsDev a, uint64_t seed, int64_t count, const int64_t* seg_off,
                                                   uint16_t* x)
{
    const int i = blockIdx.x;
    const int64_t slot = batch_slot(seed, i, count);
    const int64_t r0 = seg_off[i];
    const int nr = (int)(seg_off[i + 1] - r0);
    const uint16_t* src = a.rec_x + slot * a.Q * 64;
    for (int e = threadIdx.x; e < nr * 64; e += blockDim.x) x[r0 * 64 + e] = src[e];
}

// ---------------------------------------------------------------- tick
__global__ void k_tick(AlnsDev a)
{
    if (threadIdx.x == 0) *a.it_dev += 1u;
}

}  // namespace vrprpd

// ============================================================== host side

struct alns_state {
    const vrprpd_set* set = nullptr;
    vrprpd::AlnsDev d{};
    int32_t n_inst = 0, cpi = 0;       // instances, chains per instance
    int64_t it = 0;                    // iterations done
    int dist16 = 1;
    std::vector<void*> allocs;
    int lds_gain = 0, lds_destroy = 0, lds_enum = 0, lds_feat = 0;
    vrprpd_mlp* mlp = nullptr;         // learned destroy proposal's network (not owned)
    int32_t cand_cap = 1;              // candidates the cand_* buffers hold
    std::vector<void*> rec_allocs;     // record buffers (freed when recording restarts)
    bool use_graph = true;             // replay a captured iteration (alns_set_graph)
    hipStream_t cap = nullptr;         // capture stream (default priority)
    hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};        // per local-search mask
    hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};    // rebuilt after any change of the launch arguments
    int lds_ls = 0;
    std::vector<int32_t> inst_ids;     // host copy of the instances (checkpoint check)
    int scan_tpb = 16;                 // tuples per workgroup of the repair rounds' insertion scans
};

namespace vrprpd {

template <typename DT>
static int set_attributes(alns_state* s);

static int alloc_dev(alns_state* s, void** p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return hip_error(e, "alns_state_create: hipMalloc");
    s->allocs.push_back(*p);
    e = hipMemset(*p, 0, bytes);
    if (e != hipSuccess) return hip_error(e, "alns_state_create: hipMemset");
    return VRPRPD_OK;
}

template <typename T>
static int alloc_n(alns_state* s, T** p, size_t n)
{
    return alloc_dev(s, reinterpret_cast<void**>(p), n * sizeof(T));
}

static int tpc_bound(const alns_params& P, int n, int m, int qmin)
{
    if (P.tuple_budget <= 0) {
        const long long s = 2LL * n + m;
        return (int)(s * (s + 1));
    }
    int best = 1;
    for (int nrem = (qmin > 1 ? qmin : 1); nrem <= n; ++nrem) {
        long long tc = (long long)P.tuple_budget / ((long long)nrem * (nrem + 1) / 2);
        if (tc < 1) tc = 1;
        int KD = (int)std::floor(std::sqrt((double)tc));
        if (KD < 1) KD = 1;
        int KP = (int)(tc / KD);
        if (KP < 1) KP = 1;
        if (KD * KP > best) best = KD * KP;
        if (tc == 1) break;
    }
    return best;
}

static void qrange(const alns_params& P, int n, int* qmin, int* qmax)
{
    int a = P.q_min, b = P.q_max;
    if (a <= 0 || b <= 0) {
        b = n / 20;
        if (b < 4) b = 4;
        a = b / 2;
        if (a < 4) a = 4;
    }
    if (b > n) b = n;
    if (a > b) a = b;
    *qmin = a;
    *qmax = b;
}

}  // namespace vrprpd

extern "C" int alns_state_destroy(alns_state* s)
{
    if (!s) return VRPRPD_OK;
    // graphs of this state may still be replaying on the caller's streams:
    // let the device finish before their executables and buffers go
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 4; ++i) {
        if (s->gexec[i]) (void)hipGraphExecDestroy(s->gexec[i]);
        if (s->graph[i]) (void)hipGraphDestroy(s->graph[i]);
    }
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (void* p : s->allocs) (void)hipFree(p);
    for (void* p : s->rec_allocs) (void)hipFree(p);
    delete s;
    return VRPRPD_OK;
}

extern "C" int alns_state_create(alns_state** out, const vrprpd_set* set, int32_t n_inst, const int32_t* inst_ids,
                                 int32_t chains_per_inst, const alns_params* params, uint64_t seed,
                                 const uint16_t* init_ops, const uint16_t* init_rt, void* stream)
{
    using namespace vrprpd;
    if (!out) return set_error(VRPRPD_EINVAL, "alns_state_create: out is NULL");
    *out = nullptr;
    if (!set || n_inst < 1 || !inst_ids || chains_per_inst < 1 || !params || !init_ops || !init_rt)
        return set_error(VRPRPD_EINVAL, "alns_state_create: bad arguments");
    const alns_params& P = *params;
    if (P.tau < 1 || !(P.alpha > 0.0) || !(P.T0 > 0.0) || (P.op_mask & 0x3Fu) == 0 || ((P.op_mask >> 8) & 0xFu) == 0)
        return set_error(VRPRPD_EINVAL, "alns_state_create: tau >= 1, alpha > 0, T0 > 0 and at least one "
                                        "destroy and one repair operator are required");
    if (P.ls_repos_interval < 0 || P.ls_reloc_interval < 0 ||
        ((P.ls_repos_interval > 0 || P.ls_reloc_interval > 0) && P.ls_budget < 1))
        return set_error(VRPRPD_EINVAL, "alns_state_create: local-search intervals must be >= 0 and ls_budget >= 1 "
                                        "when one is on");
    int N = 0, M = 0, Q = 0, TPC = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (inst_ids[i] < 0 || inst_ids[i] >= set->num_inst)
            return set_error(VRPRPD_EINVAL, "alns_state_create: instance id %d out of range", inst_ids[i]);
        const InstDev& h = set->host[inst_ids[i]];
        N = std::max(N, h.n);
        M = std::max(M, h.m);
        int a, b;
        qrange(P, h.n, &a, &b);
        Q = std::max(Q, b);
        TPC = std::max(TPC, tpc_bound(P, h.n, h.m, a));
    }
    const int C = n_inst * chains_per_inst;
    if ((long long)C * Q * TPC >= (1LL << 31))
        return set_error(VRPRPD_EINVAL, "alns_state_create: %d chains x %d rounds x %d tuples is too many", C, Q, TPC);
    auto* s = new alns_state();
    s->set = set;
    s->n_inst = n_inst;
    s->inst_ids.assign(inst_ids, inst_ids + n_inst);
    s->cpi = chains_per_inst;
    s->dist16 = set->dist16;
    AlnsDev& d = s->d;
    d.inst_tab = set->d_inst;
    d.dist = set->d_dist;
    d.proc = set->d_proc;
    d.C = C;
    d.N = N;
    d.M = M;
    d.Q = Q;
    d.TPC = TPC;
    d.prm = P;
    d.seed = seed;
    int rc = VRPRPD_OK;
#define A(ptr, n)                                        \
    if (rc == VRPRPD_OK) rc = alloc_n(s, &(ptr), (size_t)(n))
    int32_t* cinst = nullptr;
    A(cinst, C);
    A(d.S_ops, (size_t)C * 2 * N); A(d.S_rt, (size_t)C * M);
    A(d.B_ops, (size_t)C * 2 * N); A(d.B_rt, (size_t)C * M);
    A(d.W_ops, (size_t)2 * C * 2 * N); A(d.W_rt, (size_t)2 * C * M);
    A(d.W_cur, C); A(d.z, C); A(d.zb, C); A(d.zn, C);
    A(d.T, C); A(d.T_init, C); A(d.wD, (size_t)kND * C); A(d.wR, (size_t)kNR * C);
    A(d.sD, (size_t)kND * C); A(d.sR, (size_t)kNR * C); A(d.aD, (size_t)kND * C); A(d.aR, (size_t)kNR * C);
    A(d.stag, C); A(d.di, C); A(d.ri, C); A(d.q, C); A(d.nrem, C); A(d.nleft, C); A(d.KD, C); A(d.KP, C);
    A(d.rstate, C); A(d.rem, (size_t)C * Q); A(d.left, (size_t)C * Q); A(d.gains, (size_t)C * (N + 1));
    A(d.tuples, (size_t)C * Q * TPC); A(d.tmk, (size_t)C * Q * TPC); A(d.tst, (size_t)C * Q * TPC);
    A(d.seg_cnt, (size_t)C * Q); A(d.seg_base, (size_t)C * Q); A(d.seg_off, (size_t)C * Q + 1);
    A(d.seg_top3, (size_t)3 * C * Q); A(d.base_op_off, C); A(d.base_rt_off, C); A(d.evals, 1);
    A(d.cand_rem, (size_t)C * Q); A(d.cand_cnt, C); A(d.chosen, C); A(d.it_dev, 1);
    if (P.ls_budget > 0) {   // periodic local search and refinement
        d.LQ = std::min(N, (int)kLsMaxCand);
        d.LB = (int64_t)P.ls_budget + d.LQ;
        const size_t CL = (size_t)C * d.LQ;
        A(d.ls_ops, CL * 2 * N); A(d.ls_rt, CL * M); A(d.ls_cand, CL); A(d.ls_pd, CL);
        A(d.ls_nc, C); A(d.ls_T, C); A(d.ls_KD, C); A(d.ls_KP, C); A(d.ls_b, C); A(d.ls_active, C); A(d.ls_any, C);
        A(d.ls_stop, C);
        A(d.ls_base_inst, CL); A(d.ls_seg_base, CL); A(d.ls_seg_cnt, CL); A(d.ls_seg_off, CL + 1);
        A(d.ls_base_off, CL); A(d.ls_rt_off, CL); A(d.ls_top3, 3 * CL);
        A(d.ls_tuples, (size_t)C * d.LB); A(d.ls_tmk, (size_t)C * d.LB); A(d.ls_tst, (size_t)C * d.LB);
    }
#undef A
    d.K = 1;
    d.eps = 1.0;
    {
        const auto it = set->alns_scan_tuned.find(std::make_tuple(N, M, (int)P.tuple_budget));
        s->scan_tpb = it != set->alns_scan_tuned.end() ? it->second : kScanTuplesPerBlock;
    }
    if (rc != VRPRPD_OK) {
        alns_state_destroy(s);
        return rc;
    }
    d.chain_inst = cinst;
    // host-side tables
    std::vector<int32_t> hc(C), hsb((size_t)C * Q);
    std::vector<int64_t> hso((size_t)C * Q + 1);
    for (int c = 0; c < C; ++c) hc[c] = inst_ids[c / chains_per_inst];
    for (size_t i = 0; i < (size_t)C * Q; ++i) {
        hsb[i] = (int32_t)(i / Q);
        hso[i] = (int64_t)i * TPC;
    }
    hso[(size_t)C * Q] = (int64_t)C * Q * TPC;
    std::vector<double> w1((size_t)kND * C, 1.0), w2((size_t)kNR * C, 1.0);
    hipError_t e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((e = hipMemcpy(cinst, hc.data(), C * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.seg_base, hsb.data(), hsb.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.seg_off, hso.data(), hso.size() * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.wD, w1.data(), w1.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.wR, w2.data(), w2.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
        alns_state_destroy(s);
        return hip_error(e, "alns_state_create: hipMemcpy");
    }
    if (d.ls_seg_base) {
        std::vector<int32_t> ident((size_t)C * d.LQ);
        for (size_t i = 0; i < ident.size(); ++i) ident[i] = (int32_t)i;
        if ((e = hipMemcpy(d.ls_seg_base, ident.data(), ident.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess) {
            alns_state_destroy(s);
            return hip_error(e, "alns_state_create: hipMemcpy");
        }
    }
    // initial solutions: instance i's solution at init_ops + i * 2N? no: the
    // caller gives one solution per instance, ops at [i * 2 n_max], route ends at [i * m_max]
    for (int c = 0; c < C; ++c) {
        const int i = c / chains_per_inst;
        const InstDev& h = set->host[inst_ids[i]];
        if ((e = hipMemcpyAsync(d.S_ops + (size_t)c * 2 * N, init_ops + (size_t)i * 2 * N, 2 * h.n * sizeof(uint16_t),
                                hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(d.S_rt + (size_t)c * M, init_rt + (size_t)i * M, h.m * sizeof(uint16_t),
                                hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(d.B_ops + (size_t)c * 2 * N, init_ops + (size_t)i * 2 * N, 2 * h.n * sizeof(uint16_t),
                                hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(d.B_rt + (size_t)c * M, init_rt + (size_t)i * M, h.m * sizeof(uint16_t),
                                hipMemcpyDeviceToDevice, st)) != hipSuccess) {
            alns_state_destroy(s);
            return hip_error(e, "alns_state_create: copy of the initial solutions");
        }
    }
    // evaluate the initial solutions; they must be feasible
    std::vector<int64_t> hoff(C), hroff(C);
    for (int c = 0; c < C; ++c) {
        hoff[c] = (int64_t)c * 2 * N;
        hroff[c] = (int64_t)c * M;
    }
    int64_t *doff = nullptr, *droff = nullptr;
    uint32_t* dst = nullptr;
    if ((rc = alloc_n(s, &doff, C)) || (rc = alloc_n(s, &droff, C)) || (rc = alloc_n(s, &dst, C))) {
        alns_state_destroy(s);
        return rc;
    }
    if ((e = hipMemcpy(doff, hoff.data(), C * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(droff, hroff.data(), C * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess) {
        alns_state_destroy(s);
        return hip_error(e, "alns_state_create: hipMemcpy");
    }
    rc = vrprpd_eval(set, C, cinst, doff, d.S_ops, droff, d.S_rt, 0, d.z, dst, stream);
    if (rc == VRPRPD_OK && (e = hipStreamSynchronize(st)) != hipSuccess) rc = hip_error(e, "alns_state_create: sync");
    std::vector<int32_t> hz(C);
    std::vector<uint32_t> hs(C);
    if (rc == VRPRPD_OK && ((e = hipMemcpy(hz.data(), d.z, C * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess ||
                            (e = hipMemcpy(hs.data(), dst, C * sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess))
        rc = hip_error(e, "alns_state_create: hipMemcpy");
    if (rc != VRPRPD_OK) {
        alns_state_destroy(s);
        return rc;
    }
    std::vector<double> hT(C);
    for (int c = 0; c < C; ++c) {
        if (hs[c] != 0) {
            alns_state_destroy(s);
            return set_error(VRPRPD_EINVAL, "alns_state_create: initial solution of chain %d has status %u", c, hs[c]);
        }
        hT[c] = P.T0 * (double)hz[c];
    }
    if ((e = hipMemcpy(d.zb, d.z, C * sizeof(int32_t), hipMemcpyDeviceToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.T, hT.data(), C * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d.T_init, hT.data(), C * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
        alns_state_destroy(s);
        return hip_error(e, "alns_state_create: hipMemcpy");
    }
    // LDS sizes of the kernels (worst case over the state's instances)
    const size_t bpo = set->dist16 ? OpStore<uint16_t>::kBytesPerOp : OpStore<int32_t>::kBytesPerOp;
    {
        LdsSize g;
        g.take<int>(N + 1);
        g.take<uint16_t>(N + 2);
        g.take<uint16_t>(N + 2);
        g.take<int>(kMaxM);
        g.take<int>(kMaxM);
        g.take<unsigned char>(bpo * (2 * N + kAlnsStep));
        g.take<int>((size_t)kGainGroups * (N + 1));
        s->lds_gain = (int)g.bytes;
        LdsSize t;
        t.take<unsigned long long>(pow2_ge(N));
        t.take<int>(2 * N + kAlnsStep);
        t.take<int>(N + 1);
        t.take<uint16_t>(N + 2);
        t.take<uint16_t>(N + 2);
        t.take<unsigned char>(N + 1);
        t.take<int>(kMaxM);
        t.take<int>(kMaxM);
        t.take<int>(Q);
        t.take<int>(N + 1);
        t.take<unsigned char>(bpo * (2 * N + kAlnsStep));
        s->lds_destroy = (int)t.bytes;
        s->lds_enum = 2 * 8 * pow2_ge(2 * N + M + 1);
        LdsSize f;
        f.take<int>(2 * N + kAlnsStep);
        f.take<int>(2 * N + kAlnsStep);
        f.take<int>(N + 1);
        f.take<uint16_t>(N + 2);
        f.take<uint16_t>(N + 2);
        f.take<int>(kMaxM);
        f.take<int>(kMaxM);
        f.take<int>(kMaxM);
        f.take<int>(N + 1);
        f.take<unsigned char>(bpo * (2 * N + kAlnsStep));
        s->lds_feat = (int)f.bytes;
        LdsSize l;
        l.take<int>(2 * N + kAlnsStep);
        l.take<int>(N + 1);
        l.take<uint16_t>(N + 2);
        l.take<uint16_t>(N + 2);
        l.take<int>(kMaxM);
        l.take<int>(kMaxM);
        l.take<long long>(kMaxM);
        l.take<int>(N + 1);
        l.take<unsigned char>(N + 1);
        l.take<int>(kLsMaxCand);
        l.take<unsigned char>(bpo * (2 * N + kAlnsStep));
        s->lds_ls = (int)l.bytes;
    }
    if ((size_t)std::max(std::max(std::max(s->lds_gain, s->lds_feat), s->lds_ls),
                         std::max(s->lds_destroy, s->lds_enum)) > kLdsPerCu) {
        alns_state_destroy(s);
        return set_error(VRPRPD_EINVAL, "alns_state_create: n = %d needs too much LDS", N);
    }
    rc = s->dist16 ? set_attributes<uint16_t>(s) : set_attributes<int32_t>(s);
    if (rc != VRPRPD_OK) {
        alns_state_destroy(s);
        return rc;
    }
    *out = s;
    return VRPRPD_OK;
}

namespace vrprpd {

template <typename DT, int GL>
static const void* gains_kernel()
{
    return reinterpret_cast<const void*>(k_gains<DT, GL, kGainWaves>);
}

// Dynamic-LDS limits of the kernels of one iteration, set once per state
// (never during a graph capture).
template <typename DT>
static int set_attributes(alns_state* s)
{
    const void* ks[6] = {s->d.M <= 16 ? gains_kernel<DT, 16>() : (s->d.M <= 32 ? gains_kernel<DT, 32>()
                                                                                : gains_kernel<DT, 64>()),
                         reinterpret_cast<const void*>(k_destroy<DT>), reinterpret_cast<const void*>(k_enum<DT>),
                         reinterpret_cast<const void*>(k_features<DT>), reinterpret_cast<const void*>(k_ls_setup<DT>),
                         reinterpret_cast<const void*>(k_ls_enum<DT>)};
    const int lds[6] = {s->lds_gain, s->lds_destroy, s->lds_enum, s->lds_feat, s->lds_ls, s->lds_enum};
    for (int i = 0; i < 6; ++i)
        if (lds[i] > 64 * 1024) VRP_HIP(hipFuncSetAttribute(ks[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds[i]));
    return VRPRPD_OK;
}

template <typename DT, int GL>
static int launch_gains(alns_state* s, hipStream_t st)
{
    constexpr int WPB = kGainWaves;
    constexpr int per_block = 2 * kGainGroups;   // two sweeps per group
    const AlnsDev& d = s->d;
    hipLaunchKernelGGL((k_gains<DT, GL, WPB>), dim3(d.C, (d.N + per_block - 1) / per_block), dim3(64 * WPB),
                       s->lds_gain, st, d, per_block);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

// Up to three passes of one local search on every active chain.
template <typename DT>
static int launch_ls_passes(alns_state* s, hipStream_t st, int kind)
{
    AlnsDev& d = s->d;
    ScanArgs la{d.inst_tab, d.dist, d.proc, d.ls_base_inst, d.ls_base_off, d.ls_ops, d.ls_rt_off, d.ls_rt,
                d.ls_seg_off, d.ls_seg_base, d.ls_tuples, d.ls_tmk, d.ls_tst, d.ls_top3, d.ls_seg_cnt,
                d.C * d.LQ, s->set->num_inst, d.N, d.C * d.LQ, 8, 1};
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_ls_setup<DT>, dim3(d.C), dim3(256), s->lds_ls, st, d, kind);
        hipLaunchKernelGGL(k_ls_enum<DT>, dim3(d.C, d.LQ), dim3(256), s->lds_enum, st, d, kind);
        VRP_HIP(hipGetLastError());
        const int rc = insert_scan_launch(la, d.M, s->dist16, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_ls_apply, dim3(d.C), dim3(256), 0, st, d);
        VRP_HIP(hipGetLastError());
    }
    return VRPRPD_OK;
}

// One refinement round on every chain not yet stopped: repositioning, then
// relocation, then the stop flags.
template <typename DT>
static int launch_refine_round(alns_state* s, hipStream_t st)
{
    AlnsDev& d = s->d;
    for (int kind = 0; kind < 2; ++kind) {
        hipLaunchKernelGGL(k_ls_begin, dim3((d.C + 63) / 64), dim3(64), 0, st, d, kind == 0 ? 1 : 0, 1);
        const int rc = launch_ls_passes<DT>(s, st, kind);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_ls_finish, dim3(d.C), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_refine_round_end, dim3((d.C + 63) / 64), dim3(64), 0, st, d);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

// The launches of one iteration.  Nothing here depends on host-side state
// that changes between iterations (the iteration number lives on the
// device), so the sequence can be captured once and replayed.
template <typename DT>
static int launch_iteration(alns_state* s, hipStream_t st, int ls_mask)
{
    AlnsDev& d = s->d;
    hipLaunchKernelGGL(k_begin, dim3((d.C + 63) / 64), dim3(64), 0, st, d);
    VRP_HIP(hipGetLastError());
    int rc;
    if (d.M <= 16) rc = launch_gains<DT, 16>(s, st);
    else if (d.M <= 32) rc = launch_gains<DT, 32>(s, st);
    else rc = launch_gains<DT, 64>(s, st);
    if (rc) return rc;
    if (d.learn_on) {
        hipLaunchKernelGGL(k_features<DT>, dim3(d.C), dim3(256), s->lds_feat, st, d);
        VRP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_destroy<DT>, dim3(d.C, d.K), dim3(256), s->lds_destroy, st, d);
    VRP_HIP(hipGetLastError());
    const int use_scores = (s->mlp && d.K > 1) ? 1 : 0;
    if (use_scores) {
        rc = vrprpd_mlp_forward(s->mlp, (int64_t)d.C * d.N, d.feat, d.score, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_apply<DT>, dim3(d.C), dim3(256), d.N + 1, st, d, use_scores);
    VRP_HIP(hipGetLastError());
    ScanArgs sa{d.inst_tab, d.dist, d.proc, d.chain_inst, d.base_op_off, d.W_ops, d.base_rt_off, d.W_rt,
                d.seg_off, d.seg_base, d.tuples, d.tmk, d.tst, d.seg_top3, d.seg_cnt, d.C, s->set->num_inst, d.N,
                d.C * d.Q, std::max(1, (d.TPC + s->scan_tpb - 1) / s->scan_tpb), 1};
    for (int r = 0; r < d.Q; ++r) {
        // round r: at most Q - r customers still wait in any chain, so only
        // those slots get blocks
        const int active = d.Q - r;
        hipLaunchKernelGGL(k_enum<DT>, dim3(d.C, active), dim3(256), s->lds_enum, st, d);
        VRP_HIP(hipGetLastError());
        ScanArgs sr = sa;
        sr.num_seg = d.C * active;
        sr.seg_active = active;
        sr.seg_stride = d.Q;
        if ((rc = insert_scan_launch(sr, d.M, s->dist16, st))) return rc;
        hipLaunchKernelGGL(k_select, dim3(d.C), dim3(256), (size_t)16 * d.Q, st, d);
        VRP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_accept, dim3(d.C), dim3(256), 0, st, d);
    VRP_HIP(hipGetLastError());
    if (ls_mask) {
        bool first = true;
        for (int kind = 0; kind < 2; ++kind) {
            if (!(ls_mask & (1 << kind))) continue;
            hipLaunchKernelGGL(k_ls_begin, dim3((d.C + 63) / 64), dim3(64), 0, st, d, first ? 1 : 0, 0);
            first = false;
            if ((rc = launch_ls_passes<DT>(s, st, kind))) return rc;
        }
        hipLaunchKernelGGL(k_ls_finish, dim3(d.C), dim3(256), 0, st, d);
        VRP_HIP(hipGetLastError());
    }
    if (s->cpi > 1 && d.prm.import_interval > 0) {
        hipLaunchKernelGGL(k_import, dim3(s->n_inst), dim3(256), 0, st, d, s->cpi);
        VRP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, d);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

static int launch_iteration_any(alns_state* s, hipStream_t st, int ls_mask)
{
    return s->dist16 ? launch_iteration<uint16_t>(s, st, ls_mask) : launch_iteration<int32_t>(s, st, ls_mask);
}

// Local searches due after iteration `it` (0-based): bit 0 repositioning,
// bit 1 relocation.
static int ls_mask_of(const alns_state* s, int64_t it)
{
    const alns_params& P = s->d.prm;
    int mask = 0;
    if (P.ls_repos_interval > 0 && (it + 1) % P.ls_repos_interval == 0) mask |= 1;
    if (P.ls_reloc_interval > 0 && (it + 1) % P.ls_reloc_interval == 0) mask |= 2;
    return mask;
}

static void drop_graph(alns_state* s)
{
    for (int i = 0; i < 4; ++i) {
        if (s->gexec[i]) (void)hipGraphExecDestroy(s->gexec[i]);
        if (s->graph[i]) (void)hipGraphDestroy(s->graph[i]);
        s->gexec[i] = nullptr;
        s->graph[i] = nullptr;
    }
}

// Captures one iteration's launches (with the local searches of `mask`) on
// the state's own stream.
static int build_graph(alns_state* s, int mask)
{
    if (!s->cap) VRP_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    VRP_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    const int rc = launch_iteration_any(s, s->cap, mask);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_error(e, "alns_step: hipStreamEndCapture");
    s->graph[mask] = g;
    VRP_HIP(hipGraphInstantiate(&s->gexec[mask], g, nullptr, nullptr, 0));
    return VRPRPD_OK;
}

}  // namespace vrprpd

extern "C" int alns_step(alns_state* s, int32_t iterations, void* stream)
{
    using namespace vrprpd;
    if (!s || iterations < 0) return set_error(VRPRPD_EINVAL, "alns_step: bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < iterations; ++i) {
        const int mask = ls_mask_of(s, s->it);
        if (s->use_graph) {
            if (!s->gexec[mask]) {
                const int rc = build_graph(s, mask);
                if (rc) return rc;
            }
            VRP_HIP(hipGraphLaunch(s->gexec[mask], st));
        } else {
            const int rc = launch_iteration_any(s, st, mask);
            if (rc) return rc;
        }
        s->it += 1;
    }
    return VRPRPD_OK;
}

extern "C" int alns_refine(alns_state* s, int32_t max_rounds, int32_t* rounds_out, void* stream)
{
    using namespace vrprpd;
    if (!s || max_rounds < 0) return set_error(VRPRPD_EINVAL, "alns_refine: bad arguments");
    if (s->it != 0) return set_error(VRPRPD_EINVAL, "alns_refine: only before the first iteration");
    if (!s->d.ls_stop) return set_error(VRPRPD_EINVAL, "alns_refine: the state was created with ls_budget < 1");
    AlnsDev& d = s->d;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    VRP_HIP(hipMemsetAsync(d.ls_stop, 0, (size_t)d.C * sizeof(int32_t), st));
    std::vector<int32_t> stop(d.C);
    int rounds = 0;
    while (rounds < max_rounds) {
        const int rc = s->dist16 ? launch_refine_round<uint16_t>(s, st) : launch_refine_round<int32_t>(s, st);
        if (rc) return rc;
        ++rounds;
        VRP_HIP(hipMemcpyAsync(stop.data(), d.ls_stop, (size_t)d.C * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VRP_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int c = 0; c < d.C && all; ++c) all = stop[c] != 0;
        if (all) break;
    }
    hipLaunchKernelGGL(k_refine_temperature, dim3((d.C + 63) / 64), dim3(64), 0, st, d);
    VRP_HIP(hipGetLastError());
    if (rounds_out) *rounds_out = rounds;
    return VRPRPD_OK;
}

extern "C" int alns_set_graph(alns_state* s, int32_t enable)
{
    if (!s) return vrprpd::set_error(VRPRPD_EINVAL, "alns_set_graph: state is NULL");
    s->use_graph = enable != 0;
    vrprpd::drop_graph(s);
    return VRPRPD_OK;
}

extern "C" int alns_set_trace(alns_state* s, int64_t* trace, int64_t capacity)
{
    if (!s || (trace && capacity < 1)) return vrprpd::set_error(VRPRPD_EINVAL, "alns_set_trace: bad arguments");
    s->d.trace = trace;
    s->d.trace_cap = trace ? capacity : 0;
    s->d.trace_base = s->it;
    vrprpd::drop_graph(s);
    return VRPRPD_OK;
}

extern "C" int alns_get_best(const alns_state* s, int32_t chain, int32_t* mk, uint16_t* ops, uint16_t* rt_end,
                             void* stream)
{
    using namespace vrprpd;
    if (!s || chain < -1 || chain >= s->d.C || !mk) return set_error(VRPRPD_EINVAL, "alns_get_best: bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::vector<int32_t> zb(s->d.C);
    VRP_HIP(hipStreamSynchronize(st));
    VRP_HIP(hipMemcpy(zb.data(), s->d.zb, s->d.C * sizeof(int32_t), hipMemcpyDeviceToHost));
    int c = chain;
    if (c < 0) {
        c = 0;
        for (int x = 1; x < s->d.C; ++x)
            if (zb[x] < zb[c]) c = x;
    }
    *mk = zb[c];
    if (ops) VRP_HIP(hipMemcpyAsync(ops, s->d.B_ops + (size_t)c * 2 * s->d.N, 2 * s->d.N * sizeof(uint16_t),
                                    hipMemcpyDeviceToDevice, st));
    if (rt_end) VRP_HIP(hipMemcpyAsync(rt_end, s->d.B_rt + (size_t)c * s->d.M, s->d.M * sizeof(uint16_t),
                                       hipMemcpyDeviceToDevice, st));
    return VRPRPD_OK;
}

extern "C" int alns_get_state(const alns_state* s, int64_t* iterations, int64_t* evals, int32_t* z, int32_t* zb,
                              double* T, double* wD, double* wR)
{
    using namespace vrprpd;
    if (!s) return set_error(VRPRPD_EINVAL, "alns_get_state: state is NULL");
    VRP_HIP(hipDeviceSynchronize());
    const int C = s->d.C;
    if (iterations) *iterations = s->it;
    if (evals) VRP_HIP(hipMemcpy(evals, s->d.evals, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (z) VRP_HIP(hipMemcpy(z, s->d.z, C * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (zb) VRP_HIP(hipMemcpy(zb, s->d.zb, C * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (T) VRP_HIP(hipMemcpy(T, s->d.T, C * sizeof(double), hipMemcpyDeviceToHost));
    if (wD) VRP_HIP(hipMemcpy(wD, s->d.wD, (size_t)kND * C * sizeof(double), hipMemcpyDeviceToHost));
    if (wR) VRP_HIP(hipMemcpy(wR, s->d.wR, (size_t)kNR * C * sizeof(double), hipMemcpyDeviceToHost));
    return VRPRPD_OK;
}

// ---------------------------------------------------------------- learned proposal
static int ensure_features(alns_state* s, hipStream_t st)
{
    using namespace vrprpd;
    AlnsDev& d = s->d;
    if (d.feat) return VRPRPD_OK;
    int rc = VRPRPD_OK;
    if ((rc = alloc_n(s, &d.feat, (size_t)d.C * d.N * 64)) || (rc = alloc_n(s, &d.fstat, (size_t)d.C * (d.N + 1) * 2)) ||
        (rc = alloc_n(s, &d.dbar, d.C)) || (rc = alloc_n(s, &d.score, (size_t)d.C * d.N)))
        return rc;
    if (s->dist16)
        hipLaunchKernelGGL(k_static<uint16_t>, dim3(d.C), dim3(256), 0, st, d);
    else
        hipLaunchKernelGGL(k_static<int32_t>, dim3(d.C), dim3(256), 0, st, d);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int alns_set_learned(alns_state* s, vrprpd_mlp* mlp, int32_t K, double eps, void* stream)
{
    using namespace vrprpd;
    if (!s || K < 1 || K > 64 || !(eps >= 0.0 && eps <= 1.0))
        return set_error(VRPRPD_EINVAL, "alns_set_learned: need 1 <= K <= 64 and 0 <= eps <= 1");
    AlnsDev& d = s->d;
    if (mlp && mlp_max_rows(mlp) < (int64_t)d.C * d.N)
        return set_error(VRPRPD_EINVAL, "alns_set_learned: the network scores %lld rows at once, %d chains x n = %d "
                                        "need %lld", (long long)mlp_max_rows(mlp), d.C, d.N, (long long)d.C * d.N);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!mlp) K = 1;
    if (K > s->cand_cap) {
        int rc;
        if ((rc = alloc_n(s, &d.cand_rem, (size_t)d.C * K * d.Q)) || (rc = alloc_n(s, &d.cand_cnt, (size_t)d.C * K)))
            return rc;
        s->cand_cap = K;
    }
    if (mlp) {
        const int rc = ensure_features(s, st);
        if (rc) return rc;
    }
    s->mlp = mlp;
    d.K = K;
    d.eps = eps;
    d.learn_on = (mlp != nullptr || d.rec_x != nullptr) ? 1 : 0;
    drop_graph(s);
    return VRPRPD_OK;
}

extern "C" int alns_record(alns_state* s, int64_t capacity, void* stream)
{
    using namespace vrprpd;
    if (!s || capacity < 0) return set_error(VRPRPD_EINVAL, "alns_record: bad arguments");
    AlnsDev& d = s->d;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    VRP_HIP(hipStreamSynchronize(st));
    for (void* p : s->rec_allocs) (void)hipFree(p);
    s->rec_allocs.clear();
    d.rec_x = nullptr;
    d.rec_t = nullptr;
    d.rec_n = nullptr;
    d.rec_cap = 0;
    if (capacity > 0) {
        int rc = ensure_features(s, st);
        if (rc) return rc;
        const size_t bytes[3] = {(size_t)capacity * d.Q * 64 * sizeof(uint16_t), (size_t)capacity * sizeof(float),
                                 (size_t)capacity * sizeof(int32_t)};
        void* p[3] = {nullptr, nullptr, nullptr};
        for (int i = 0; i < 3; ++i) {
            hipError_t e = hipMalloc(&p[i], bytes[i]);
            if (e != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipFree(p[j]);
                return set_error(VRPRPD_ENOMEM, "alns_record: %lld sets do not fit (%s)", (long long)capacity,
                                 hipGetErrorString(e));
            }
            s->rec_allocs.push_back(p[i]);
        }
        d.rec_x = static_cast<uint16_t*>(p[0]);
        d.rec_t = static_cast<float*>(p[1]);
        d.rec_n = static_cast<int32_t*>(p[2]);
        d.rec_cap = capacity;
        d.rec_base = s->it;
    }
    d.learn_on = (s->mlp != nullptr || d.rec_x != nullptr) ? 1 : 0;
    drop_graph(s);
    return VRPRPD_OK;
}

static int64_t record_count(const alns_state* s)
{
    if (!s->d.rec_x) return 0;
    const int64_t done = (s->it - s->d.rec_base) * s->d.C;
    return done < s->d.rec_cap ? done : s->d.rec_cap;
}

extern "C" int alns_record_info(const alns_state* s, int64_t* sets, int32_t* q_max)
{
    if (!s) return vrprpd::set_error(VRPRPD_EINVAL, "alns_record_info: state is NULL");
    if (sets) *sets = record_count(s);
    if (q_max) *q_max = s->d.Q;
    return VRPRPD_OK;
}

extern "C" int alns_record_batch(const alns_state* s, int32_t num_sets, uint64_t seed, uint16_t* x, int64_t* seg_off,
                                 float* target, void* stream)
{
    using namespace vrprpd;
    if (!s || num_sets < 1 || !x || !seg_off || !target)
        return set_error(VRPRPD_EINVAL, "alns_record_batch: bad arguments");
    const int64_t count = record_count(s);
    if (count < 1) return set_error(VRPRPD_EINVAL, "alns_record_batch: nothing recorded yet");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_batch_index, dim3(1), dim3(1024), 0, st, s->d, num_sets, seed, count, seg_off, target);
    hipLaunchKernelGGL(k_batch_rows, dim3(num_sets), dim3(256), 0, st, s->d, seed, count, seg_off, x);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int alns_get_learned(const alns_state* s, uint16_t* feat, int32_t* cand_rem, int32_t* cand_cnt,
                                int32_t* chosen, void* stream)
{
    using namespace vrprpd;
    if (!s) return set_error(VRPRPD_EINVAL, "alns_get_learned: state is NULL");
    const AlnsDev& d = s->d;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (feat) {
        if (!d.feat) return set_error(VRPRPD_EINVAL, "alns_get_learned: features are off");
        VRP_HIP(hipMemcpyAsync(feat, d.feat, (size_t)d.C * d.N * 64 * 2, hipMemcpyDeviceToDevice, st));
    }
    if (cand_rem)
        VRP_HIP(hipMemcpyAsync(cand_rem, d.cand_rem, (size_t)d.C * d.K * d.Q * 4, hipMemcpyDeviceToDevice, st));
    if (cand_cnt) VRP_HIP(hipMemcpyAsync(cand_cnt, d.cand_cnt, (size_t)d.C * d.K * 4, hipMemcpyDeviceToDevice, st));
    if (chosen) VRP_HIP(hipMemcpyAsync(chosen, d.chosen, (size_t)d.C * 4, hipMemcpyDeviceToDevice, st));
    return VRPRPD_OK;
}

// ---------------------------------------------------------------- checkpoint
namespace vrprpd {

struct AlnsCkptHead {
    char magic[8];           // "VRPALNS1"
    int32_t C, N, M, Q, TPC, n_inst, cpi, dist16;
    uint64_t seed;
    int64_t it;
    alns_params prm;
};

static bool same_params(const alns_params& a, const alns_params& b)
{
    return a.T0 == b.T0 && a.alpha == b.alpha && a.reheat == b.reheat && a.gate == b.gate &&
           a.stag_limit == b.stag_limit && a.tau == b.tau && a.r == b.r && a.sigma1 == b.sigma1 &&
           a.sigma2 == b.sigma2 && a.sigma3 == b.sigma3 && a.w_min == b.w_min && a.q_min == b.q_min &&
           a.q_max == b.q_max && a.tuple_budget == b.tuple_budget && a.import_interval == b.import_interval &&
           a.op_mask == b.op_mask && a.ls_repos_interval == b.ls_repos_interval &&
           a.ls_reloc_interval == b.ls_reloc_interval && a.ls_budget == b.ls_budget && a.chain_base == b.chain_base;
}

// Everything an iteration reads from the previous one: both solutions of
// every chain, makespans, temperatures, operator weights, the scores and
// attempts of the running period, stagnation, the evaluation count and the
// device iteration counter; then the chains' instance ids.
static std::vector<DevField> alns_fields(const alns_state* s)
{
    const AlnsDev& d = s->d;
    const size_t C = (size_t)d.C;
    return {{d.S_ops, C * 2 * d.N * 2}, {d.S_rt, C * d.M * 2}, {d.B_ops, C * 2 * d.N * 2}, {d.B_rt, C * d.M * 2},
            {d.z, C * 4}, {d.zb, C * 4}, {d.T, C * 8}, {d.T_init, C * 8}, {d.wD, kND * C * 8},
            {d.wR, kNR * C * 8}, {d.sD, kND * C * 8}, {d.sR, kNR * C * 8}, {d.aD, kND * C * 4},
            {d.aR, kNR * C * 4}, {d.stag, C * 4}, {d.evals, 8}, {d.it_dev, 4}};
}

static AlnsCkptHead alns_head(const alns_state* s)
{
    AlnsCkptHead h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "VRPALNS1", 8);
    h.C = s->d.C;
    h.N = s->d.N;
    h.M = s->d.M;
    h.Q = s->d.Q;
    h.TPC = s->d.TPC;
    h.n_inst = s->n_inst;
    h.cpi = s->cpi;
    h.dist16 = s->dist16;
    h.seed = s->d.seed;
    h.it = s->it;
    h.prm = s->d.prm;
    return h;
}

}  // namespace vrprpd

extern "C" int alns_state_save(const alns_state* s, void* buf, int64_t capacity, int64_t* bytes, void* stream)
{
    using namespace vrprpd;
    if (!s || (!buf && !bytes)) return set_error(VRPRPD_EINVAL, "alns_state_save: bad arguments");
    std::vector<unsigned char> head(sizeof(AlnsCkptHead) + s->inst_ids.size() * sizeof(int32_t));
    const AlnsCkptHead h = alns_head(s);
    std::memcpy(head.data(), &h, sizeof h);
    std::memcpy(head.data() + sizeof h, s->inst_ids.data(), s->inst_ids.size() * sizeof(int32_t));
    return ckpt_save(head.data(), head.size(), alns_fields(s), buf, capacity, bytes,
                     reinterpret_cast<hipStream_t>(stream), "alns_state_save");
}

extern "C" int alns_state_load(alns_state* s, const void* buf, int64_t bytes, void* stream)
{
    using namespace vrprpd;
    if (!s || !buf || bytes < (int64_t)sizeof(AlnsCkptHead))
        return set_error(VRPRPD_EINVAL, "alns_state_load: bad arguments");
    AlnsCkptHead h;
    std::memcpy(&h, buf, sizeof h);
    const AlnsCkptHead mine = alns_head(s);
    if (std::memcmp(h.magic, "VRPALNS1", 8) != 0)
        return set_error(VRPRPD_EINVAL, "alns_state_load: not an ALNS checkpoint");
    if (h.C != mine.C || h.N != mine.N || h.M != mine.M || h.Q != mine.Q || h.TPC != mine.TPC ||
        h.n_inst != mine.n_inst || h.cpi != mine.cpi || h.dist16 != mine.dist16 || h.seed != mine.seed ||
        !same_params(h.prm, mine.prm))
        return set_error(VRPRPD_EINVAL, "alns_state_load: the checkpoint was taken from a state with other "
                                        "instances, chains, seed or parameters");
    const size_t ids_bytes = s->inst_ids.size() * sizeof(int32_t);
    if (bytes < (int64_t)(sizeof h + ids_bytes) ||
        std::memcmp(static_cast<const unsigned char*>(buf) + sizeof h, s->inst_ids.data(), ids_bytes) != 0)
        return set_error(VRPRPD_EINVAL, "alns_state_load: the checkpoint's chains belong to other instances");
    const int rc = ckpt_load(buf, bytes, sizeof h + ids_bytes, alns_fields(s), reinterpret_cast<hipStream_t>(stream),
                             "alns_state_load");
    if (rc) return rc;
    s->it = h.it;
    return VRPRPD_OK;
}

extern "C" int alns_autotune(alns_state* s, int32_t iterations, int32_t* tpb_out, float* ms_out, void* stream)
{
    using namespace vrprpd;
    if (!s || iterations < 1) return set_error(VRPRPD_EINVAL, "alns_autotune: need a state and iterations >= 1");
    if (s->d.rec_x) return set_error(VRPRPD_EINVAL, "alns_autotune: not while recording");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int64_t bytes = 0;
    int rc = alns_state_save(s, nullptr, 0, &bytes, stream);
    if (rc) return rc;
    std::vector<unsigned char> saved((size_t)bytes), ref, cur((size_t)bytes);
    if ((rc = alns_state_save(s, saved.data(), bytes, &bytes, stream))) return rc;
    // the trace, if any, is not written while shapes are tried
    int64_t* trace = s->d.trace;
    const int64_t trace_cap = s->d.trace_cap, trace_base = s->d.trace_base;
    s->d.trace = nullptr;
    s->d.trace_cap = 0;
    const int keep = s->scan_tpb;
    const int opts[4] = {8, 16, 32, 64};
    int best = keep;
    float best_ms = 0.f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto finish = [&](int code) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        drop_graph(s);
        s->d.trace = trace;
        s->d.trace_cap = trace_cap;
        s->d.trace_base = trace_base;
        const int lr = alns_state_load(s, saved.data(), (int64_t)saved.size(), stream);
        return code ? code : lr;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        s->scan_tpb = keep;
        return finish(set_error(VRPRPD_EHIP, "alns_autotune: hipEventCreate"));
    }
    for (int i = 0; i < 4; ++i) {
        s->scan_tpb = opts[i];
        drop_graph(s);
        float ms = 0.f;
        if ((rc = alns_state_load(s, saved.data(), (int64_t)saved.size(), stream)) ||
            (rc = alns_step(s, 1, stream)))   // warm-up: captures the graph
            break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = set_error(VRPRPD_EHIP, "alns_autotune: event"); break; }
        if ((rc = alns_step(s, iterations, stream))) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = set_error(VRPRPD_EHIP, "alns_autotune: timing failed");
            break;
        }
        if ((rc = alns_state_save(s, cur.data(), bytes, &bytes, stream))) break;
        if (i == 0) {
            ref = cur;
        } else if (cur != ref) {
            rc = set_error(VRPRPD_EHIP, "alns_autotune: %d tuples per workgroup change the search's state", opts[i]);
            break;
        }
        ms /= (float)iterations;
        if (ms_out) ms_out[i] = ms;
        if (i == 0 || ms < best_ms) {
            best_ms = ms;
            best = opts[i];
        }
    }
    s->scan_tpb = rc ? keep : best;
    if (!rc) {
        s->set->alns_scan_tuned[std::make_tuple(s->d.N, s->d.M, (int)s->d.prm.tuple_budget)] = best;
        if (tpb_out) *tpb_out = best;
    }
    return finish(rc);
}
