// Construction heuristics: the initial solution of Section 4.2 ("Initial
// Solution Construction": sweep clustering by a pseudo-angle taken from the
// distance matrix, sector balancing by the workload estimate 2 d(0,c) + p_c,
// a nearest-neighbour route per vehicle) and the three BRKGA warm-start
// seeds of Section 4.4.4 (nearest neighbour, load balanced, shortest
// processing time).  Readings of the phases are stated with vrprpd_construct
// in the public header.
//
// One block per instance.  The steps are sequential by nature (each greedy
// choice depends on the previous one); the block parallelises what one step
// scans: customers for the angle keys and the balancing move, (vehicle, op)
// pairs for the dispatch rules, and one wave per vehicle for the
// per-vehicle routes, which are independent.  Per-instance arrays live in a
// global workspace private to the block (L2-resident at these sizes).
#include <hip/hip_runtime.h>

#include "common.h"
#include "vrprpd.h"

namespace vrprpd {
namespace {

constexpr int kCT = 256;          // threads per block
constexpr int kCW = kCT / 64;     // waves per block
constexpr unsigned long long kNone = ~0ull;

struct ConsArgs {
    const InstDev* tab;
    int num_inst;
    const void* dist;
    const int32_t* proc;
    const int32_t* inst;          // [B] or null (block b builds instance b)
    int heuristic, N, M;          // N, M: n_max, m_max
    int64_t op_stride, rt_stride;
    uint16_t* ops;
    uint16_t* rt_end;
    unsigned char* ws;
    int64_t ws_stride;
};

// Per-block workspace carve (sizes from n_max).
struct Ws {
    unsigned long long* key;      // [pow2 >= N] sort keys
    int32_t* aux;                 // [N + 1] sector of a customer / slot in the pending list
    int32_t* ready;               // [N + 1] drop time + p
    int32_t* clist;               // [N] customers grouped by vehicle / pending pickups
    uint32_t* seq;                // [2N] placement order, vehicle << 16 | op
    unsigned char* state;         // [N + 1] 0 waiting, 1 dropped, 2 picked
};

__host__ __device__ inline int64_t ws_bytes(int N)
{
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    return up(8 * (int64_t)pow2_ge(N)) + 3 * up(4 * ((int64_t)N + 1)) + up(8 * (int64_t)N) + up((int64_t)N + 1);
}

__device__ inline Ws carve(unsigned char* p, int N)
{
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    Ws w;
    w.key = reinterpret_cast<unsigned long long*>(p);
    p += up(8 * (int64_t)pow2_ge(N));
    w.aux = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)N + 1));
    w.ready = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)N + 1));
    w.clist = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)N + 1));
    w.seq = reinterpret_cast<uint32_t*>(p);
    p += up(8 * (int64_t)N);
    w.state = p;
    return w;
}

__device__ inline unsigned long long wave_min_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Minimum over the block; every thread gets it.  red: LDS [kCW].
__device__ inline unsigned long long block_min_u64(unsigned long long x, unsigned long long* red)
{
    x = wave_min_u64(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long r = red[0];
    for (int w = 1; w < kCW; ++w) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

__device__ inline unsigned long long umin(unsigned long long a, unsigned long long b) { return a < b ? a : b; }

// Signed 64-bit order as unsigned order.
__device__ inline unsigned long long biased(long long v) { return (unsigned long long)v ^ (1ull << 63); }

__device__ inline int vehicles_used(const InstDev& I)
{
    if (I.load_model == VRPRPD_FULL_START) return I.m;
    const int mv = I.m < I.R ? I.m : I.R;
    return mv < 1 ? 1 : mv;
}

__device__ inline int cap_of(const InstDev& I, int mv, int v)
{
    if (I.load_model == VRPRPD_FULL_START) return I.k;
    const int share = I.R / mv + (v < I.R % mv);
    return share < I.k ? share : I.k;
}

template <typename DT>
struct Dist {
    const DT* D;
    int N1;
    __device__ int operator()(int a, int b) const { return (int)D[(int64_t)a * N1 + b]; }
};

// Phase 1: customers in pseudo-angle order (as keys[0, n) with the customer
// in the low 15 bits), then the cut into mv contiguous sectors (ws.aux).
template <typename DT>
__device__ void angle_sectors(const InstDev& I, const Dist<DT>& d, const Ws& ws, int mv, unsigned long long* red)
{
    const int n = I.n, s = I.ashift;
    __shared__ long long sh_b, sh_X2, sh_a2, sh_h;
    __shared__ int sh_r, sh_r2;
    // r: farthest from the depot, lowest index on ties
    unsigned long long x = kNone;
    for (int c = threadIdx.x + 1; c <= n; c += kCT)
        x = umin(x, ((unsigned long long)(0xFFFFFFFFu - (uint32_t)(d(0, c) >> s)) << 16) | (unsigned)c);
    x = block_min_u64(x, red);
    if (threadIdx.x == 0) {
        sh_r = (int)(x & 0xFFFF);
        sh_b = (long long)(d(0, sh_r) >> s);
    }
    __syncthreads();
    const int r = sh_r;
    const long long b = sh_b;
    auto Xof = [&](int c) {
        const long long a = d(0, c) >> s, e = d(r, c) >> s;
        return a * a + b * b - e * e;
    };
    // r2: farthest from the axis (largest 4 a^2 b^2 - X^2), lowest index on ties
    x = kNone;
    for (int c = threadIdx.x + 1; c <= n; c += kCT) {
        const long long a = d(0, c) >> s, X = Xof(c);
        x = umin(x, biased(-(4 * a * a * b * b - X * X)));
    }
    x = block_min_u64(x, red);
    const long long hbest = -(long long)(x ^ (1ull << 63));
    x = kNone;
    for (int c = threadIdx.x + 1; c <= n; c += kCT) {
        const long long a = d(0, c) >> s, X = Xof(c);
        if (4 * a * a * b * b - X * X == hbest) x = umin(x, (unsigned long long)c);
    }
    x = block_min_u64(x, red);
    if (threadIdx.x == 0) {
        sh_r2 = (int)x;
        sh_a2 = d(0, sh_r2) >> s;
        sh_X2 = Xof(sh_r2);
        sh_h = hbest;
    }
    __syncthreads();
    const int r2 = sh_r2;
    const long long a2 = sh_a2, X2 = sh_X2;
    const long long one = 1ll << 30;
    for (int c = threadIdx.x + 1; c <= n; c += kCT) {
        const long long a = d(0, c) >> s, e2 = d(r2, c) >> s, X = Xof(c);
        int side = 0;
        if (sh_h > 0) {
            const long long t = 2 * b * b * (a * a + a2 * a2 - e2 * e2) - X * X2;
            side = t > 0 ? 1 : (t < 0 ? -1 : 0);
        }
        long long q;
        if (a == 0 || b == 0) {
            q = one;
        } else {
            q = X * one / (2 * a * b);
            q = q > one ? one : (q < -one ? -one : q);
        }
        const int half = side < 0 || (side == 0 && X < 0);
        const unsigned long long u = half ? (unsigned long long)(q + one) : (unsigned long long)(one - q);
        ws.key[c - 1] = ((unsigned long long)half << 47) | (u << 15) | (unsigned long long)c;
    }
    const int np = pow2_ge(n);
    for (int i = n + threadIdx.x; i < np; i += kCT) ws.key[i] = kNone;
    __syncthreads();
    block_sort_u64(ws.key, np);
    const int base = n / mv, extra = n % mv;
    for (int i = threadIdx.x; i < n; i += kCT) {
        const int c = (int)(ws.key[i] & 0x7FFF);
        const int v = i < extra * (base + 1) ? i / (base + 1) : extra + (i - extra * (base + 1)) / base;
        ws.aux[c] = v;
    }
    __syncthreads();
}

// Phase 2: moves from the heaviest to the lightest sector while they differ
// by 10% of the heaviest or more.
template <typename DT>
__device__ void balance(const InstDev& I, const Dist<DT>& d, const int32_t* P, const Ws& ws, int mv,
                        unsigned long long* red)
{
    const int n = I.n;
    __shared__ long long W[kMaxM];
    __shared__ int sh_hi, sh_lo, sh_go;
    __shared__ long long sh_gap;
    if (threadIdx.x < kMaxM) W[threadIdx.x] = 0;
    __syncthreads();
    for (int c = threadIdx.x + 1; c <= n; c += kCT)
        atomicAdd(reinterpret_cast<unsigned long long*>(&W[ws.aux[c]]), (unsigned long long)(2ll * d(0, c) + P[c]));
    __syncthreads();
    // Every move lowers the sum of squared workloads by 2 w (gap - w) > 0
    // (0 < w < gap), so the loop ends without a move limit.
    for (;;) {
        if (threadIdx.x == 0) {
            int hi = 0, lo = 0;
            for (int v = 1; v < mv; ++v) {
                if (W[v] > W[hi]) hi = v;
                if (W[v] < W[lo]) lo = v;
            }
            sh_hi = hi;
            sh_lo = lo;
            sh_gap = W[hi] - W[lo];
            sh_go = !(10 * sh_gap < W[hi]);
        }
        __syncthreads();
        if (!sh_go) break;
        const int hi = sh_hi;
        const long long gap = sh_gap;
        unsigned long long x = kNone;
        for (int c = threadIdx.x + 1; c <= n; c += kCT) {
            if (ws.aux[c] != hi) continue;
            const long long w = 2ll * d(0, c) + P[c];
            if (w <= 0 || w >= gap) continue;
            const long long dev = gap - 2 * w >= 0 ? gap - 2 * w : 2 * w - gap;
            x = umin(x, ((unsigned long long)dev << 15) | (unsigned)c);
        }
        x = block_min_u64(x, red);
        if (x == kNone) break;
        if (threadIdx.x == 0) {
            const int c = (int)(x & 0x7FFF);
            const long long w = 2ll * d(0, c) + P[c];
            ws.aux[c] = sh_lo;
            W[hi] -= w;
            W[sh_lo] += w;
        }
        __syncthreads();
    }
    __syncthreads();
}

// LB: whole customers, heaviest workload first, each to the vehicle of least
// workload so far (one wave, lanes = vehicles).
template <typename DT>
__device__ void lb_sectors(const InstDev& I, const Dist<DT>& d, const int32_t* P, const Ws& ws, int mv)
{
    const int n = I.n;
    const long long WMAX = 1ll << 34;
    for (int c = threadIdx.x + 1; c <= n; c += kCT)
        ws.key[c - 1] = ((unsigned long long)(WMAX - (2ll * d(0, c) + P[c])) << 15) | (unsigned)c;
    const int np = pow2_ge(n);
    for (int i = n + threadIdx.x; i < np; i += kCT) ws.key[i] = kNone;
    __syncthreads();
    block_sort_u64(ws.key, np);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        unsigned long long W = 0;
        for (int i = 0; i < n; ++i) {
            const int c = (int)(ws.key[i] & 0x7FFF);
            const unsigned long long k = lane < mv ? (W << 6) | (unsigned)lane : kNone;
            const unsigned long long best = wave_min_u64(k);
            if (lane == (int)(best & 63)) {
                W += (unsigned long long)(2ll * d(0, c) + P[c]);
                ws.aux[c] = lane;
            }
        }
    }
    __syncthreads();
}

// Phase 3 (and LB's routes): each vehicle serves its sector alone; one wave
// per vehicle, each step the op of earliest completion (ties by op).
template <typename DT>
__device__ void own_routes(const InstDev& I, const Dist<DT>& d, const int32_t* P, const Ws& ws, int mv,
                           uint16_t* ops, uint16_t* rt)
{
    const int n = I.n, m = I.m;
    __shared__ int cnt[kMaxM + 1], start[kMaxM + 1], placed[kMaxM];
    if (threadIdx.x <= kMaxM) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int c = threadIdx.x + 1; c <= n; c += kCT) {
        atomicAdd(&cnt[ws.aux[c]], 1);
        ws.state[c] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        start[0] = 0;
        for (int v = 0; v < m; ++v) start[v + 1] = start[v] + cnt[v];
        for (int v = 0; v < m; ++v) cnt[v] = start[v];       // fill cursors
    }
    __syncthreads();
    for (int c = threadIdx.x + 1; c <= n; c += kCT) ws.clist[atomicAdd(&cnt[ws.aux[c]], 1)] = c;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int v = threadIdx.x >> 6; v < m; v += kCW) {
        const int s0 = start[v], len = start[v + 1] - s0;
        const int cap = v < mv ? cap_of(I, mv, v) : 0;
        long long t = 0;
        int loc = 0, out = 0, step = 0;
        for (; step < 2 * len; ++step) {
            unsigned long long best = kNone;
            for (int j = lane; j < len; j += 64) {
                const int c = ws.clist[s0 + j];
                const int st = ws.state[c];
                if (st == 2) continue;
                const long long arr = t + d(loc, c);
                unsigned long long k;
                if (st == 0) {
                    if (out >= cap) continue;
                    k = ((unsigned long long)arr << 16) | (unsigned)(2 * (c - 1));
                } else {
                    const long long rd = ws.ready[c];
                    k = ((unsigned long long)(arr > rd ? arr : rd) << 16) | (unsigned)(2 * (c - 1) + 1);
                }
                best = k < best ? k : best;
            }
            const unsigned long long g = wave_min_u64(best);
            if (g == kNone) break;
            const int o = (int)(g & 0xFFFF), c = o / 2 + 1;
            t = (long long)(g >> 16);
            loc = c;
            if (best == g) {            // the lane that scanned c owns its entries
                if (o & 1) {
                    ws.state[c] = 2;
                } else {
                    ws.state[c] = 1;
                    ws.ready[c] = (int32_t)(t + P[c]);
                }
            }
            out += (o & 1) ? -1 : 1;
            if (lane == 0) ops[2 * s0 + step] = (uint16_t)((c << 1) | (o & 1));
        }
        if (lane == 0) placed[v] = step;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // A vehicle stops short only when it may carry nothing (R = 0 under
        // MIN_PRELOAD), and then it placed nothing; later routes move down.
        int pos = 0;
        for (int v = 0; v < m; ++v) {
            const int s0 = 2 * start[v];
            if (pos != s0)
                for (int j = 0; j < placed[v]; ++j) ops[pos + j] = ops[s0 + j];
            pos += placed[v];
            rt[v] = (uint16_t)pos;
        }
    }
}

// NN and SPT: one dispatch loop over all vehicles with the decoder's load
// rules; placement order goes to ws.seq, routes are written at the end.
template <typename DT>
__device__ void dispatch(const InstDev& I, const Dist<DT>& d, const int32_t* P, const Ws& ws, int rule,
                         uint16_t* ops, uint16_t* rt, unsigned long long* red)
{
    const int n = I.n, m = I.m, k = I.k, full = I.load_model == VRPRPD_FULL_START;
    __shared__ long long t[kMaxM];
    __shared__ int loc[kMaxM], q[kMaxM], M[kMaxM];
    __shared__ int Lsum, undropped, npend, spt_next, sh_v, sh_nxt, placed;
    if (threadIdx.x < m) {
        t[threadIdx.x] = 0;
        loc[threadIdx.x] = 0;
        q[threadIdx.x] = full ? k : 0;
        M[threadIdx.x] = full ? k : 0;
    }
    if (threadIdx.x == 0) {
        Lsum = 0;
        undropped = n;
        npend = 0;
        spt_next = 0;
        placed = 0;
    }
    for (int c = threadIdx.x + 1; c <= n; c += kCT) ws.state[c] = 0;
    if (rule == VRPRPD_CONS_SPT) {
        for (int c = threadIdx.x + 1; c <= n; c += kCT) ws.key[c - 1] = ((unsigned long long)P[c] << 15) | (unsigned)c;
        const int np = pow2_ge(n);
        for (int i = n + threadIdx.x; i < np; i += kCT) ws.key[i] = kNone;
        __syncthreads();
        block_sort_u64(ws.key, np);
    }
    __syncthreads();
    for (int step = 0; step < 2 * n; ++step) {
        if (threadIdx.x == 0) {
            if (rule == VRPRPD_CONS_NN) {
                int bv = -1;
                for (int v = 0; v < m; ++v) {
                    const int canD = q[v] > 0 || (!full && M[v] < k && Lsum < I.R);
                    const int canP = q[v] < k;
                    if (!((canD && undropped > 0) || (canP && npend > 0))) continue;
                    if (bv < 0 || t[v] < t[bv]) bv = v;
                }
                sh_v = bv;
            } else {
                while (spt_next < n && ws.state[ws.key[spt_next] & 0x7FFF] != 0) ++spt_next;
                sh_nxt = spt_next < n ? (int)(ws.key[spt_next] & 0x7FFF) : 0;
            }
        }
        __syncthreads();
        unsigned long long x = kNone;
        if (rule == VRPRPD_CONS_NN) {
            const int v = sh_v;
            if (v < 0) break;
            const int canD = q[v] > 0 || (!full && M[v] < k && Lsum < I.R);
            const int canP = q[v] < k;
            for (int c = threadIdx.x + 1; c <= n; c += kCT) {
                const int st = ws.state[c];
                if (st == 2 || (st == 1 && !canP) || (st == 0 && !canD)) continue;
                x = umin(x, ((unsigned long long)d(loc[v], c) << 16) | (unsigned)(2 * (c - 1) + st));
            }
            x = block_min_u64(x, red);
            if (x != kNone) x = (x & 0xFFFF) << 6 | (unsigned)v;      // op << 6 | vehicle
        } else {
            const int nxt = sh_nxt, np = npend;
            const int pairs = (1 + np) * m;
            for (int e = threadIdx.x; e < pairs; e += kCT) {
                const int i = e / m, v = e - i * m;
                int c, isP;
                if (i == 0) {
                    if (!nxt || !(q[v] > 0 || (!full && M[v] < k && Lsum < I.R))) continue;
                    c = nxt;
                    isP = 0;
                } else {
                    if (!(q[v] < k)) continue;
                    c = ws.clist[i - 1];
                    isP = 1;
                }
                const long long arr = t[v] + d(loc[v], c);
                const long long rd = isP ? (long long)ws.ready[c] : arr;
                const long long comp = arr > rd ? arr : rd;
                x = umin(x, ((unsigned long long)comp << 22) | ((unsigned)(2 * (c - 1) + isP) << 6) | (unsigned)v);
            }
            x = block_min_u64(x, red);
            if (x != kNone) x &= (1ull << 22) - 1;                 // op << 6 | vehicle
        }
        if (x == kNone) break;
        if (threadIdx.x == 0) {
            const int v = (int)(x & 63), o = (int)(x >> 6), c = o / 2 + 1;
            const long long arr = t[v] + d(loc[v], c);
            if (o & 1) {
                const long long rd = ws.ready[c];
                t[v] = arr > rd ? arr : rd;
                ws.state[c] = 2;
                ++q[v];
                if (q[v] > M[v]) M[v] = q[v];
                const int at = ws.aux[c], last = ws.clist[npend - 1];   // swap-remove from the pending list
                ws.clist[at] = last;
                ws.aux[last] = at;
                --npend;
            } else {
                t[v] = arr;
                if (q[v] == 0) {
                    ++M[v];
                    ++Lsum;
                    ++q[v];
                }
                --q[v];
                ws.state[c] = 1;
                ws.ready[c] = (int32_t)(arr + P[c]);
                --undropped;
                ws.clist[npend] = c;
                ws.aux[c] = npend;
                ++npend;
            }
            loc[v] = c;
            ws.seq[placed++] = ((uint32_t)v << 16) | (uint32_t)o;
        }
        __syncthreads();
    }
    __syncthreads();
    // routes: vehicle v's placements in order (lanes = vehicles)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x, L = placed;
        int mine = 0;
        for (int i = 0; i < L; ++i) mine += (int)(ws.seq[i] >> 16) == lane;
        int incl = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        int pos = incl - mine;
        if (lane < m) {
            for (int i = 0; i < L; ++i) {
                const uint32_t e = ws.seq[i];
                if ((int)(e >> 16) != lane) continue;
                const int o = (int)(e & 0xFFFF);
                ops[pos++] = (uint16_t)(((o / 2 + 1) << 1) | (o & 1));
            }
            rt[lane] = (uint16_t)incl;
        }
    }
}

template <typename DT>
__global__ __launch_bounds__(kCT) void k_construct(ConsArgs a)
{
    __shared__ unsigned long long red[kCW];
    const int b = blockIdx.x;
    const int i = a.inst ? a.inst[b] : b;
    uint16_t* ops = a.ops + (int64_t)b * a.op_stride;
    uint16_t* rt = a.rt_end + (int64_t)b * a.rt_stride;
    if (i < 0 || i >= a.num_inst) {         // no such instance: an empty solution
        for (int v = threadIdx.x; v < a.M; v += kCT) rt[v] = 0;
        return;
    }
    const InstDev I = a.tab[i];
    const Dist<DT> d{reinterpret_cast<const DT*>(a.dist) + I.d_off, I.n + 1};
    const int32_t* P = a.proc + I.p_off;
    const Ws ws = carve(a.ws + (int64_t)b * a.ws_stride, a.N);
    const int mv = vehicles_used(I);
    if (a.heuristic == VRPRPD_CONS_SWEEP || a.heuristic == VRPRPD_CONS_LB) {
        if (a.heuristic == VRPRPD_CONS_SWEEP) {
            angle_sectors(I, d, ws, mv, red);
            balance(I, d, P, ws, mv, red);
        } else {
            lb_sectors(I, d, P, ws, mv);
        }
        own_routes(I, d, P, ws, mv, ops, rt);
    } else {
        dispatch(I, d, P, ws, a.heuristic, ops, rt, red);
    }
}

}  // namespace
}  // namespace vrprpd

extern "C" int vrprpd_construct(const vrprpd_set* set, int32_t B, const int32_t* inst, int32_t heuristic,
                                int64_t op_stride, uint16_t* ops, int64_t rt_stride, uint16_t* rt_end, void* stream)
{
    using namespace vrprpd;
    if (!set || B < 0 || heuristic < VRPRPD_CONS_SWEEP || heuristic > VRPRPD_CONS_SPT || (B > 0 && (!ops || !rt_end)))
        return set_error(VRPRPD_EINVAL, "vrprpd_construct: bad arguments");
    if (op_stride < 2 * (int64_t)set->n_max || rt_stride < set->m_max)
        return set_error(VRPRPD_EINVAL, "vrprpd_construct: op_stride must be >= 2 n_max (%d) and rt_stride >= m_max (%d)",
                         2 * set->n_max, set->m_max);
    if (B == 0) return VRPRPD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    ConsArgs a;
    a.tab = set->d_inst;
    a.num_inst = set->num_inst;
    a.dist = set->d_dist;
    a.proc = set->d_proc;
    a.inst = inst;
    a.heuristic = heuristic;
    a.N = set->n_max;
    a.M = set->m_max;
    a.op_stride = op_stride;
    a.rt_stride = rt_stride;
    a.ops = ops;
    a.rt_end = rt_end;
    a.ws_stride = ws_bytes(set->n_max);
    void* ws = nullptr;
    VRP_HIP(hipMallocAsync(&ws, (size_t)(a.ws_stride * B), st));
    a.ws = static_cast<unsigned char*>(ws);
    if (set->dist16)
        hipLaunchKernelGGL(k_construct<uint16_t>, dim3(B), dim3(kCT), 0, st, a);
    else
        hipLaunchKernelGGL(k_construct<int32_t>, dim3(B), dim3(kCT), 0, st, a);
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_error(e, "vrprpd_construct: launch");
    return VRPRPD_OK;
}
