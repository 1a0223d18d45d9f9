// The timing sweep shared by the evaluation kernels.
//
// A group of GL lanes holds one candidate whose ops are staged in LDS (see
// OpStore): for op j its code (c << 1 | isPickup) and leg[j], the travel time
// into op j from the previous stop of its route.  ready[c] holds ~p_c
// (negative: "not dropped yet") until c's drop, then the drop time + p_c, the
// earliest pickup (Eq. 9).
//
// Lane v < m walks route v.  At each step a lane takes up to K consecutive
// ops of its route: a drop happens on arrival (Eq. 7) and publishes ready[c];
// a pickup departs at max(arrival, ready[c]) (Eq. 8-10) or, if its drop has
// not happened yet, holds the vehicle and ends the lane's step.  ready values
// are written once, so a pickup that reads one reads its final value; taking
// ops in any order that respects these waits yields the same earliest-start
// schedule.  A step in which no lane of the group moves while some still have
// ops proves a cycle of waits (deadlock).
#pragma once

#include "common.h"

namespace vrprpd {

// Ops of one candidate in LDS.  With 16-bit travel times, code and leg share
// a 32-bit word (one LDS read per op); otherwise they live in two arrays.
template <typename DT>
struct OpStore;

template <>
struct OpStore<uint16_t> {
    uint32_t* w;
    static constexpr int kBytesPerOp = 4;
    __device__ __forceinline__ void init(unsigned char* base, int /*cap*/) { w = reinterpret_cast<uint32_t*>(base); }
    __device__ __forceinline__ void set_code(int j, uint32_t cd) { w[j] = cd; }
    __device__ __forceinline__ uint32_t code(int j) const { return w[j] & 0xFFFFu; }
    __device__ __forceinline__ void set_leg(int j, int leg) { w[j] = (w[j] & 0xFFFFu) | ((uint32_t)leg << 16); }
    __device__ __forceinline__ void set(int j, uint32_t cd, int leg) { w[j] = cd | ((uint32_t)leg << 16); }
    // halves written separately (no read-modify-write)
    __device__ __forceinline__ void put_code(int j, uint32_t cd) { reinterpret_cast<uint16_t*>(w)[2 * j] = (uint16_t)cd; }
    __device__ __forceinline__ void put_leg(int j, int leg) { reinterpret_cast<uint16_t*>(w)[2 * j + 1] = (uint16_t)leg; }
    __device__ __forceinline__ void load(int j, uint32_t& cd, int& leg) const
    {
        const uint32_t x = w[j];
        cd = x & 0xFFFFu;
        leg = (int)(x >> 16);
    }
};

template <>
struct OpStore<int32_t> {
    uint16_t* c;
    int32_t* l;
    static constexpr int kBytesPerOp = 6;
    __device__ __forceinline__ void init(unsigned char* base, int cap)
    {
        l = reinterpret_cast<int32_t*>(base);
        c = reinterpret_cast<uint16_t*>(base + 4 * (size_t)cap);
    }
    __device__ __forceinline__ void set_code(int j, uint32_t cd) { c[j] = (uint16_t)cd; }
    __device__ __forceinline__ uint32_t code(int j) const { return c[j]; }
    __device__ __forceinline__ void set_leg(int j, int leg) { l[j] = leg; }
    __device__ __forceinline__ void set(int j, uint32_t cd, int leg)
    {
        c[j] = (uint16_t)cd;
        l[j] = leg;
    }
    __device__ __forceinline__ void put_code(int j, uint32_t cd) { c[j] = (uint16_t)cd; }
    __device__ __forceinline__ void put_leg(int j, int leg) { l[j] = leg; }
    __device__ __forceinline__ void load(int j, uint32_t& cd, int& leg) const
    {
        cd = c[j];
        leg = l[j];
    }
};

struct SweepOut {
    int t;              // lane's vehicle clock after its last op
    int w, wmax, wmin;  // drops-minus-pickups walk of the lane's route
    bool dead;          // group deadlocked
};

// One lane's attempt at its next K ops (branch-free).  cd/leg: the ops; r:
// ready[] entries read at the start of the step; n_left: ops left on the
// route.  Returns the number of ops taken.
// kPolarity: ready[] entries are stored XOR pm (pm = 0 or -1, the sign
// convention of the evaluation, see sweep_route) and pv[u] = p_c of op u,
// read beside r[u]; otherwise (the explicit evaluation) ready[c] = ~p_c
// before the drop, so the drop's ready time is arr + p_c with p_c = ~r.
template <int K, bool kPolarity>
__device__ __forceinline__ int sweep_step(SweepOut& o, const uint32_t* cd, const int* leg, const int* r,
                                          int n_left, int* ready, const int* pv, int pm)
{
    bool go = true;
    int took = 0;
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const bool isP = cd[u] & 1u;
        const int c = (int)(cd[u] >> 1);
        const int arr = o.t + leg[u];
        const int rv = kPolarity ? (r[u] ^ pm) : r[u];
        const bool rdy = rv >= 0;
        const bool ok = go && (u < n_left) && (!isP || rdy);
        const int tn = isP ? (arr > rv ? arr : rv) : arr;
        // A drop publishes its ready time.  Every other case writes to the
        // unused slot ready[0] instead of branching around the store.
        const bool pub = ok && !isP;
        const int val = kPolarity ? ((arr + pv[u]) ^ pm) : arr + ~r[u];
        lds_store(&ready[pub ? c : 0], val);
        o.t = ok ? tn : o.t;
        o.w += ok ? (isP ? -1 : 1) : 0;
        o.wmax = o.w > o.wmax ? o.w : o.wmax;
        o.wmin = o.w < o.wmin ? o.w : o.wmin;
        took += ok ? 1 : 0;
        go = ok;
    }
    return took;
}

// The op store must hold valid codes for K entries past the last route.
template <int GL, int K, typename DT>
__device__ __forceinline__ SweepOut sweep_group(const OpStore<DT>& S, int* ready, int s, int e)
{
    SweepOut o{0, 0, 0, 0, false};
    int ptr = s;
    for (;;) {
        int took = 0;
        if (ptr < e) {
            uint32_t cd[K];
            int leg[K], r[K];
#pragma unroll
            for (int u = 0; u < K; ++u) S.load(ptr + u, cd[u], leg[u]);
#pragma unroll
            for (int u = 0; u < K; ++u) r[u] = lds_load(&ready[cd[u] >> 1]);   // valid codes past e (padding)
            took = sweep_step<K, false>(o, cd, leg, r, e - ptr, ready, nullptr, 0);
            ptr += took;
        }
        const uint64_t left = group_ballot<GL>(ptr < e);
        if (!left) break;
        const uint64_t moved = group_ballot<GL>(took > 0);
        if (!moved) {
            o.dead = true;
            break;
        }
    }
    // A deadlock stops the clocks but the load check covers whole routes.
    for (; ptr < e; ++ptr) {
        o.w += (S.code(ptr) & 1u) ? -1 : 1;
        o.wmax = o.w > o.wmax ? o.w : o.wmax;
        o.wmin = o.w < o.wmin ? o.w : o.wmin;
    }
    return o;
}


// ---------------------------------------------------------------------------
// Sweep over "virtual" routes: a staged base solution seen through a Route
// object that splices ops in or out (Route::vlen, Route::fetch(i, code, leg)).
// A step fetches its K ops without testing the route's end: the op store
// holds valid codes past every route (the next route's ops, then K padding
// entries of code 0), so every fetch and ready[] read stays in range and the
// ops past the end are never taken.
// ready[] keeps no per-evaluation initialisation: its sign convention flips
// with `pol` after every completed evaluation (see the insertion scan).
// pblk[c] = p_c for the drop's ready time.  Route::record(i, t) may keep the
// time of each op taken.
template <int K, int GL, typename Route>
__device__ __forceinline__ SweepOut sweep_route(const Route& R, int* ready, const int* pblk, int pol)
{
    SweepOut o{0, 0, 0, 0, false};
    int ptr = 0;
    const int e = R.vlen;
    const int pm = -pol;   // stored entries are XOR pm: 0 or all ones
    for (;;) {
        int took = 0;
        if (ptr < e) {
            uint32_t cd[K];
            int leg[K], r[K], pv[K];
            // Most steps of the wave touch no splice point: their ops are a
            // contiguous slice of the base, read without the selects.
            if (__builtin_amdgcn_ballot_w64(!R.plain(ptr, K)) == 0) {
                const int j0 = R.plain_base(ptr);
#pragma unroll
                for (int u = 0; u < K; ++u) R.S->load(j0 + u, cd[u], leg[u]);
            } else {
#pragma unroll
                for (int u = 0; u < K; ++u) R.fetch(ptr + u, cd[u], leg[u]);
            }
#pragma unroll
            for (int u = 0; u < K; ++u) {
                r[u] = lds_load(&ready[cd[u] >> 1]);
                pv[u] = lds_load(&pblk[cd[u] >> 1]);
            }
            if constexpr (Route::kRecords) {
                // record needs each op's own time: take the ops one by one
                SweepOut o2 = o;
                took = sweep_step<K, true>(o2, cd, leg, r, e - ptr, ready, pv, pm);
                int t = o.t;
                for (int u = 0; u < took; ++u) {
                    const int arr = t + leg[u];
                    const int rv = r[u] ^ pm;
                    t = (cd[u] & 1u) ? (arr > rv ? arr : rv) : arr;
                    R.record(ptr + u, t);
                }
                o = o2;
            } else {
                took = sweep_step<K, true>(o, cd, leg, r, e - ptr, ready, pv, pm);
            }
            ptr += took;
        }
        if (!group_ballot<GL>(ptr < e)) break;
        if (!group_ballot<GL>(took > 0)) {
            o.dead = true;
            break;
        }
    }
    for (; ptr < e; ++ptr) {
        uint32_t cd;
        int leg;
        R.fetch(ptr, cd, leg);
        o.w += (cd & 1u) ? -1 : 1;
        o.wmax = o.w > o.wmax ? o.w : o.wmax;
        o.wmin = o.w < o.wmin ? o.w : o.wmin;
    }
    return o;
}

constexpr int kNoPos = 1 << 30;  // far past any route, and x + 1 cannot overflow

// A base route with up to two ops spliced in at virtual positions x1 < x2
// (kNoPos when absent).  lgX is the leg into the spliced op, laX the leg into
// the base op right after it; ret is the leg from the last stop to the depot.
template <typename DT>
struct InsRoute {
    static constexpr bool kRecords = false;
    const OpStore<DT>* S;
    int bs, len, vlen;
    int x1, x2;
    uint32_t k1, k2;
    int lg1, lg2, la1, la2;
    int ret;
    // Branch-free: the base op is loaded in every case and replaced by
    // selects (at i = x1 or x2 the load reads a neighbouring base op).
    __device__ __forceinline__ void fetch(int i, uint32_t& cd, int& leg) const
    {
        uint32_t c0;
        int l0;
        S->load(bs + i - (i > x1) - (i > x2), c0, l0);
        cd = i == x1 ? k1 : (i == x2 ? k2 : c0);
        leg = i == x1 ? lg1 : (i == x2 ? lg2 : (i == x1 + 1 ? la1 : (i == x2 + 1 ? la2 : l0)));
    }
    // Ops ptr .. ptr + K - 1 are base ops plain_base(ptr) + u with their own
    // legs when the window holds neither spliced op nor the op after one.
    __device__ __forceinline__ bool plain(int ptr, int K) const
    {
        return (ptr > x1 + 1 || ptr + K <= x1) && (ptr > x2 + 1 || ptr + K <= x2);
    }
    __device__ __forceinline__ int plain_base(int ptr) const { return bs + ptr - (ptr > x1) - (ptr > x2); }
    __device__ __forceinline__ void record(int, int) const {}
};

// A base route with up to two ops taken out (base positions y1 < y2 relative
// to the route start, kNoPos when absent).  lb1 / lb2 are the legs into the
// first kept op after y1 / after y2; times, when set, receive the time of
// each kept op at its base index.
template <typename DT, bool kRec>
struct DelRouteT {
    static constexpr bool kRecords = kRec;
    const OpStore<DT>* S;
    int bs, vlen;
    int y1, y2;      // virtual index of the first kept op after each removal
    int lb1, lb2;
    int* times;
    __device__ __forceinline__ int base_index(int i) const { return bs + i + (i >= y1) + (i >= y2); }
    __device__ __forceinline__ void fetch(int i, uint32_t& cd, int& leg) const
    {
        int l0;
        S->load(base_index(i), cd, l0);
        leg = i == y2 ? lb2 : (i == y1 ? lb1 : l0);
    }
    // As for InsRoute: the window holds no op whose leg was replaced.
    __device__ __forceinline__ bool plain(int ptr, int K) const
    {
        return (ptr > y1 || ptr + K <= y1) && (ptr > y2 || ptr + K <= y2);
    }
    __device__ __forceinline__ int plain_base(int ptr) const { return base_index(ptr); }
    __device__ __forceinline__ void record(int i, int t) const
    {
        if (times) times[base_index(i)] = t;
    }
};

// Load and resource status of a group (Eq. 13-18 under the load model).
template <int GL>
__device__ __forceinline__ uint32_t load_status(const SweepOut& o, bool is_vehicle, int m, int k, int R, int lm)
{
    bool bad = false;
    int pre = 0;
    if (is_vehicle) {
        if (lm == VRPRPD_FULL_START) {
            bad = o.wmin < 0 || o.wmax > k;
        } else {
            bad = o.wmax - o.wmin > k;
            pre = o.wmax;
        }
    }
    uint32_t st = group_ballot<GL>(bad) ? VRPRPD_ST_LOAD : 0u;
    const int need = group_sum<GL>(pre);
    if (lm == VRPRPD_FULL_START) {
        if ((long long)m * k > R) st |= VRPRPD_ST_RES;
    } else if (need > R) {
        st |= VRPRPD_ST_RES;
    }
    return st;
}

}  // namespace vrprpd
