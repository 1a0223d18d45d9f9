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
            for (int u = 0; u < K; ++u) {
                const int c = (ptr + u < e) ? (int)(cd[u] >> 1) : 0;
                r[u] = lds_load(&ready[c]);
            }
            bool go = true;
#pragma unroll
            for (int u = 0; u < K; ++u) {
                go = go && (ptr + u < e);
                if (go) {
                    const int c = (int)(cd[u] >> 1);
                    const int arr = o.t + leg[u];
                    if (!(cd[u] & 1u)) {
                        o.t = arr;
                        lds_store(&ready[c], arr + ~r[u]);  // ~r = p_c before the drop
                        o.w += 1;
                    } else if (r[u] >= 0) {
                        o.t = arr > r[u] ? arr : r[u];
                        o.w -= 1;
                    } else {
                        go = false;
                    }
                    if (go) {
                        ++took;
                        o.wmax = o.w > o.wmax ? o.w : o.wmax;
                        o.wmin = o.w < o.wmin ? o.w : o.wmin;
                    }
                }
            }
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
