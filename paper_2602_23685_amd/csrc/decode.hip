// brkga_decode_eval: the multi-pass decoder of Section 4.4.2 (Algorithm 2)
// and the makespan / penalised fitness of the schedule it builds.
//
// Mapping: one wavefront per chromosome.  The wave
//  1. loads and checks the 2n priority keys (and hints),
//  2. sorts (key, op index) pairs with a bitonic network in LDS,
//  3. runs the passes: the ops in priority order are scanned in chunks of 64
//     lanes; a ballot finds the next unscheduled op that is feasible at its
//     turn, lanes v < m price it on vehicle v (completion time, hint-rotated
//     tie index) and a 64-bit min-reduction picks the vehicle,
//  4. scatters the schedule into per-vehicle sequences (optional output).
#include <climits>

#include "common.h"

namespace vrprpd {

struct DecodeArgs {
    const InstDev* inst_tab;
    const void* dist;
    const int32_t* proc;
    const int32_t* inst;
    const float* prio;
    const float* hint;
    int64_t key_stride;
    int64_t* fitness;
    int32_t* makespan;
    int32_t* unscheduled;
    uint32_t* status;
    uint16_t* ops_out;     // [B][ops_stride]
    uint16_t* rt_out;      // [B][rt_stride]
    int64_t ops_stride, rt_stride;
    int64_t B;
    int32_t num_inst, n_max, cap, nblocks;
};

struct DecodeLayout {
    int keys_off, idx_off, ready_off, bits_off, bytes;
};

__host__ __device__ inline int d16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline DecodeLayout decode_layout(int n_max, int cap)
{
    DecodeLayout L;
    L.keys_off = 0;                                   // later reused for the schedule log
    L.idx_off = d16(4 * cap);
    L.ready_off = L.idx_off + d16(2 * cap);
    L.bits_off = L.ready_off + d16(4 * (n_max + 1));
    L.bytes = L.bits_off + d16(4 * ((cap + 31) / 32));
    return L;
}

__host__ __device__ inline int pow2_at_least(int x)
{
    int p = 64;
    while (p < x) p <<= 1;
    return p;
}

// -0.0 counts as 0.0; a key must lie in [0, 1) (NaN fails the test).
__device__ __forceinline__ bool key_ok(float x, uint32_t& bits)
{
    if (x == 0.0f) x = 0.0f;
    bits = __float_as_uint(x);
    return x >= 0.0f && x < 1.0f;
}

__device__ __forceinline__ int wave_min_i32(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

template <typename DT>
__global__ __launch_bounds__(64) void decode_kernel(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int64_t b = xcd_remap(blockIdx.x, a.nblocks);
    if (b >= a.B) return;
    const DecodeLayout L = decode_layout(a.n_max, a.cap);
    uint32_t* keys = reinterpret_cast<uint32_t*>(smem + L.keys_off);
    uint16_t* idx = reinterpret_cast<uint16_t*>(smem + L.idx_off);
    int* ready = reinterpret_cast<int*>(smem + L.ready_off);
    uint32_t* sched = reinterpret_cast<uint32_t*>(smem + L.bits_off);
    // schedule log, written after the sort no longer needs keys[]
    uint16_t* log_code = reinterpret_cast<uint16_t*>(smem + L.keys_off);
    uint8_t* log_veh = reinterpret_cast<uint8_t*>(smem + L.keys_off + 2 * a.cap);

    int ii = a.inst ? a.inst[b] : 0;
    const bool bad_inst = ii < 0 || ii >= a.num_inst;
    if (bad_inst) ii = 0;
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, k = I.k, R = I.R, N1 = n + 1, O = 2 * n;
    const bool minpre = I.load_model != VRPRPD_FULL_START;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const float* pr = a.prio + b * a.key_stride;
    const float* hn = a.hint ? a.hint + b * a.key_stride : nullptr;
    int cap = 64;
    while (cap < O) cap <<= 1;

    // ---- 1. keys ------------------------------------------------------------
    bool bad = bad_inst;
    for (int o = lane; o < cap; o += 64) {
        uint32_t kb = 0xFFFFFFFFu;
        if (o < O) {
            if (!key_ok(pr[o], kb)) bad = true;
            uint32_t hb;
            if (hn && !key_ok(hn[o], hb)) bad = true;
        }
        keys[o] = kb;
        idx[o] = (uint16_t)(o < O ? o : 0xFFFF);
    }
    for (int w = lane; w < (cap + 31) / 32; w += 64) sched[w] = 0u;
    for (int c = lane; c <= n; c += 64) ready[c] = 0;
    if (__ballot(bad)) {
        if (lane == 0) {
            a.fitness[b] = INT64_MAX;
            a.makespan[b] = INT32_MAX;
            a.unscheduled[b] = O;
            a.status[b] = VRPRPD_ST_BAD_KEY;
        }
        if (a.rt_out)
            for (int v = lane; v < m; v += 64) a.rt_out[b * a.rt_stride + v] = 0;
        return;
    }
    wave_lds_fence();

    // ---- 2. bitonic sort of (key, op) pairs ----------------------------------
    for (int kk = 2; kk <= cap; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < cap; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t ki = keys[i], kl = keys[l];
                    const uint16_t xi = idx[i], xl = idx[l];
                    const bool gt = ki > kl || (ki == kl && xi > xl);
                    if (gt == ((i & kk) == 0)) {
                        keys[i] = kl;
                        keys[l] = ki;
                        idx[i] = xl;
                        idx[l] = xi;
                    }
                }
            }
            wave_lds_fence();
        }
    }

    // ---- 3. passes -------------------------------------------------------------
    const bool veh = lane < m;
    int t = 0, loc = 0, q = minpre ? 0 : k, M = 0;
    bool used = false;
    int Lsum = 0, nsched = 0;
    auto can_drop = [&]() { return veh && (q > 0 || (minpre && M < k && Lsum < R)); };
    auto can_pick = [&]() { return veh && q < k; };
    bool anyD = __ballot(can_drop()) != 0, anyP = __ballot(can_pick()) != 0;
    // Per chunk of 64 ops in priority order each lane keeps its op's state in
    // registers (unscheduled, and for a pickup whether its drop is scheduled),
    // so scheduling an op needs no LDS round trip for feasibility.
    for (int pass = 0; pass < O; ++pass) {
        bool progressed = false;
        for (int base = 0; base < O; base += 64) {
            const int j = base + lane;
            const int o = j < O ? idx[j] : 0;
            bool unsched = j < O && !((sched[o >> 5] >> (o & 31)) & 1u);
            if (!__ballot(unsched)) continue;
            const int c = o / 2 + 1, isP = o & 1;
            bool dropdone = isP && unsched && ((sched[(o - 1) >> 5] >> ((o - 1) & 31)) & 1u);
            int h = 0;
            if (hn && unsched) {
                const float prod = (float)m * hn[o];
                h = (int)floorf(prod);
                h = h < m - 1 ? h : m - 1;
            }
            const int pc = (unsched && !isP) ? P[c] : 0;
            int cursor = 0;
            for (;;) {
                bool feas = false;
                if (unsched && lane >= cursor) feas = isP ? (anyP && dropdone) : anyD;
                const unsigned long long mask = __ballot(feas);
                if (!mask) break;
                const int i = __ffsll((long long)mask) - 1;   // wave-uniform: read lanes directly
                const int oi = __builtin_amdgcn_readlane(o, i), hi = __builtin_amdgcn_readlane(h, i);
                const int pci = __builtin_amdgcn_readlane(pc, i);
                const int ci = oi / 2 + 1, isPi = oi & 1;
                const int dv = veh ? (int)D[loc * N1 + ci] : 0;
                // SelectVehicle: least completion time, ties to the first
                // vehicle at or after the hint vehicle (cyclically)
                int kv = INT_MAX;
                if (veh) {
                    const int arr = t + dv;
                    bool cand;
                    int key;
                    if (!isPi) {
                        cand = q > 0 || (minpre && M < k && Lsum < R);
                        key = arr;
                    } else {
                        cand = q < k;
                        const int r = lds_load(&ready[ci]);
                        key = arr > r ? arr : r;
                    }
                    if (cand) kv = key;
                }
                // minimum over the m vehicle lanes, read one by one (no LDS crossbar)
                int ks = INT_MAX;
                for (int v = 0; v < m; ++v) {
                    const int x = __builtin_amdgcn_readlane(kv, v);
                    ks = x < ks ? x : ks;
                }
                const unsigned long long tie = __ballot(kv == ks && veh);
                const unsigned long long upper = tie & (~0ull << hi);
                const int vs = __ffsll((long long)(upper ? upper : tie)) - 1;
                const int took_preload = __builtin_amdgcn_readlane((!isPi && q == 0) ? 1 : 0, vs);
                if (lane == vs) {
                    if (!isPi) {
                        if (q == 0) { ++M; ++q; }
                        --q;
                        lds_store(&ready[ci], ks + pci);
                    } else {
                        ++q;
                        M = q > M ? q : M;
                    }
                    t = ks;
                    loc = ci;
                    used = true;
                }
                Lsum += took_preload;
                if (lane == 0) {
                    atomicOr(&sched[oi >> 5], 1u << (oi & 31));
                    log_code[nsched] = (uint16_t)((ci << 1) | isPi);
                    log_veh[nsched] = (uint8_t)vs;
                }
                ++nsched;
                if (lane == i) unsched = false;
                if (!isPi && isP && o == oi + 1) dropdone = true;   // this pickup's drop just went in
                cursor = i + 1;
                progressed = true;
                anyD = __ballot(can_drop()) != 0;
                anyP = __ballot(can_pick()) != 0;
            }
            wave_lds_fence();   // sched[] bits of this chunk before the next chunk reads them
        }
        if (nsched == O || !progressed) break;
    }

    // ---- 4. makespan, fitness, optional sequences ---------------------------------
    int ret = (veh && used) ? t + (int)D[loc * N1] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ret = max(ret, __shfl_xor(ret, o, 64));
    if (lane == 0) {
        a.makespan[b] = ret;
        a.unscheduled[b] = O - nsched;
        a.fitness[b] = (int64_t)ret + 1000000LL * (O - nsched);
        a.status[b] = (!minpre && (long long)m * k > R) ? VRPRPD_ST_RES : 0u;
    }
    if (a.ops_out && a.rt_out) {
        wave_lds_fence();
        // per-vehicle counts, then a stable scatter in schedule order
        int cnt = 0;
        for (int j0 = 0; j0 < nsched; j0 += 64) {
            const int j = j0 + lane;
            const int v = j < nsched ? log_veh[j] : -1;
            for (int u = 0; u < m; ++u) {
                const unsigned long long mk = __ballot(v == u);
                if (lane == u) cnt += __popcll(mk);
            }
        }
        // exclusive prefix over vehicles
        int incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (veh) a.rt_out[b * a.rt_stride + lane] = (uint16_t)incl;
        int off = incl - cnt;   // lane u: where vehicle u's sequence starts
        uint16_t* dst = a.ops_out + b * a.ops_stride;
        for (int j0 = 0; j0 < nsched; j0 += 64) {
            const int j = j0 + lane;
            const int v = j < nsched ? log_veh[j] : -1;
            int pos = 0;
            for (int u = 0; u < m; ++u) {
                const unsigned long long mk = __ballot(v == u);
                const int start = __shfl(off, u, 64);
                if (v == u) pos = start + __popcll(mk & ((1ull << lane) - 1));
                if (lane == u) off += __popcll(mk);
            }
            if (v >= 0) dst[pos] = log_code[j];
        }
    }
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" int brkga_decode_eval(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio,
                                 const float* hint, int64_t key_stride, int64_t* fitness, int32_t* makespan,
                                 int32_t* unscheduled, uint32_t* status, uint16_t* ops_out, uint16_t* rt_end_out,
                                 void* stream)
{
    if (!set) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: set is NULL");
    if (B < 0) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: B < 0");
    if (B == 0) return VRPRPD_OK;
    if (!prio || !fitness || !makespan || !unscheduled || !status)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: prio, fitness, makespan, unscheduled and status "
                                        "are required");
    if ((ops_out == nullptr) != (rt_end_out == nullptr))
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: pass both ops_out and rt_end_out or neither");
    const int n_lds = inst ? set->n_max : set->host[0].n;
    const int m_max = inst ? set->m_max : set->host[0].m;
    if (key_stride < 2 * (int64_t)n_lds)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: key_stride %lld < 2n = %d", (long long)key_stride,
                         2 * n_lds);
    if (2 * n_lds > 8192)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: 2n = %d exceeds the 8192 ops one CU can sort",
                         2 * n_lds);
    (void)m_max;
    const int cap = pow2_at_least(2 * n_lds);
    const DecodeLayout L = decode_layout(n_lds, cap);
    if (B > INT32_MAX) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: B too large");
    DecodeArgs a{set->d_inst, set->d_dist, set->d_proc, inst, prio, hint, key_stride, fitness, makespan,
                 unscheduled, status, ops_out, rt_end_out, 2 * (int64_t)n_lds, (int64_t)(inst ? set->m_max
                                                                                             : set->host[0].m),
                 B, set->num_inst, n_lds, cap, (int32_t)B};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto launch = [&](auto* k) -> int {
        if (L.bytes > 64 * 1024)
            VRP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, L.bytes));
        hipLaunchKernelGGL(k, dim3((unsigned)B), dim3(64), L.bytes, st, a);
        VRP_HIP(hipGetLastError());
        return VRPRPD_OK;
    };
    return set->dist16 ? launch(decode_kernel<uint16_t>) : launch(decode_kernel<int32_t>);
}
