// brkga_decode_eval: the multi-pass decoder of Section 4.4.2 (Algorithm 2)
// and the makespan / penalised fitness of the schedule it builds.
//
// Mapping: one block per chromosome in each of two launches.
//  decode_sort_kernel (four waves): loads and checks the 2n priority keys (and
//     hints) and sorts (key, op index) pairs with a bitonic network in LDS;
//     the op order goes to a workspace in global memory.
//  decode_kernel (one wave): runs the passes: the ops in priority order are
//     read in chunks of 64 lanes (the next chunk's load in flight); lane masks
//     give the next unscheduled op that is feasible at its turn, lanes v < m
//     price it on vehicle v (completion time, hint-rotated tie index) and the
//     least key picks the vehicle; then optionally scatters the schedule into
//     per-vehicle sequences.
// The passes, a long chain of dependent wave-wide decisions, keep only
// ready[] and the scheduled-op bits in LDS (about 4n bytes), so many more
// chromosomes are in flight per CU than if the sort's 6 bytes per op stayed
// allocated through them.
#include <climits>
#include <mutex>

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
    uint16_t* order;       // [B][cap] op indices in priority order (workspace)
    uint8_t* badkey;       // [B] 1: the chromosome's keys failed the check (workspace)
    uint32_t* log;         // [B][cap] schedule log, code | vehicle << 16 (workspace, with ops_out)
};

__host__ __device__ inline int d16(int x) { return (x + 15) & ~15; }

// LDS of the sort launch: (key << 16 | op index) pairs.
__host__ __device__ inline int sort_lds_bytes(int cap) { return 8 * cap; }
// LDS of the pass launch: ready[], scheduled bits.
struct DecodeLayout {
    int ready_off, bits_off, bytes;
};
__host__ __device__ inline DecodeLayout decode_layout(int n_max, int cap)
{
    DecodeLayout L;
    L.ready_off = 0;
    L.bits_off = d16(4 * (n_max + 1));
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

constexpr int kSortThreads = 256;   // threads per chromosome in the key sort

__global__ __launch_bounds__(kSortThreads) void decode_sort_kernel(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int64_t b = xcd_remap(blockIdx.x, a.nblocks);
    if (b >= a.B) return;
    unsigned long long* kx = reinterpret_cast<unsigned long long*>(smem);
    int ii = a.inst ? a.inst[b] : 0;
    const bool bad_inst = ii < 0 || ii >= a.num_inst;
    if (bad_inst) ii = 0;
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, O = 2 * n;
    const float* pr = a.prio + b * a.key_stride;
    const float* hn = a.hint ? a.hint + b * a.key_stride : nullptr;
    int cap = 64;
    while (cap < O) cap <<= 1;

    // ---- 1. keys ------------------------------------------------------------
    bool bad = bad_inst;
    // A valid key is a non-negative float, so its bits order like the value;
    // the op index in the low 16 bits breaks ties (padding sorts last).
    for (int o = tid; o < cap; o += kSortThreads) {
        uint32_t kb = 0xFFFFFFFFu;
        if (o < O) {
            if (!key_ok(pr[o], kb)) bad = true;
            uint32_t hb;
            if (hn && !key_ok(hn[o], hb)) bad = true;
        }
        kx[o] = ((unsigned long long)kb << 16) | (unsigned)(o < O ? o : 0xFFFF);
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) {
            a.badkey[b] = 1;
            a.fitness[b] = INT64_MAX;
            a.makespan[b] = INT32_MAX;
            a.unscheduled[b] = O;
            a.status[b] = VRPRPD_ST_BAD_KEY;
        }
        if (a.rt_out)
            for (int v = tid; v < m; v += kSortThreads) a.rt_out[b * a.rt_stride + v] = 0;
        return;
    }

    // ---- 2. bitonic sort of (key, op) pairs ----------------------------------
    block_sort_u64(kx, cap);
    uint16_t* ord = a.order + b * a.cap;
    for (int j = tid; j < O; j += kSortThreads) ord[j] = (uint16_t)(kx[j] & 0xFFFFu);
    if (tid == 0) a.badkey[b] = 0;
}

// Minima by DPP row shifts (VALU only, no LDS crossbar, no scalar chain):
// after shifts by 1, 2, 4, 8 within each row of 16 lanes, lane 15 of a row
// holds the row's minimum; row broadcasts fold rows 0-3 into lane 63.
// Lanes a shift reads from outside the row keep INT_MAX.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_min_step(int x)
{
    const int y = __builtin_amdgcn_update_dpp(INT_MAX, x, CTRL, ROWS, 0xF, false);
    return y < x ? y : x;
}
__device__ __forceinline__ int row0_min(int x)   // minimum over lanes 0-15
{
    x = dpp_min_step<0x111, 0xF>(x);   // row_shr:1
    x = dpp_min_step<0x112, 0xF>(x);   // row_shr:2
    x = dpp_min_step<0x114, 0xF>(x);   // row_shr:4
    x = dpp_min_step<0x118, 0xF>(x);   // row_shr:8
    return __builtin_amdgcn_readlane(x, 15);
}
__device__ __forceinline__ int wave_min_dpp(int x)   // minimum over all 64 lanes
{
    x = dpp_min_step<0x111, 0xF>(x);
    x = dpp_min_step<0x112, 0xF>(x);
    x = dpp_min_step<0x114, 0xF>(x);
    x = dpp_min_step<0x118, 0xF>(x);
    x = dpp_min_step<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_min_step<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(x, 63);
}

// kSmallM: every instance has m <= 16 (vehicle minimum within one DPP row).
// kLog: the schedule is logged for the op sequences (ops_out).
// kPacked (with kSmallM): every time is below 2^27, so a vehicle's key
// (completion time << 4 | its rank in the hint-rotated order) fits 31 bits
// and one minimum gives both the time and the vehicle.
// kHintFirst: the hint-first vehicle rule (VRPRPD_DECODE_HINT_FIRST).
template <typename DT, bool kSmallM, bool kLog, bool kPacked, bool kHintFirst>
__global__ __launch_bounds__(64) void decode_kernel(DecodeArgs a)
{
    static_assert(!kPacked || kSmallM, "packed keys need m <= 16");
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int64_t b = xcd_remap(blockIdx.x, a.nblocks);
    if (b >= a.B || a.badkey[b]) return;
    const DecodeLayout L = decode_layout(a.n_max, a.cap);
    int* ready = reinterpret_cast<int*>(smem + L.ready_off);
    uint32_t* sched = reinterpret_cast<uint32_t*>(smem + L.bits_off);
    const uint16_t* ord = a.order + b * a.cap;
    uint32_t* log = kLog ? a.log + b * a.cap : nullptr;

    const int ii = a.inst ? a.inst[b] : 0;    // in range: the sort launch checked it
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, k = I.k, R = I.R, N1 = n + 1, O = 2 * n;
    const bool minpre = I.load_model != VRPRPD_FULL_START;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const float* hn = a.hint ? a.hint + b * a.key_stride : nullptr;
    for (int w = lane; w < (O + 31) / 32; w += 64) sched[w] = 0u;
    for (int c = lane; c <= n; c += 64) ready[c] = 0;
    wave_lds_fence();

    // ---- 3. passes -------------------------------------------------------------
    const bool veh = lane < m;
    const unsigned long long VEH = m >= 64 ? ~0ull : (1ull << m) - 1ull;   // vehicle lanes
    // lrow: matrix row offset of the vehicle's location (the depot's, 0, at
    // the start; lanes past m stay there and read valid entries)
    int t = 0, lrow = 0, q = minpre ? 0 : k, M = 0;
    int used = 0;
    int Lsum = 0, nsched = 0;
    // dok / pok: this lane's vehicle can take a drop (holds a resource, or
    // may preload one) / a pickup; anyD / anyP: the lanes where it holds.
    // Bitwise forms keep the tests free of branches.
    bool dok, pok;
    unsigned long long anyD, anyP;
    auto vehicle_tests = [&]() {
        dok = veh & ((q > 0) | (minpre & (Lsum < R) & (M < k)));
        pok = veh & (q < k);
        anyD = __builtin_amdgcn_ballot_w64(dok);
        anyP = __builtin_amdgcn_ballot_w64(pok);
    };
    vehicle_tests();
    // Per chunk of 64 ops in priority order the wave keeps the chunk's state
    // as lane masks (unscheduled, pickup, pickup whose drop is scheduled), so
    // finding the next feasible op is a few scalar operations.  Every lane
    // runs the vehicle arithmetic; vehicle lanes differ only in their data.
    for (int pass = 0; pass < O; ++pass) {
        bool progressed = false;
        int o_next = lane < O ? ord[lane] : 0;
        for (int base = 0; base < O; base += 64) {
            const int j = base + lane;
            const int o = o_next;
            if (base + 64 < O) o_next = j + 64 < O ? ord[j + 64] : 0;   // next chunk's load in flight
            const bool uns = j < O && !((sched[o >> 5] >> (o & 31)) & 1u);
            unsigned long long U = __ballot(uns);
            if (!U) continue;
            const unsigned long long U0 = U;
            const int c = o / 2 + 1, isP = o & 1;
            const unsigned long long PM = __ballot(isP);
            unsigned long long DD = __ballot(isP && uns && ((sched[(o - 1) >> 5] >> ((o - 1) & 31)) & 1u));
            int h = 0;
            if (hn && uns) {
                const float prod = (float)m * hn[o];
                h = (int)floorf(prod);
                h = h < m - 1 ? h : m - 1;
            }
            const int pc = (uns && !isP) ? P[c] : 0;
            unsigned long long avail = ~0ull;   // lanes after the last op taken in this chunk
            for (;;) {
                const unsigned long long mask =
                    avail & U & ((anyD ? ~PM : 0ull) | (anyP ? (PM & DD) : 0ull));
                if (!mask) break;
                const int i = __ffsll((long long)mask) - 1;
                const int oi = __builtin_amdgcn_readlane(o, i), hi = __builtin_amdgcn_readlane(h, i);
                const int pci = __builtin_amdgcn_readlane(pc, i);
                const int ci = (int)((unsigned)oi >> 1) + 1;
                const bool isPi = oi & 1;
                // SelectVehicle: least completion time, ties to the first
                // vehicle at or after the hint vehicle (cyclically).  The
                // travel time is read at a 32-bit byte offset from the
                // uniform matrix base; a drop reads ready[] too and ignores it.
                const uint32_t eoff = (uint32_t)(lrow + ci) * (uint32_t)sizeof(DT);
                const int arr = t + (int)*reinterpret_cast<const DT*>(reinterpret_cast<const unsigned char*>(D) + eoff);
                const int r = lds_load(&ready[ci]);
                const int key = isPi ? (arr > r ? arr : r) : arr;
                const int kv = (isPi ? pok : dok) ? key : INT_MAX;
                int ks, vs;
                // hint-first rule: the hint vehicle, if it can take the op
                const int kh = kHintFirst ? __builtin_amdgcn_readlane(kv, hi) : INT_MAX;
                if (kHintFirst && kh != INT_MAX) {
                    ks = kh;
                    vs = hi;
                } else if constexpr (kPacked) {
                    // rank (v - hint) mod 16: the hint vehicle first, then
                    // the following ones cyclically (lanes >= m hold INT_MAX)
                    const int kp = kv == INT_MAX ? INT_MAX : (kv << 4) | ((lane - hi) & 15);
                    const int kq = row0_min(kp);
                    ks = kq >> 4;
                    vs = ((kq & 15) + hi) & 15;
                } else {
                    ks = kSmallM ? row0_min(kv) : wave_min_dpp(kv);
                    const unsigned long long tie = __builtin_amdgcn_ballot_w64(kv == ks) & VEH;
                    const unsigned long long upper = tie & (~0ull << hi);
                    vs = __ffsll((long long)(upper ? upper : tie)) - 1;
                }
                const bool me = lane == vs;
                // a drop on an empty vehicle preloads one resource (the
                // chosen vehicle's update computed in every lane, then kept
                // in its lane by selects)
                const int qv = __builtin_amdgcn_readlane(q, vs);
                const int pre = (int)(!isPi & (qv == 0));
                Lsum += pre;
                const int qn = q + (isPi ? 1 : pre - 1);
                const int Mp = qn > M ? qn : M;
                const int Mn = isPi ? Mp : M + pre;
                q = me ? qn : q;
                M = me ? Mn : M;
                // a drop publishes its ready time; a pickup writes the unused
                // depot slot (same address and value in every lane)
                lds_store(&ready[isPi ? 0 : ci], ks + pci);
                // this drop's pickup, if in the chunk (after a pickup the
                // match is a drop lane, whose bit is never read)
                DD |= __builtin_amdgcn_ballot_w64(o == oi + 1);
                t = me ? ks : t;
                lrow = me ? ci * N1 : lrow;
                used |= me ? 1 : 0;
                if constexpr (kLog) log[nsched] = (uint32_t)((ci << 1) | (int)isPi) | ((uint32_t)vs << 16);
                ++nsched;
                U &= ~(1ull << i);
                avail = ~((2ull << i) - 1ull);
                progressed = true;
                vehicle_tests();
            }
            // the chunk's newly scheduled ops, published before the next chunk reads them
            if (((U0 & ~U) >> lane) & 1ull) atomicOr(&sched[o >> 5], 1u << (o & 31));
            wave_lds_fence();
        }
        if (nsched == O || !progressed) break;
    }

    // ---- 4. makespan, fitness, optional sequences ---------------------------------
    int ret = (veh && used) ? t + (int)D[lrow] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ret = max(ret, __shfl_xor(ret, o, 64));
    if (lane == 0) {
        a.makespan[b] = ret;
        a.unscheduled[b] = O - nsched;
        a.fitness[b] = (int64_t)ret + 1000000LL * (O - nsched);
        a.status[b] = (!minpre && (long long)m * k > R) ? VRPRPD_ST_RES : 0u;
    }
    if constexpr (kLog) {
        __threadfence_block();   // the log written by lane 0, read by every lane
        // per-vehicle counts, then a stable scatter in schedule order
        int cnt = 0;
        for (int j0 = 0; j0 < nsched; j0 += 64) {
            const int j = j0 + lane;
            const int v = j < nsched ? (int)(log[j] >> 16) : -1;
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
            const uint32_t e = j < nsched ? log[j] : 0u;
            const int v = j < nsched ? (int)(e >> 16) : -1;
            int pos = 0;
            for (int u = 0; u < m; ++u) {
                const unsigned long long mk = __ballot(v == u);
                const int start = __shfl(off, u, 64);
                if (v == u) pos = start + __popcll(mk & ((1ull << lane) - 1));
                if (lane == u) off += __popcll(mk);
            }
            if (v >= 0) dst[pos] = (uint16_t)(e & 0xFFFFu);
        }
    }
}

// Workspace of one launch over B chromosomes: op orders, key flags and, when
// the sequences are wanted, the schedule logs.
template <typename DT, bool kHintFirst>
static const void* decode_kernel_for(bool small_m, bool packed, bool log)
{
    if (small_m && packed)
        return log ? (const void*)decode_kernel<DT, true, true, true, kHintFirst>
                   : (const void*)decode_kernel<DT, true, false, true, kHintFirst>;
    if (small_m)
        return log ? (const void*)decode_kernel<DT, true, true, false, kHintFirst>
                   : (const void*)decode_kernel<DT, true, false, false, kHintFirst>;
    return log ? (const void*)decode_kernel<DT, false, true, false, kHintFirst>
               : (const void*)decode_kernel<DT, false, false, false, kHintFirst>;
}

int64_t decode_ws_bytes(const vrprpd_set* set, int64_t B, bool by_inst, bool want_ops)
{
    const int n_lds = by_inst ? set->n_max : set->host[0].n;
    const int64_t cap = pow2_at_least(2 * n_lds);
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    return up(2 * cap * B) + up(B) + (want_ops ? up(4 * cap * B) : 0);
}

int decode_launch(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio, const float* hint,
                  int64_t key_stride, int32_t flags, int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                  uint32_t* status, uint16_t* ops_out, uint16_t* rt_end_out, void* ws, hipStream_t st)
{
    if (!set) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: set is NULL");
    if (flags & ~VRPRPD_DECODE_HINT_FIRST) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: unknown flags %d", flags);
    if (B < 0) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: B < 0");
    if (B == 0) return VRPRPD_OK;
    if (!prio || !fitness || !makespan || !unscheduled || !status)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: prio, fitness, makespan, unscheduled and status "
                                        "are required");
    if ((ops_out == nullptr) != (rt_end_out == nullptr))
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: pass both ops_out and rt_end_out or neither");
    const int n_lds = inst ? set->n_max : set->host[0].n;
    if (key_stride < 2 * (int64_t)n_lds)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: key_stride %lld < 2n = %d", (long long)key_stride,
                         2 * n_lds);
    if (2 * n_lds > 8192)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval: 2n = %d exceeds the 8192 ops one CU can sort",
                         2 * n_lds);
    if (B > INT32_MAX) return set_error(VRPRPD_EINVAL, "brkga_decode_eval: B too large");
    const int cap = pow2_at_least(2 * n_lds);
    const DecodeLayout L = decode_layout(n_lds, cap);
    const int sort_lds = sort_lds_bytes(cap);
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    unsigned char* w = static_cast<unsigned char*>(ws);
    uint16_t* order = reinterpret_cast<uint16_t*>(w);
    uint8_t* badkey = w + up(2 * (int64_t)cap * B);
    uint32_t* log = ops_out ? reinterpret_cast<uint32_t*>(w + up(2 * (int64_t)cap * B) + up(B)) : nullptr;
    DecodeArgs a{set->d_inst, set->d_dist, set->d_proc, inst, prio, hint, key_stride, fitness, makespan,
                 unscheduled, status, ops_out, rt_end_out, 2 * (int64_t)n_lds, (int64_t)(inst ? set->m_max
                                                                                             : set->host[0].m),
                 B, set->num_inst, n_lds, cap, (int32_t)B, order, badkey, log};
    auto launch = [&](const void* k, int lds) -> int {
        if (lds > 64 * 1024) VRP_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        return VRPRPD_OK;
    };
    int rc = launch(reinterpret_cast<const void*>(decode_sort_kernel), sort_lds);
    if (rc) return rc;
    hipLaunchKernelGGL(decode_sort_kernel, dim3((unsigned)B), dim3(kSortThreads), sort_lds, st, a);
    VRP_HIP(hipGetLastError());
    const bool small_m = (inst ? set->m_max : set->host[0].m) <= 16;
    const bool packed = set->time_bound < (int64_t(1) << 27);   // (time << 4) | 15 stays below 2^31
    const bool hf = (flags & VRPRPD_DECODE_HINT_FIRST) != 0;
    const void* kern = set->dist16 ? (hf ? decode_kernel_for<uint16_t, true>(small_m, packed, log != nullptr)
                                         : decode_kernel_for<uint16_t, false>(small_m, packed, log != nullptr))
                                   : (hf ? decode_kernel_for<int32_t, true>(small_m, packed, log != nullptr)
                                         : decode_kernel_for<int32_t, false>(small_m, packed, log != nullptr));
    if ((rc = launch(kern, L.bytes))) return rc;
    void* kargs[] = {&a};
    VRP_HIP(hipLaunchKernel(kern, dim3((unsigned)B), dim3(64), kargs, (size_t)L.bytes, st));
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" int brkga_decode_eval(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio,
                                 const float* hint, int64_t key_stride, int32_t flags, int64_t* fitness,
                                 int32_t* makespan, int32_t* unscheduled, uint32_t* status, uint16_t* ops_out,
                                 uint16_t* rt_end_out, void* stream)
{
    if (!set || B <= 0)   // argument errors and the empty batch: no workspace
        return decode_launch(set, B, inst, prio, hint, key_stride, flags, fitness, makespan, unscheduled, status, ops_out,
                             rt_end_out, nullptr, reinterpret_cast<hipStream_t>(stream));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    void* ws = nullptr;
    VRP_HIP(hipMallocAsync(&ws, (size_t)decode_ws_bytes(set, B, inst != nullptr, ops_out != nullptr), st));
    const int rc = decode_launch(set, B, inst, prio, hint, key_stride, flags, fitness, makespan, unscheduled, status,
                                 ops_out, rt_end_out, ws, st);
    (void)hipFreeAsync(ws, st);
    return rc;
}

// ---------------------------------------------------------------- no-allocation variant
// The workspace of brkga_decode_eval_noalloc: one file-scope device array.
// Each GPU the library runs on holds its own copy (at its own address) from
// the module's load to the end of the process.  In host code the name stands
// for a host-side shadow, never for device memory: kernels get the address
// hipGetSymbolAddress returns for the current device.
static constexpr int64_t kDecodeScratchBytes = int64_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kDecodeScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};   // device ordinal -> address of that device's scratch
}  // namespace

// Address of the current device's scratch array, looked up once per device.
static int scratch_for_current_device(void** out)
{
    int dev = -1;
    VRP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices)
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval_noalloc: device %d (at most %d devices)", dev,
                         kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                             "brkga_decode_eval_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return VRPRPD_OK;
}

extern "C" int64_t brkga_decode_noalloc_max_bytes(void) { return kDecodeScratchBytes; }

extern "C" int brkga_decode_eval_noalloc(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio,
                                         const float* hint, int64_t key_stride, int32_t flags, int64_t* fitness,
                                         int32_t* makespan, int32_t* unscheduled, uint32_t* status,
                                         uint16_t* ops_out, uint16_t* rt_end_out, void* stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!set || B <= 0)   // argument errors and the empty batch: no workspace touched
        return decode_launch(set, B, inst, prio, hint, key_stride, flags, fitness, makespan, unscheduled, status, ops_out,
                             rt_end_out, nullptr, st);
    const int n_lds = inst ? set->n_max : set->host[0].n;
    if (2 * n_lds > 8192)   // decode_launch reports it; keep the size arithmetic below in range
        return decode_launch(set, B, inst, prio, hint, key_stride, flags, fitness, makespan, unscheduled, status, ops_out,
                             rt_end_out, nullptr, st);
    if (B > (int64_t(1) << 40))
        return set_error(VRPRPD_EINVAL, "brkga_decode_eval_noalloc: B = %lld is beyond the %lld-byte workspace",
                         (long long)B, (long long)kDecodeScratchBytes);
    const int64_t need = decode_ws_bytes(set, B, inst != nullptr, ops_out != nullptr);
    if (need > kDecodeScratchBytes)
        return set_error(VRPRPD_EINVAL,
                         "brkga_decode_eval_noalloc: %lld chromosomes of 2n = %d ops need a %lld-byte workspace; "
                         "the fixed one holds %lld bytes (use brkga_decode_eval or a smaller batch)",
                         (long long)B, 2 * n_lds, (long long)need, (long long)kDecodeScratchBytes);
    void* ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    return decode_launch(set, B, inst, prio, hint, key_stride, flags, fitness, makespan, unscheduled, status, ops_out,
                         rt_end_out, ws, st);
}
