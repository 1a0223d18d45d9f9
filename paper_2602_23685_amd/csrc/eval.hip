// vrprpd_eval: exact makespan of explicit candidates (Section 3, Eq. 1-23).
//
// Mapping: a group of GL lanes (GL = 16, 32 or 64, at least m) owns one
// candidate; up to 64/GL groups share a one-wave block (candidates per wave
// is a tuned launch parameter).
// Phase 1 streams the candidate's ops from HBM once (coalesced, route by
// route) and checks cover with an LDS bitmap.  Phase 2 is the lockstep
// timing sweep (sweep.h), lane v = vehicle v.  Two forms, chosen per (n, m)
// by the autotuner: "staged" (eval_kernel) gathers every travel time
// d[prev][c] into LDS in phase 1, so the sweep reads only LDS; "live legs"
// (eval_live_kernel) keeps only the op codes in LDS and reads each travel
// time from the L2-resident matrix as the sweep takes its op -- 7.0 instead of
// 12.3 KB of LDS per candidate at n = 1000, so more candidates stay resident.
#include "common.h"
#include "sweep.h"

namespace vrprpd {

struct EvalArgs {
    const InstDev* inst_tab;
    const void* dist;
    const int32_t* proc;
    const int32_t* inst;
    const int64_t* op_off;
    const uint16_t* ops;
    const int64_t* rt_off;
    const uint16_t* rt_end;
    int32_t* makespan;
    uint32_t* status;
    int64_t B;
    int32_t partial;
    int32_t nblocks;
    int32_t n_max;
    int32_t group_bytes;
    int32_t num_inst;
};

// LDS carve-up of one group, shared with the host-side size computation.
struct GroupLayout {
    int ready_off, bits_off, ops_off, bytes;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

constexpr int kStepOps = 8;   // most ops a lane may take per sweep step (LDS padding)

__host__ __device__ inline int op_capacity(int n_max) { return 2 * n_max + kStepOps; }

__host__ __device__ inline GroupLayout group_layout(int n_max, int bytes_per_op)
{
    GroupLayout g;
    g.ready_off = 0;
    g.bits_off = align16(4 * (n_max + 1));
    g.ops_off = g.bits_off + align16(4 * ((2 * (n_max + 1) + 31) / 32));
    g.bytes = g.ops_off + align16(bytes_per_op * op_capacity(n_max));
    return g;
}

// Stages op j of the candidate: marks its cover bit (a second copy of an op
// sets `dup`, a code outside [1, n] sets `bad`) and stores its code with the
// travel time from the previous op of the flat list (pc; route starts are
// re-pointed at the depot afterwards).  Branch-free so that many ops' LDS
// atomics and distance gathers issue back to back.
struct Staged {
    uint32_t cd;
    int idx;
};

// `live` false stages nothing (a clamped duplicate load): no cover bit, no flag.
__device__ __forceinline__ Staged stage_code(uint32_t* bits, uint32_t cd, uint32_t pc, int n, int N1, bool live,
                                            bool& bad)
{
    const int c = (int)(cd >> 1);
    const bool ok = c >= 1 && c <= n;
    const int bitpos = ok ? 2 * c + (int)(cd & 1u) : 0;
    const uint32_t mask = (ok && live) ? 1u << (bitpos & 31) : 0u;
    const uint32_t old = atomicOr(&bits[bitpos >> 5], mask);
    bad = bad || (live && (!ok || (old & mask)));
    int p = (int)(pc >> 1);
    p = p <= n ? p : 0;
    return Staged{ok ? cd : 0u, p * N1 + (ok ? c : 0)};
}

// One wave per block holding NG candidates (NG <= 64 / GL; lanes past NG
// groups stay idle, so that the LDS of NG groups lets more waves reside).
// kOneInst: every candidate uses instance 0 (no instance array), so the
// instance's distance and processing rows are wave-uniform (scalar bases).
template <typename DT, int GL, int NG, int K, bool kOneInst>
__global__ __launch_bounds__(64) void eval_kernel(EvalArgs a)
{
    static_assert(NG * GL <= 64, "groups per wave");
    static_assert(K <= kStepOps && K <= GL, "sweep step within the op padding");
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int grp = lane / GL, li = lane % GL;
    if (grp >= NG) return;
    const int blk = xcd_remap(blockIdx.x, a.nblocks);
    const int64_t b = (int64_t)blk * NG + grp;
    const bool live = b < a.B;

    const GroupLayout L = group_layout(a.n_max, OpStore<DT>::kBytesPerOp);
    unsigned char* gs = smem + (size_t)grp * a.group_bytes;
    int* ready = reinterpret_cast<int*>(gs + L.ready_off);
    uint32_t* bits = reinterpret_cast<uint32_t*>(gs + L.bits_off);
    OpStore<DT> S;
    S.init(gs + L.ops_off, op_capacity(a.n_max));

    int ii = (!kOneInst && live && a.inst) ? a.inst[b] : 0;
    const bool bad_inst = ii < 0 || ii >= a.num_inst;
    if (bad_inst) ii = 0;
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const int64_t ob = live ? (a.op_off ? a.op_off[b] : b * 2 * (int64_t)n) : 0;
    const int64_t rb = live ? (a.rt_off ? a.rt_off[b] : b * (int64_t)m) : 0;
    const uint16_t* ops = a.ops + ob;

    // Route bounds: lane v < m holds [s, e) of route v.
    int e = 0;
    if (live && !bad_inst && li < m) e = a.rt_end[rb + li];
    int s = __shfl_up(e, 1, GL);
    if (li == 0) s = 0;
    const int total = __shfl(e, m - 1, GL);
    bool bad = bad_inst || (live && li < m && s > e);
    if (total > 2 * n) bad = true;
    bool gbad = !live || group_ballot<GL>(bad) != 0;

    // ---- phase 1: stage ready[], the ops and every travel time -----------
    const int nwords = (2 * N1 + 31) / 32;
    for (int w = li; w < nwords; w += GL) bits[w] = 0u;
    wave_lds_fence();
    bool cbad = false;
    if (!gbad) {
        // ready[c] = ~p_c ("not dropped yet"; the drop reads p_c back from
        // it).  The p row is 16-byte aligned and padded: int4 loads, all of a
        // lane's in flight together (clamped, not predicated).
        {
            const int4* P4 = reinterpret_cast<const int4*>(P);
            int4* R4 = reinterpret_cast<int4*>(ready);
            const int np4 = (N1 + 3) >> 2;
            constexpr int VP = 8;
            for (int q0 = li; q0 < np4; q0 += VP * GL) {
                int4 x[VP];
#pragma unroll
                for (int v = 0; v < VP; ++v) {
                    const int q = q0 + v * GL;
                    x[v] = P4[q < np4 ? q : np4 - 1];
                }
#pragma unroll
                for (int v = 0; v < VP; ++v) {
                    const int q = q0 + v * GL;
                    if (q < np4) R4[q] = make_int4(~x[v].x, ~x[v].y, ~x[v].z, ~x[v].w);
                }
            }
        }
        // Ops: 16-byte vectors of 8 codes from HBM (plus the code before each
        // vector, an L1/L2 hit), then all their distance gathers at once.
        int head = (int)((8 - (((uintptr_t)ops >> 1) & 7)) & 7);
        head = head < total ? head : total;
        const int nvec = (total - head) >> 3;
        const int tail0 = head + 8 * nvec;
        const int nscalar = head + (total - tail0);
        for (int t = li; t < nscalar; t += GL) {
            const int j = t < head ? t : tail0 + (t - head);
            const uint32_t cd = ops[j];
            const uint32_t pt = ops[j > 0 ? j - 1 : 0];
            const Staged g = stage_code(bits, cd, j > 0 ? pt : 0u, n, N1, true, cbad);
            S.set(j, g.cd, (int)ld_elem(D, g.idx));
        }
        const uint4* vec = reinterpret_cast<const uint4*>(ops + head);
        constexpr int V = 4;   // vectors per lane per batch: 32 gathers in flight
        for (int q0 = li; q0 < nvec; q0 += V * GL) {
            uint4 x[V];
            uint32_t pv[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                int q = q0 + v * GL;
                q = q < nvec ? q : nvec - 1;
                x[v] = vec[q];
                const int j = head + 8 * q;
                const uint32_t pt = ops[j > 0 ? j - 1 : 0];
                pv[v] = j > 0 ? pt : 0u;
            }
            int idx[V][8];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int q = q0 + v * GL;
                const bool in = q < nvec;
                const uint32_t w4[4] = {x[v].x, x[v].y, x[v].z, x[v].w};
                uint32_t prev = pv[v];
#pragma unroll
                for (int h = 0; h < 8; ++h) {
                    const uint32_t cd = (w4[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
                    const Staged g = stage_code(bits, cd, prev, n, N1, in, cbad);
                    if (in) S.put_code(head + 8 * q + h, g.cd);
                    idx[v][h] = g.idx;
                    prev = cd;
                }
            }
            int lg[V][8];
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int h = 0; h < 8; ++h) lg[v][h] = (int)ld_elem(D, idx[v][h]);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int q = q0 + v * GL;
                if (q < nvec) {
                    const int j = head + 8 * q;
#pragma unroll
                    for (int h = 0; h < 8; ++h) S.put_leg(j + h, lg[v][h]);
                }
            }
        }
    }
    // padding past the last route: the sweep reads ready[] for its next K ops
    // without testing the route's end
    if (!gbad && li < K) S.set(total + li, 0u, 0);
    wave_lds_fence();
    if (!gbad) {
        for (int c = 1 + li; c <= n; c += GL) {
            const uint32_t two = (bits[(2 * c) >> 5] >> ((2 * c) & 31)) & 3u;
            if (!(two == 3u || (two == 0u && a.partial))) cbad = true;
        }
        // the first op of each route comes from the depot
        if (li < m && s < e) S.set_leg(s, (int)D[(int)(S.code(s) >> 1)]);
    }
    wave_lds_fence();
    gbad = gbad || group_ballot<GL>(cbad) != 0;

    // ---- phase 2: timing sweep ----------------------------------------------
    const bool veh = li < m;
    SweepOut o{0, 0, 0, 0, false};
    if (!gbad) o = sweep_group<GL, K, DT>(S, ready, veh ? s : 0, veh ? e : 0);

    uint32_t st = 0;
    int z = 0;
    if (!gbad) {
        st = load_status<GL>(o, veh, m, I.k, I.R, I.load_model);
        int ret = 0;
        if (veh && e > s) ret = o.t + (int)D[(int64_t)(S.code(e - 1) >> 1) * N1];
        z = group_max<GL>(ret);
        if (o.dead) st |= VRPRPD_ST_DEADLOCK;
    }
    if (live && li == 0) {
        if (gbad) {
            a.makespan[b] = INT32_MAX;
            a.status[b] = VRPRPD_ST_BAD_COVER;
        } else {
            a.makespan[b] = o.dead ? INT32_MAX : z;
            a.status[b] = st;
        }
    }
}

// ---------------------------------------------------------------------------
// Live-leg form: phase 1 stages only the op codes and the cover bits; the
// sweep gathers each op's travel time d[prev][c] from the L2 in the same
// round trip as its ready[] read.  The cover bits share ready[]'s space (the
// cover check is done before ready[] is written), and when every code fits
// 12 bits (n < 2048) the codes are packed 12 bits each: 7.0 KB of LDS per
// candidate at n = 1000 (12.3 KB staged), which is what sets how many
// candidates stay resident.

constexpr int kC12MaxN = 2047;   // codes (c << 1 | isP) below 4096

__host__ __device__ inline int live_code_entries(int n_max) { return 2 * n_max + kStepOps + 8; }

__host__ __device__ inline GroupLayout live_layout(int n_max, bool c12)
{
    GroupLayout g;
    g.ready_off = 0;
    g.bits_off = 0;
    g.ops_off = align16(4 * (n_max + 1));
    // 12-bit codes: a read of up to four codes from position p <= 2n + 6
    // (the last op, shifted by up to 7) takes the words up to
    // 12 (p + 2) / 32 + 1, and the writes stay below that
    g.bytes = g.ops_off + (c12 ? align16(4 * ((12 * (2 * n_max + 8)) / 32 + 2))
                               : align16(2 * live_code_entries(n_max)));
    return g;
}

// Op codes of one candidate in LDS, entry j at position j + sh (sh aligns
// the vector stores of phase 1).
template <bool kC12>
struct LiveCodes;

template <>
struct LiveCodes<false> {
    uint16_t* c;
    __device__ __forceinline__ void init(unsigned char* base, int sh) { c = reinterpret_cast<uint16_t*>(base) + sh; }
    __device__ __forceinline__ uint32_t get(int j) const { return c[j]; }
    template <int K>
    __device__ __forceinline__ void get_k(int j, uint32_t* cd) const
    {
#pragma unroll
        for (int u = 0; u < K; ++u) cd[u] = c[j + u];
    }
    __device__ __forceinline__ void put(int j, uint32_t cd) { c[j] = (uint16_t)cd; }
    // eight codes at j (j + sh a multiple of 8): 16-byte store
    __device__ __forceinline__ void put8(int j, const uint32_t* cd)
    {
        *reinterpret_cast<uint4*>(c + j) = make_uint4(cd[0] | cd[1] << 16, cd[2] | cd[3] << 16, cd[4] | cd[5] << 16,
                                                      cd[6] | cd[7] << 16);
    }
};

template <>
struct LiveCodes<true> {
    uint32_t* w;
    int sh;
    __device__ __forceinline__ void init(unsigned char* base, int s) { w = reinterpret_cast<uint32_t*>(base); sh = s; }
    // the 32 bits from bit b of the packed array
    __device__ __forceinline__ uint32_t bits_at(int b) const
    {
        const uint32_t lo = w[b >> 5], hi = w[(b >> 5) + 1];
        return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(b & 31));
    }
    __device__ __forceinline__ uint32_t get(int j) const { return bits_at(12 * (j + sh)) & 0xFFFu; }
    template <int K>
    __device__ __forceinline__ void get_k(int j, uint32_t* cd) const
    {
        static_assert(K == 2 || K == 4, "two or four codes per read");
        const int b = 12 * (j + sh);
        const uint32_t y0 = bits_at(b);
        cd[0] = y0 & 0xFFFu;
        cd[1] = (y0 >> 12) & 0xFFFu;
        if constexpr (K == 4) {
            const uint32_t y1 = bits_at(b + 24);
            cd[2] = y1 & 0xFFFu;
            cd[3] = (y1 >> 12) & 0xFFFu;
        }
    }
    // one code into a cleared field (it may straddle two words)
    __device__ __forceinline__ void put(int j, uint32_t cd)
    {
        const int b = 12 * (j + sh), o = b & 31;
        atomicOr(&w[b >> 5], cd << o);
        if (o > 20) atomicOr(&w[(b >> 5) + 1], cd >> (32 - o));
    }
    // eight codes at j (j + sh a multiple of 8): three whole words
    __device__ __forceinline__ void put8(int j, const uint32_t* cd)
    {
        uint32_t* q = w + 3 * ((j + sh) >> 3);
        q[0] = cd[0] | cd[1] << 12 | cd[2] << 24;
        q[1] = cd[2] >> 8 | cd[3] << 4 | cd[4] << 16 | cd[5] << 28;
        q[2] = cd[5] >> 4 | cd[6] << 8 | cd[7] << 20;
    }
};

// Cover bit of one code; returns the code, or 0 for a code outside [1, n].
__device__ __forceinline__ uint32_t cover_code(uint32_t* bits, uint32_t cd, int n, bool live, bool& bad)
{
    const int c = (int)(cd >> 1);
    const bool ok = c >= 1 && c <= n;
    const int bitpos = ok ? 2 * c + (int)(cd & 1u) : 0;
    const uint32_t mask = (ok && live) ? 1u << (bitpos & 31) : 0u;
    const uint32_t old = atomicOr(&bits[bitpos >> 5], mask);
    bad = bad || (live && (!ok || (old & mask)));
    return ok ? cd : 0u;
}

// Travel time at a 32-bit byte offset from the uniform matrix base.
template <typename DT>
__device__ __forceinline__ int leg_at(const DT* D, uint32_t entry)
{
    return (int)*reinterpret_cast<const DT*>(reinterpret_cast<const unsigned char*>(D) + entry * (uint32_t)sizeof(DT));
}

// The lockstep sweep of sweep_group with the travel times read from the
// matrix as the ops are taken: lane v keeps the matrix row of its route's
// last stop (the depot's at the start) for the next op's leg, so a step
// reads its K codes from LDS, then their ready[] entries (LDS) and legs (L2)
// together.  The code store holds valid codes (0) for K entries past the
// last route.
template <int GL, int K, typename DT, typename Codes>
__device__ __forceinline__ SweepOut sweep_live(const Codes& C, const DT* D, uint32_t N1, int* ready, int s, int e)
{
    SweepOut o{0, 0, 0, 0, false};
    int ptr = s;
    uint32_t prow = 0;
    for (;;) {
        int took = 0;
        if (ptr < e) {
            uint32_t cd[K], row[K];
            int leg[K], r[K];
            C.template get_k<K>(ptr, cd);
#pragma unroll
            for (int u = 0; u < K; ++u) {
                // codes are 16-bit, so customers and n + 1 are below 2^16
                // and the 24-bit multiply is exact
                row[u] = __umul24(cd[u] >> 1, N1);
                leg[u] = leg_at(D, (u == 0 ? prow : row[u > 0 ? u - 1 : 0]) + (cd[u] >> 1));
            }
#pragma unroll
            for (int u = 0; u < K; ++u) r[u] = lds_load(&ready[cd[u] >> 1]);
            took = sweep_step<K, false>(o, cd, leg, r, e - ptr, ready, nullptr, 0);
#pragma unroll
            for (int u = 0; u < K; ++u) prow = took == u + 1 ? row[u] : prow;
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
        o.w += (C.get(ptr) & 1u) ? -1 : 1;
        o.wmax = o.w > o.wmax ? o.w : o.wmax;
        o.wmin = o.w < o.wmin ? o.w : o.wmin;
    }
    return o;
}

template <typename DT, int GL, int NG, int K, bool kOneInst, bool kC12>
__global__ __launch_bounds__(64) void eval_live_kernel(EvalArgs a)
{
    static_assert(NG * GL <= 64, "groups per wave");
    static_assert(K <= kStepOps && K <= GL, "sweep step within the op padding");
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int grp = lane / GL, li = lane % GL;
    if (grp >= NG) return;
    const int blk = xcd_remap(blockIdx.x, a.nblocks);
    const int64_t b = (int64_t)blk * NG + grp;
    const bool live = b < a.B;

    const GroupLayout L = live_layout(a.n_max, kC12);
    unsigned char* gs = smem + (size_t)grp * a.group_bytes;
    int* ready = reinterpret_cast<int*>(gs + L.ready_off);
    uint32_t* bits = reinterpret_cast<uint32_t*>(gs + L.bits_off);

    int ii = (!kOneInst && live && a.inst) ? a.inst[b] : 0;
    const bool bad_inst = ii < 0 || ii >= a.num_inst;
    if (bad_inst) ii = 0;
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const int64_t ob = live ? (a.op_off ? a.op_off[b] : b * 2 * (int64_t)n) : 0;
    const int64_t rb = live ? (a.rt_off ? a.rt_off[b] : b * (int64_t)m) : 0;
    const uint16_t* ops = a.ops + ob;

    int e = 0;
    if (live && !bad_inst && li < m) e = a.rt_end[rb + li];
    int s = __shfl_up(e, 1, GL);
    if (li == 0) s = 0;
    const int total = __shfl(e, m - 1, GL);
    bool bad = bad_inst || (live && li < m && s > e);
    if (total > 2 * n) bad = true;
    bool gbad = !live || group_ballot<GL>(bad) != 0;

    // op j at position j + sh, so that the vector stores from `head` on align
    int head = (int)((8 - (((uintptr_t)ops >> 1) & 7)) & 7);
    head = head < total ? head : total;
    LiveCodes<kC12> C;
    C.init(gs + L.ops_off, (8 - head) & 7);

    // ---- phase 1: cover bits and op codes, then ready[] ----------------------
    const int nwords = (2 * N1 + 31) / 32;
    for (int w = li; w < nwords; w += GL) bits[w] = 0u;
    if constexpr (kC12) {   // the packed fields are or-ed into cleared words
        uint4* z = reinterpret_cast<uint4*>(gs + L.ops_off);
        const int nz = (L.bytes - L.ops_off) >> 4;
        for (int q = li; q < nz; q += GL) z[q] = make_uint4(0u, 0u, 0u, 0u);
    }
    wave_lds_fence();
    bool cbad = false;
    if (!gbad) {
        const int nvec = (total - head) >> 3;
        const int tail0 = head + 8 * nvec;
        const int nscalar = head + (total - tail0);
        for (int t = li; t < nscalar; t += GL) {
            const int j = t < head ? t : tail0 + (t - head);
            C.put(j, cover_code(bits, ops[j], n, true, cbad));
        }
        const uint4* vec = reinterpret_cast<const uint4*>(ops + head);
        constexpr int V = 8;
        for (int q0 = li; q0 < nvec; q0 += V * GL) {
            uint4 x[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int q = q0 + v * GL;
                x[v] = vec[q < nvec ? q : nvec - 1];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int q = q0 + v * GL;
                const bool in = q < nvec;
                const uint32_t w4[4] = {x[v].x, x[v].y, x[v].z, x[v].w};
                uint32_t cd[8];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    cd[2 * h] = cover_code(bits, w4[h] & 0xFFFFu, n, in, cbad);
                    cd[2 * h + 1] = cover_code(bits, w4[h] >> 16, n, in, cbad);
                }
                if (in) C.put8(head + 8 * q, cd);
            }
        }
    }
    // padding past the last route: the sweep reads its next K codes without
    // testing the route's end (the packed store was cleared)
    if constexpr (!kC12) {
        if (!gbad && li < K) C.put(total + li, 0u);
    }
    wave_lds_fence();
    if (!gbad) {
        for (int c = 1 + li; c <= n; c += GL) {
            const uint32_t two = (bits[(2 * c) >> 5] >> ((2 * c) & 31)) & 3u;
            if (!(two == 3u || (two == 0u && a.partial))) cbad = true;
        }
    }
    gbad = gbad || group_ballot<GL>(cbad) != 0;
    wave_lds_fence();
    // ready[c] = ~p_c ("not dropped yet"; the drop reads p_c back from it),
    // over the cover bits.  The p row is 16-byte aligned and padded: int4
    // loads, all of a lane's in flight together.
    if (!gbad) {
        const int4* P4 = reinterpret_cast<const int4*>(P);
        int4* R4 = reinterpret_cast<int4*>(ready);
        const int np4 = (N1 + 3) >> 2;
        constexpr int VP = 8;
        for (int q0 = li; q0 < np4; q0 += VP * GL) {
            int4 x[VP];
#pragma unroll
            for (int v = 0; v < VP; ++v) {
                const int q = q0 + v * GL;
                x[v] = P4[q < np4 ? q : np4 - 1];
            }
#pragma unroll
            for (int v = 0; v < VP; ++v) {
                const int q = q0 + v * GL;
                if (q < np4) R4[q] = make_int4(~x[v].x, ~x[v].y, ~x[v].z, ~x[v].w);
            }
        }
    }
    wave_lds_fence();

    // ---- phase 2: timing sweep ----------------------------------------------
    const bool veh = li < m;
    SweepOut o{0, 0, 0, 0, false};
    if (!gbad) o = sweep_live<GL, K, DT>(C, D, (uint32_t)N1, ready, veh ? s : 0, veh ? e : 0);

    uint32_t st = 0;
    int z = 0;
    if (!gbad) {
        st = load_status<GL>(o, veh, m, I.k, I.R, I.load_model);
        int ret = 0;
        if (veh && e > s) ret = o.t + (int)D[(int64_t)(C.get(e - 1) >> 1) * N1];
        z = group_max<GL>(ret);
        if (o.dead) st |= VRPRPD_ST_DEADLOCK;
    }
    if (live && li == 0) {
        if (gbad) {
            a.makespan[b] = INT32_MAX;
            a.status[b] = VRPRPD_ST_BAD_COVER;
        } else {
            a.makespan[b] = o.dead ? INT32_MAX : z;
            a.status[b] = st;
        }
    }
}

constexpr int kEvalStep = 4;   // default ops per lane per sweep step

struct LaunchShape {
    int gl, ng, group_bytes, lds, step, live;
};

static int group_bytes_of(int n_max, int dist16, int live)
{
    if (live) return live_layout(n_max, n_max <= kC12MaxN).bytes;
    return group_layout(n_max, dist16 ? OpStore<uint16_t>::kBytesPerOp : OpStore<int32_t>::kBytesPerOp).bytes;
}

// Default form without tuning: live legs once the staged layout (ops, legs
// and ready[] of a candidate) outgrows 8 KB of LDS, about n > 650 with
// 16-bit travel times: below that both forms keep enough waves resident and
// the staged form's sweep reads only LDS.
static int default_live(int n_max, int dist16) { return group_bytes_of(n_max, dist16, 0) > 8 * 1024 ? 1 : 0; }

// Candidates per wave tried for a group width: 16 lanes -> 2, 3, 4; 32 -> 1, 2; 64 -> 1.
static int ng_options(int gl, int* out)
{
    if (gl == 16) { out[0] = 2; out[1] = 3; out[2] = 4; return 3; }
    if (gl == 32) { out[0] = 1; out[1] = 2; return 2; }
    out[0] = 1;
    return 1;
}

// Default: the most candidates per wave that still leave LDS room for two
// waves per SIMD (8 per CU: the sweep is latency-bound and needs a second
// wave to hide it), else the fewest.
static int default_ng(int gl, int gb)
{
    int opts[3];
    const int k = ng_options(gl, opts);
    int best = opts[0];
    for (int i = 0; i < k; ++i)
        if ((size_t)opts[i] * gb * 8 <= kLdsPerCu) best = opts[i];
    return best;
}

static LaunchShape eval_shape(int n_max, int m_max, int dist16, int ng, int step, int live)
{
    LaunchShape sh;
    sh.gl = m_max <= 16 ? 16 : (m_max <= 32 ? 32 : 64);
    sh.live = live >= 0 ? live : default_live(n_max, dist16);
    sh.group_bytes = group_bytes_of(n_max, dist16, sh.live);
    sh.ng = ng > 0 ? ng : default_ng(sh.gl, sh.group_bytes);
    sh.lds = sh.ng * sh.group_bytes;
    sh.step = step > 0 ? step : kEvalStep;
    return sh;
}

template <typename DT, int GL, int NG, int K>
static int launch_eval(const EvalArgs& a, int lds, int live, hipStream_t stream)
{
    const bool c12 = a.n_max <= kC12MaxN;
    auto* k = live ? (a.inst ? (c12 ? eval_live_kernel<DT, GL, NG, K, false, true>
                                    : eval_live_kernel<DT, GL, NG, K, false, false>)
                             : (c12 ? eval_live_kernel<DT, GL, NG, K, true, true>
                                    : eval_live_kernel<DT, GL, NG, K, true, false>))
                   : (a.inst ? eval_kernel<DT, GL, NG, K, false> : eval_kernel<DT, GL, NG, K, true>);
    if (lds > 64 * 1024)
        VRP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    hipLaunchKernelGGL(k, dim3(a.nblocks), dim3(64), lds, stream, a);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

template <typename DT, int GL, int NG>
static int dispatch_step(const EvalArgs& a, const LaunchShape& sh, hipStream_t st)
{
    return sh.step == 2 ? launch_eval<DT, GL, NG, 2>(a, sh.lds, sh.live, st)
                        : launch_eval<DT, GL, NG, 4>(a, sh.lds, sh.live, st);
}

template <typename DT>
static int dispatch_gl(const EvalArgs& a, const LaunchShape& sh, hipStream_t st)
{
    if (sh.gl == 16) {
        switch (sh.ng) {
        case 2: return dispatch_step<DT, 16, 2>(a, sh, st);
        case 3: return dispatch_step<DT, 16, 3>(a, sh, st);
        default: return dispatch_step<DT, 16, 4>(a, sh, st);
        }
    }
    if (sh.gl == 32) {
        if (sh.ng == 1) return dispatch_step<DT, 32, 1>(a, sh, st);
        return dispatch_step<DT, 32, 2>(a, sh, st);
    }
    return dispatch_step<DT, 64, 1>(a, sh, st);
}

// Validates the arguments and launches one shape (ng, step <= 0: default).
static int eval_launch(const vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                       const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t flags,
                       int32_t* makespan, uint32_t* status, hipStream_t st, int ng, int step, int live)
{
    if (!set) return set_error(VRPRPD_EINVAL, "vrprpd_eval: set is NULL");
    if (B < 0) return set_error(VRPRPD_EINVAL, "vrprpd_eval: B < 0");
    if (flags & ~VRPRPD_ALLOW_PARTIAL) return set_error(VRPRPD_EINVAL, "vrprpd_eval: unknown flags 0x%x", flags);
    if (B == 0) return VRPRPD_OK;
    if (!ops || !rt_end || !makespan || !status)
        return set_error(VRPRPD_EINVAL, "vrprpd_eval: ops, rt_end, makespan and status are required");
    if (inst && (!op_off || !rt_off) && !set->uniform_nm)
        return set_error(VRPRPD_EINVAL, "vrprpd_eval: instances differ in n or m; pass op_off and rt_off");
    const int n_lds = inst ? set->n_max : set->host[0].n;
    const int m_max = inst ? set->m_max : set->host[0].m;
    if (ng <= 0 && step <= 0 && live < 0) {
        const auto it = set->eval_tuned.find({n_lds, m_max});
        if (it != set->eval_tuned.end()) std::tie(ng, step, live) = it->second;
    }
    const LaunchShape sh = eval_shape(n_lds, m_max, set->dist16, ng, step, live);
    if ((size_t)sh.lds > kLdsPerCu)
        return set_error(VRPRPD_EINVAL, "vrprpd_eval: n=%d needs %d B of LDS per candidate", n_lds, sh.lds);
    const int64_t per_block = sh.ng;
    const int64_t nb = (B + per_block - 1) / per_block;
    if (nb > INT32_MAX) return set_error(VRPRPD_EINVAL, "vrprpd_eval: B too large");
    EvalArgs a{set->d_inst, set->d_dist, set->d_proc, inst, op_off, ops, rt_off, rt_end, makespan, status,
               B, (flags & VRPRPD_ALLOW_PARTIAL) ? 1 : 0, (int32_t)nb, n_lds, sh.group_bytes,
               set->num_inst};
    return set->dist16 ? dispatch_gl<uint16_t>(a, sh, st) : dispatch_gl<int32_t>(a, sh, st);
}

// Random reads of one instance's travel-time matrix: thread t makes `per`
// reads at uniformly distributed entries (a multiplicative hash of (t, i),
// scaled into [0, (n+1)^2)), 16 in flight per thread, and adds them up; the
// block's sum is written so that no read is dropped.
template <typename DT>
__global__ __launch_bounds__(256) void gather_rate_kernel(const DT* D, uint32_t entries, int per, int32_t* sink)
{
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    uint32_t acc = 0;
    for (int i0 = 0; i0 < per; i0 += 16) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint32_t x = t * 0x9E3779B1u + (uint32_t)(i0 + u) * 0x85EBCA77u;
            x ^= x >> 15;
            x *= 0x2C1B3C6Du;
            x ^= x >> 12;
            const uint32_t idx = (uint32_t)(((uint64_t)x * entries) >> 32);
            v[u] = (uint32_t)D[idx];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = (int32_t)red[0];
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" int vrprpd_eval(const vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                           const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t flags,
                           int32_t* makespan, uint32_t* status, void* stream)
{
    return eval_launch(set, B, inst, op_off, ops, rt_off, rt_end, flags, makespan, status,
                       reinterpret_cast<hipStream_t>(stream), 0, 0, -1);
}

extern "C" int vrprpd_autotune_eval(vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                                    const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end, int32_t flags,
                                    int32_t* makespan, uint32_t* status, int32_t reps, int32_t* ng_out,
                                    int32_t* step_out, float* ms_out, void* stream)
{
    if (!set || B < 1 || reps < 1 || !makespan || !status)
        return set_error(VRPRPD_EINVAL, "vrprpd_autotune_eval: need a set, B >= 1, reps >= 1 and outputs");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n_lds = inst ? set->n_max : set->host[0].n;
    const int m_max = inst ? set->m_max : set->host[0].m;
    const int gl = m_max <= 16 ? 16 : (m_max <= 32 ? 32 : 64);
    // reference outputs of the default shape, kept on the host
    int rc = eval_launch(set, B, inst, op_off, ops, rt_off, rt_end, flags, makespan, status, st, -1, kEvalStep, -1);
    if (rc) return rc;
    std::vector<int32_t> mk0(B), mk1(B);
    std::vector<uint32_t> st0(B), st1(B);
    VRP_HIP(hipStreamSynchronize(st));
    VRP_HIP(hipMemcpy(mk0.data(), makespan, B * 4, hipMemcpyDeviceToHost));
    VRP_HIP(hipMemcpy(st0.data(), status, B * 4, hipMemcpyDeviceToHost));
    hipEvent_t e0, e1;
    VRP_HIP(hipEventCreate(&e0));
    VRP_HIP(hipEventCreate(&e1));
    float best = 0.f;
    const int live0 = default_live(n_lds, set->dist16);
    int bw = default_ng(gl, group_bytes_of(n_lds, set->dist16, live0)), bs = kEvalStep, bl = live0, v = 0;
    int ngs[3];
    const int nng = ng_options(gl, ngs);
    const int steps[2] = {2, 4};
    for (int lv = 0; lv < 2; ++lv) {
        const int gb = group_bytes_of(n_lds, set->dist16, lv);
        for (int wi = 0; wi < 3; ++wi) {
            for (int si = 0; si < 2; ++si, ++v) {
                float ms = -1.f;
                const int w = wi < nng ? ngs[wi] : 0;
                const int k = steps[si];
                if (w > 0 && (size_t)w * gb <= kLdsPerCu) {
                    auto run = [&]() {
                        return eval_launch(set, B, inst, op_off, ops, rt_off, rt_end, flags, makespan, status, st,
                                           w, k, lv);
                    };
                    rc = run();
                    if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = set_error(VRPRPD_EHIP, "event");
                    for (int r = 0; r < reps && !rc; ++r) rc = run();
                    if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                        rc = set_error(VRPRPD_EHIP, "vrprpd_autotune_eval: timing failed");
                    if (!rc && (hipMemcpy(mk1.data(), makespan, B * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                                hipMemcpy(st1.data(), status, B * 4, hipMemcpyDeviceToHost) != hipSuccess))
                        rc = set_error(VRPRPD_EHIP, "vrprpd_autotune_eval: copy failed");
                    if (!rc && (mk1 != mk0 || st1 != st0))
                        rc = set_error(VRPRPD_EHIP, "vrprpd_autotune_eval: shape (%s, %d candidates per wave, "
                                                    "step %d) disagrees with the default shape",
                                       lv ? "live legs" : "staged legs", w, k);
                    if (rc) {
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                        return rc;
                    }
                    ms /= (float)reps;
                    if (best == 0.f || ms < best) {
                        best = ms;
                        bw = w;
                        bs = k;
                        bl = lv;
                    }
                }
                if (ms_out) ms_out[v] = ms;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set->eval_tuned[{n_lds, m_max}] = {bw, bs, bl};
    if (ng_out) *ng_out = bw;
    if (step_out) *step_out = bs;
    return VRPRPD_OK;
}

extern "C" int vrprpd_eval_set_shape(vrprpd_set* set, int32_t n, int32_t m, int32_t ng, int32_t step, int32_t live)
{
    if (!set || n < 1 || m < 1 || (step != 2 && step != 4) || (live != 0 && live != 1) || ng < 0)
        return set_error(VRPRPD_EINVAL, "vrprpd_eval_set_shape: need a set, n >= 1, m >= 1, step 2 or 4, "
                                        "live 0 or 1 and ng >= 0");
    const int gl = m <= 16 ? 16 : (m <= 32 ? 32 : 64);
    int opts[3];
    const int k = ng_options(gl, opts);
    const int gb = group_bytes_of(n, set->dist16, live);
    if (ng == 0) ng = default_ng(gl, gb);
    bool ok = false;
    for (int i = 0; i < k; ++i) ok = ok || opts[i] == ng;
    if (!ok) return set_error(VRPRPD_EINVAL, "vrprpd_eval_set_shape: %d candidates per wave is not an option for m=%d",
                              ng, m);
    if ((size_t)ng * gb > kLdsPerCu)
        return set_error(VRPRPD_EINVAL, "vrprpd_eval_set_shape: %d candidates per wave need %d B of LDS", ng, ng * gb);
    set->eval_tuned[{n, m}] = {ng, step, live};
    return VRPRPD_OK;
}

extern "C" int vrprpd_gather_rate(const vrprpd_set* set, int32_t inst, int32_t blocks, int32_t per_thread,
                                  int32_t* sink, float* ms_out, void* stream)
{
    if (!set || inst < 0 || inst >= set->num_inst || blocks < 1 || per_thread < 16 || per_thread % 16 || !sink ||
        !ms_out)
        return set_error(VRPRPD_EINVAL, "vrprpd_gather_rate: need a set, an instance index, blocks >= 1, "
                                        "per_thread a positive multiple of 16, sink and ms_out");
    const InstDev& h = set->host[inst];
    const uint32_t entries = (uint32_t)((h.n + 1) * (int64_t)(h.n + 1));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    VRP_HIP(hipEventCreate(&e0));
    VRP_HIP(hipEventCreate(&e1));
    auto launch = [&]() {
        if (set->dist16)
            hipLaunchKernelGGL(gather_rate_kernel<uint16_t>, dim3(blocks), dim3(256), 0, st,
                               static_cast<const uint16_t*>(set->d_dist) + h.d_off, entries, per_thread, sink);
        else
            hipLaunchKernelGGL(gather_rate_kernel<int32_t>, dim3(blocks), dim3(256), 0, st,
                               static_cast<const int32_t*>(set->d_dist) + h.d_off, entries, per_thread, sink);
    };
    launch();   // warm the matrix into the caches
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_error(e, "vrprpd_gather_rate");
    return VRPRPD_OK;
}
