// vrprpd_insert_scan: exact makespan of insertion tuples (Section 4.2.3).
//
// Mapping: one block per segment.  The block stages its base solution once
// (op codes and every travel time into LDS, shared by all its groups), then
// each group of GL lanes evaluates the segment's tuples one after another:
// lane v walks route v of the base with the tuple's drop and pickup spliced
// in ("virtual route"), so a tuple costs four travel-time gathers and a sweep
// over LDS, never a copy of the solution.
//
// ready[] per group is not re-initialised between tuples.  Its sign convention
// flips every tuple: after a completed sweep every customer of the solution
// has been dropped, so all entries read as "not dropped yet" under the next
// tuple's convention.  Only the inserted customer's entry (and, after a
// deadlock, every entry) is reset explicitly.
#include "common.h"
#include "sweep.h"
#include "scan.h"

namespace vrprpd {



constexpr int kScanStep = 4;

struct ScanLayout {
    int p_off, bits_off, route_off, ops_off, top_off, ready_off, ready_bytes, bytes;
};

__host__ __device__ inline int a16(int x) { return (x + 15) & ~15; }

template <int WPB, int GL>
__host__ __device__ inline ScanLayout scan_layout(int n_max, int bytes_per_op)
{
    constexpr int G = 64 / GL;
    ScanLayout L;
    L.p_off = 0;
    L.bits_off = a16(4 * (n_max + 1));
    L.route_off = L.bits_off + a16(4 * ((2 * (n_max + 1) + 31) / 32));
    L.ops_off = L.route_off + a16(4 * 3 * kMaxM);                   // s, e, return leg per route
    L.top_off = L.ops_off + a16(bytes_per_op * (2 * n_max + kScanStep));
    L.ready_off = L.top_off + a16(8 * 3 * WPB * G);
    L.ready_bytes = a16(4 * (n_max + 1));
    L.bytes = L.ready_off + L.ready_bytes * WPB * G;
    return L;
}

__device__ __forceinline__ void top3_insert(long long* t, long long key)
{
    if (key < t[2]) {
        t[2] = key;
        if (t[2] < t[1]) { long long x = t[1]; t[1] = t[2]; t[2] = x; }
        if (t[1] < t[0]) { long long x = t[0]; t[0] = t[1]; t[1] = x; }
    }
}

template <typename DT, int GL, int WPB>
__global__ __launch_bounds__(64 * WPB) void scan_kernel(ScanArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int G = 64 / GL;
    constexpr int NT = 64 * WPB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane / GL, li = lane % GL, gidx = wave * G + grp;
    const int seg = a.seg_active > 0 ? (int)(blockIdx.x / a.seg_active) * a.seg_stride + (int)(blockIdx.x % a.seg_active)
                                     : (int)blockIdx.x;
    const int ychunk = blockIdx.y, ny = gridDim.y;   // blocks sharing the segment
    const ScanLayout L = scan_layout<WPB, GL>(a.n_max, OpStore<DT>::kBytesPerOp);
    int* pblk = reinterpret_cast<int*>(smem + L.p_off);
    uint32_t* bits = reinterpret_cast<uint32_t*>(smem + L.bits_off);
    int* rs_ = reinterpret_cast<int*>(smem + L.route_off);
    int* re_ = rs_ + kMaxM;
    int* rret = re_ + kMaxM;
    long long* topbuf = reinterpret_cast<long long*>(smem + L.top_off);
    int* ready = reinterpret_cast<int*>(smem + L.ready_off + gidx * L.ready_bytes);
    OpStore<DT> S;
    S.init(smem + L.ops_off, 2 * a.n_max + kScanStep);
    // [0] base breaks cover rules, [1] segment's base/instance index out of
    // range, [2] base route-end table invalid
    __shared__ int flags[3];

    const int64_t t0 = a.seg_off[seg];
    const int64_t t1 = a.seg_cnt ? t0 + a.seg_cnt[seg] : a.seg_off[seg + 1];
    if (t1 <= t0 + (int64_t)ychunk * WPB * G) return;   // nothing for this block: skip the staging
    int bi = a.seg_base ? a.seg_base[seg] : 0;
    const bool bad_base_idx = bi < 0 || bi >= a.num_bases;
    if (bad_base_idx) bi = 0;
    int ii = a.base_inst ? a.base_inst[bi] : 0;
    const bool bad_inst = ii < 0 || ii >= a.num_inst;
    if (bad_inst) ii = 0;
    const bool seg_bad = bad_base_idx || bad_inst;
    const InstDev I = a.inst_tab[ii];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const uint16_t* bops = a.base_ops + (a.base_op_off ? a.base_op_off[bi] : (int64_t)bi * 2 * n);
    const uint16_t* brt = a.base_rt_end + (a.base_rt_off ? a.base_rt_off[bi] : (int64_t)bi * m);

    // ---- stage the base -------------------------------------------------------
    if (tid < 3) flags[tid] = (tid == 1 && seg_bad) ? 1 : 0;
    const int nwords = (2 * N1 + 31) / 32;
    for (int w = tid; w < nwords; w += NT) bits[w] = 0u;
    for (int c = tid; c <= n; c += NT) pblk[c] = c ? P[c] : 0;
    __syncthreads();
    if (!seg_bad && tid < m) {
        const int e = brt[tid];
        const int s = tid ? brt[tid - 1] : 0;
        rs_[tid] = s;
        re_[tid] = e;
        if (s > e || (tid == m - 1 && e > 2 * n)) flags[2] = 1;
    }
    __syncthreads();
    const bool rt_bad = flags[2] != 0;
    const int total = (rt_bad || seg_bad) ? 0 : re_[m - 1];
    for (int j = tid; j < total; j += NT) {
        uint32_t cd = bops[j];
        const int c = (int)(cd >> 1);
        if (c < 1 || c > n) {
            flags[0] = 1;
            cd = 0;
        } else {
            const int bitpos = 2 * c + (int)(cd & 1u);
            const uint32_t mask = 1u << (bitpos & 31);
            if (atomicOr(&bits[bitpos >> 5], mask) & mask) flags[0] = 1;
        }
        S.set_code(j, cd);
    }
    // padding past the last route for the sweep's unguarded fetches
    for (int j = total + tid; j < total + kScanStep; j += NT) S.set(j, 0u, 0);
    __syncthreads();
    if (!rt_bad && !seg_bad) {
        for (int c = 1 + tid; c <= n; c += NT) {
            const uint32_t two = (bits[(2 * c) >> 5] >> ((2 * c) & 31)) & 3u;
            if (two == 1u || two == 2u) flags[0] = 1;
        }
    }
    __syncthreads();
    const bool base_bad = flags[0] != 0 || rt_bad;
    if (!base_bad && !seg_bad) {
        for (int j = tid; j < total; j += NT) {
            const int c = (int)(S.code(j) >> 1);
            const int pc = j > 0 ? (int)(S.code(j - 1) >> 1) : 0;
            S.set_leg(j, (int)D[pc * N1 + c]);
        }
        __syncthreads();
        if (tid < m) {
            const int s = rs_[tid], e = re_[tid];
            if (s < e) {
                S.set_leg(s, (int)D[(int)(S.code(s) >> 1)]);
                rret[tid] = (int)D[(int)(S.code(e - 1) >> 1) * N1];
            } else {
                rret[tid] = 0;
            }
        }
    }
    __syncthreads();

    // ---- per-group tuple loop --------------------------------------------------
    long long best[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
    int pol = 0;
    for (int c = li; c <= n; c += GL) ready[c] = -1;   // "not dropped yet" for pol = 0
    wave_lds_fence();
    const bool veh = li < m;
    const int my_s = veh && !base_bad && !seg_bad ? rs_[li] : 0;
    const int my_len = veh && !base_bad && !seg_bad ? re_[li] - my_s : 0;
    for (int64_t t = t0 + (int64_t)ychunk * WPB * G + gidx; t < t1; t += (int64_t)ny * WPB * G) {
        const vrprpd_tuple tp = a.tuples[t];
        const int c = tp.c, vD = tp.vD, vP = tp.vP, pD = tp.pD, pP = tp.pP;
        bool valid = !seg_bad && c >= 1 && c <= n && vD < m && vP < m;
        if (valid && !rt_bad) {
            const uint32_t two = (bits[(2 * c) >> 5] >> ((2 * c) & 31)) & 3u;
            const int lenD = re_[vD] - rs_[vD], lenP = re_[vP] - rs_[vP];
            valid = two == 0u && pD <= lenD &&
                    (vP == vD ? (pP >= pD + 1 && pP <= lenD + 1) : (pP <= lenP));
        }
        // With an invalid route-end table the positions mean nothing: every
        // tuple of the segment reports BAD_COVER.
        int mk = INT32_MAX;
        uint32_t st;
        if (rt_bad && !seg_bad) {
            st = VRPRPD_ST_BAD_COVER;
        } else if (!valid) {
            st = VRPRPD_ST_BAD_TUPLE;
        } else if (base_bad) {
            st = VRPRPD_ST_BAD_COVER;
        } else {
            InsRoute<DT> R;
            R.S = &S;
            R.bs = my_s;
            R.len = my_len;
            R.x1 = R.x2 = kNoPos;
            R.k1 = R.k2 = 0;
            R.lg1 = R.lg2 = R.la1 = R.la2 = 0;
            R.ret = veh ? rret[li] : 0;
            const uint32_t kd = (uint32_t)c << 1, kp = kd | 1u;
            auto base_c = [&](int j) { return (int)(S.code(my_s + j) >> 1); };
            if (veh && li == vD && li == vP) {
                R.x1 = pD;
                R.k1 = kd;
                R.x2 = pP;
                R.k2 = kp;
                const int prevD = pD > 0 ? base_c(pD - 1) : 0;
                R.lg1 = (int)D[prevD * N1 + c];
                if (pP == pD + 1) {
                    R.lg2 = 0;  // d[c][c]
                } else {
                    R.la1 = (int)D[c * N1 + base_c(pD)];
                    R.lg2 = (int)D[base_c(pP - 2) * N1 + c];
                }
                if (pP - 1 < my_len) R.la2 = (int)D[c * N1 + base_c(pP - 1)];
                else R.ret = (int)D[c * N1];
            } else if (veh && (li == vD || li == vP)) {
                const int x = li == vD ? pD : pP;
                R.x1 = x;
                R.k1 = li == vD ? kd : kp;
                const int prev = x > 0 ? base_c(x - 1) : 0;
                R.lg1 = (int)D[prev * N1 + c];
                if (x < my_len) R.la1 = (int)D[c * N1 + base_c(x)];
                else R.ret = (int)D[c * N1];
            }
            R.vlen = my_len + (R.x1 != kNoPos) + (R.x2 != kNoPos);
            if (li == 0) ready[c] = pol ? 0 : -1;
            wave_lds_fence();
            const SweepOut o = sweep_route<kScanStep, GL>(R, ready, pblk, pol);
            st = load_status<GL>(o, veh, m, I.k, I.R, I.load_model);
            const int ret = (veh && R.vlen > 0) ? o.t + R.ret : 0;
            const int z = group_max<GL>(ret);
            if (o.dead) {
                st |= VRPRPD_ST_DEADLOCK;
                pol = 0;
                for (int cc = li; cc <= n; cc += GL) ready[cc] = -1;
            } else {
                mk = z;
                pol ^= 1;
            }
            wave_lds_fence();
        }
        if (li == 0) {
            if (a.mk_out) a.mk_out[t] = mk;
            if (a.st_out) a.st_out[t] = st;
        }
        if (st == 0) top3_insert(best, ((long long)mk << 32) | (long long)(uint32_t)t);
    }

    // ---- segment top-3 -----------------------------------------------------------
    if (li == 0) {
        topbuf[3 * gidx + 0] = best[0];
        topbuf[3 * gidx + 1] = best[1];
        topbuf[3 * gidx + 2] = best[2];
    }
    __syncthreads();
    if (tid == 0) {
        long long t3[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        for (int i = 0; i < 3 * WPB * G; ++i) top3_insert(t3, topbuf[i]);
        // Merge into the segment's sorted triple, shared with the other blocks
        // of the segment: each key goes through the three slots with atomicMin,
        // carrying down whatever it displaces, so the slots end up holding the
        // three smallest keys whatever the order of the blocks.
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(a.seg_top3 + 3 * seg);
        for (int i = 0; i < 3 && t3[i] != INT64_MAX; ++i) {
            unsigned long long carry = (unsigned long long)t3[i];
            for (int sl = 0; sl < 3; ++sl) {
                const unsigned long long old = atomicMin(&dst[sl], carry);
                carry = old > carry ? old : carry;
            }
        }
    }
}

// seg_top3 <- INT64_MAX before the scan blocks merge into it.
__global__ void top3_fill_kernel(int64_t* top, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) top[i] = INT64_MAX;
}

template <typename DT, int GL>
int launch_scan(const ScanArgs& a, hipStream_t stream)
{
    constexpr int WPB = 4;
    const ScanLayout L = scan_layout<WPB, GL>(a.n_max, OpStore<DT>::kBytesPerOp);
    if ((size_t)L.bytes > kLdsPerCu)
        return set_error(VRPRPD_EINVAL, "vrprpd_insert_scan: n=%d needs %d B of LDS per block", a.n_max, L.bytes);
    auto* k = scan_kernel<DT, GL, WPB>;
    if (L.bytes > 64 * 1024)
        VRP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    L.bytes));
    if (!a.top3_ready) {
        const int64_t cnt = 3 * (int64_t)a.num_seg;
        hipLaunchKernelGGL(top3_fill_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, a.seg_top3,
                           cnt);
        VRP_HIP(hipGetLastError());
    }
    const int ny = a.blocks_per_seg > 0 ? a.blocks_per_seg : 1;
    hipLaunchKernelGGL(k, dim3(a.num_seg, ny), dim3(64 * WPB), L.bytes, stream, a);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

template <typename DT>
static int scan_gl(const ScanArgs& a, int m_max, hipStream_t st)
{
    if (m_max <= 16) return launch_scan<DT, 16>(a, st);
    if (m_max <= 32) return launch_scan<DT, 32>(a, st);
    return launch_scan<DT, 64>(a, st);
}

int insert_scan_launch(const ScanArgs& a, int m_max, int dist16, hipStream_t st)
{
    return dist16 ? scan_gl<uint16_t>(a, m_max, st) : scan_gl<int32_t>(a, m_max, st);
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" int vrprpd_insert_scan(const vrprpd_set* set, int32_t num_bases, const int32_t* base_inst,
                                  const int64_t* base_op_off, const uint16_t* base_ops,
                                  const int64_t* base_rt_off, const uint16_t* base_rt_end, int32_t num_seg,
                                  const int64_t* seg_off, const int32_t* seg_base, const vrprpd_tuple* tuples,
                                  int32_t* mk_out, uint32_t* st_out, int64_t* seg_top3, int32_t blocks_per_seg,
                                  void* stream)
{
    if (!set) return set_error(VRPRPD_EINVAL, "vrprpd_insert_scan: set is NULL");
    if (num_bases < 1 || num_seg < 0 || blocks_per_seg < 0 || blocks_per_seg > 65535)
        return set_error(VRPRPD_EINVAL, "vrprpd_insert_scan: need num_bases >= 1 and num_seg >= 0");
    if (num_seg == 0) return VRPRPD_OK;
    if (!base_ops || !base_rt_end || !seg_off || !tuples || !seg_top3)
        return set_error(VRPRPD_EINVAL, "vrprpd_insert_scan: base_ops, base_rt_end, seg_off, tuples and "
                                        "seg_top3 are required");
    if (base_inst && (!base_op_off || !base_rt_off) && !set->uniform_nm)
        return set_error(VRPRPD_EINVAL, "vrprpd_insert_scan: instances differ in n or m; pass base offsets");
    const int n_lds = base_inst ? set->n_max : set->host[0].n;
    const int m_max = base_inst ? set->m_max : set->host[0].m;
    ScanArgs a{set->d_inst, set->d_dist, set->d_proc, base_inst, base_op_off, base_ops, base_rt_off, base_rt_end,
               seg_off, seg_base, tuples, mk_out, st_out, seg_top3, nullptr, num_bases, set->num_inst, n_lds,
               num_seg, blocks_per_seg};
    return insert_scan_launch(a, m_max, set->dist16, reinterpret_cast<hipStream_t>(stream));
}
