// Solution statistics (Section 5.2): per solution, the customers served
// cross-vehicle (drop and pickup on different vehicles) and the customers
// interleaved (the drop vehicle does another operation between the drop and
// the pickup: on one vehicle, an operation between the two in the route;
// across vehicles, the drop vehicle's next operation, if it happens before
// the pickup).  Times are those of the earliest-start schedule.
//
// One block per solution at a time.  Wave 0 runs the schedule with lane = vehicle in
// rounds: each lane advances until a pickup whose drop is not yet published,
// and a block barrier publishes the round's drops.  A round where no lane
// moves is a wait cycle.  The cover check and the counting run over all
// threads.  Per-solution arrays live in a global workspace.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "vrprpd.h"

namespace vrprpd {
namespace {

constexpr int kST = 256;

struct StatsArgs {
    const InstDev* tab;
    int num_inst;
    const void* dist;
    const int32_t* proc;
    const int32_t* inst;
    const int64_t* op_off;
    const uint16_t* ops;
    const int64_t* rt_off;
    const uint16_t* rt_end;
    int32_t* cross;
    int32_t* inter;
    int N;                     // n_max
    int n0, m0;                // instance 0's n, m (default strides)
    unsigned char* ws;
    int64_t ws_stride;
};

__host__ __device__ inline int64_t stats_ws_bytes(int N)
{
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    return up(4 * 2 * (int64_t)N) + 3 * up(4 * ((int64_t)N + 1)) + up(2 * 2 * (int64_t)N);
}

template <typename DT>
__device__ void stats_one(const StatsArgs& a, int64_t b, unsigned char* p)
{
    __shared__ int bad, moved, left, nx, ni;
    __shared__ int rs[kMaxM], re[kMaxM];
    const int i = a.inst ? a.inst[b] : 0;
    auto fail = [&]() {
        if (threadIdx.x == 0) {
            a.cross[b] = -1;
            a.inter[b] = -1;
        }
    };
    if (i < 0 || i >= a.num_inst) {
        fail();
        return;
    }
    const InstDev I = a.tab[i];
    const int n = I.n, m = I.m, N1 = n + 1;
    const DT* D = reinterpret_cast<const DT*>(a.dist) + I.d_off;
    const int32_t* P = a.proc + I.p_off;
    const uint16_t* ops = a.ops + (a.op_off ? a.op_off[b] : (int64_t)b * 2 * a.n0);
    const uint16_t* rt = a.rt_end + (a.rt_off ? a.rt_off[b] : (int64_t)b * a.m0);
    auto up = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    int32_t* times = reinterpret_cast<int32_t*>(p);
    p += up(4 * 2 * (int64_t)a.N);
    int32_t* ready = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)a.N + 1));
    int32_t* posD = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)a.N + 1));
    int32_t* posP = reinterpret_cast<int32_t*>(p);
    p += up(4 * ((int64_t)a.N + 1));
    uint16_t* veh = reinterpret_cast<uint16_t*>(p);

    if (threadIdx.x == 0) {
        bad = 0;
        nx = 0;
        ni = 0;
        int prev = 0;
        for (int v = 0; v < m; ++v) {
            const int e = rt[v];
            if (e < prev || e > 2 * n) bad = 1;
            rs[v] = prev;
            re[v] = e;
            prev = e < prev ? prev : e;
        }
    }
    for (int c = threadIdx.x; c <= n; c += kST) {
        posD[c] = -1;
        posP[c] = -1;
        ready[c] = -1;
    }
    __syncthreads();
    if (bad) {
        fail();
        return;
    }
    const int L = re[m - 1];
    // cover: every customer exactly one drop and one pickup
    for (int j = threadIdx.x; j < L; j += kST) {
        const int cd = ops[j], c = cd >> 1;
        if (c < 1 || c > n) {
            atomicOr(&bad, 1);
            continue;
        }
        int v = 0;
        while (v < m - 1 && j >= re[v]) ++v;
        veh[j] = (uint16_t)v;
        if (atomicExch((cd & 1) ? &posP[c] : &posD[c], j) != -1) atomicOr(&bad, 1);
    }
    __syncthreads();
    for (int c = 1 + threadIdx.x; c <= n; c += kST)
        if (posD[c] < 0 || posP[c] < 0) atomicOr(&bad, 1);
    __syncthreads();
    if (bad) {
        fail();
        return;
    }
    // schedule in rounds (wave 0, lane = vehicle)
    const int v = threadIdx.x;
    const bool lane = threadIdx.x < m;
    int ptr = lane ? rs[v] : 0, t = 0, loc = 0;
    for (;;) {
        int step = 0;
        if (lane) {
            while (ptr < re[v]) {
                const int cd = ops[ptr], c = cd >> 1;
                const int arr = t + (int)D[loc * N1 + c];
                int tn = arr;
                if (cd & 1) {
                    const int r = ready[c];
                    if (r < 0) break;
                    tn = arr > r ? arr : r;
                } else {
                    ready[c] = arr + P[c];
                }
                t = tn;
                times[ptr] = t;
                loc = c;
                ++ptr;
                ++step;
            }
        }
        if (threadIdx.x == 0) {
            moved = 0;
            left = 0;
        }
        __syncthreads();
        if (step) atomicOr(&moved, 1);
        if (lane && ptr < re[v]) atomicOr(&left, 1);
        __syncthreads();
        if (!left) break;
        if (!moved) {
            fail();
            return;
        }
    }
    // counts
    for (int c = 1 + threadIdx.x; c <= n; c += kST) {
        const int jd = posD[c], jp = posP[c];
        const int vd = veh[jd], vp = veh[jp];
        if (vd != vp) {
            atomicAdd(&nx, 1);
            if (jd + 1 < re[vd] && times[jd + 1] < times[jp]) atomicAdd(&ni, 1);
        } else if (jp != jd + 1) {
            atomicAdd(&ni, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.cross[b] = nx;
        a.inter[b] = ni;
    }
}

// Blocks take solutions b, b + gridDim.x, ...; each block owns one slice of
// the workspace.
template <typename DT>
__global__ __launch_bounds__(kST) void k_stats(StatsArgs a, int64_t B)
{
    unsigned char* ws = a.ws + (int64_t)blockIdx.x * a.ws_stride;
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        stats_one<DT>(a, b, ws);
        __syncthreads();
    }
}

}  // namespace
}  // namespace vrprpd

extern "C" int vrprpd_solution_stats(const vrprpd_set* set, int64_t B, const int32_t* inst, const int64_t* op_off,
                                     const uint16_t* ops, const int64_t* rt_off, const uint16_t* rt_end,
                                     int32_t* cross, int32_t* interleaved, void* stream)
{
    using namespace vrprpd;
    if (!set || B < 0 || (B > 0 && (!ops || !rt_end || !cross || !interleaved)))
        return set_error(VRPRPD_EINVAL, "vrprpd_solution_stats: bad arguments");
    if (B == 0) return VRPRPD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    StatsArgs a;
    a.tab = set->d_inst;
    a.num_inst = set->num_inst;
    a.dist = set->d_dist;
    a.proc = set->d_proc;
    a.inst = inst;
    a.op_off = op_off;
    a.ops = ops;
    a.rt_off = rt_off;
    a.rt_end = rt_end;
    a.cross = cross;
    a.inter = interleaved;
    a.N = set->n_max;
    a.n0 = set->host[0].n;
    a.m0 = set->host[0].m;
    a.ws_stride = stats_ws_bytes(set->n_max);
    const int grid = (int)std::min<int64_t>(B, 2048);
    void* ws = nullptr;
    VRP_HIP(hipMallocAsync(&ws, (size_t)(a.ws_stride * grid), st));
    a.ws = static_cast<unsigned char*>(ws);
    if (set->dist16)
        hipLaunchKernelGGL(k_stats<uint16_t>, dim3(grid), dim3(kST), 0, st, a, B);
    else
        hipLaunchKernelGGL(k_stats<int32_t>, dim3(grid), dim3(kST), 0, st, a, B);
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_error(e, "vrprpd_solution_stats: launch");
    return VRPRPD_OK;
}
