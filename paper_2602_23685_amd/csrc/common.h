// Internal definitions shared by the library's translation units (not part of
// the C-ABI).  gfx950 only: 64-lane wavefronts, 160 KB LDS per CU, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
#include <tuple>
#include <utility>
#include <vector>

#include "vrprpd.h"

namespace vrprpd {

constexpr int kWave = 64;
constexpr int kXcds = 8;
constexpr int kMaxN = 10000;          // per-candidate state must fit in one CU's LDS
constexpr int kMaxM = 64;             // one lane per vehicle
constexpr size_t kLdsPerCu = 160 * 1024;

// Per-instance description as the kernels see it.
struct InstDev {
    int32_t n, m, k, R, load_model;
    int32_t ashift;  // right shift bringing every distance below 2^14 (pseudo-angles)
    int64_t d_off;  // element offset of d[0][0] in the packed distance buffer
    int64_t p_off;  // element offset of p[0] in the processing-time buffer
};

// Records a message for vrprpd_last_error() and returns code.
int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
int64_t mlp_max_rows(const vrprpd_mlp* h);   // rows a network handle can score at once
// brkga_decode_eval with a caller-provided workspace of decode_ws_bytes
// (by_inst: an instance array is passed; want_ops: sequences are written).
int64_t decode_ws_bytes(const vrprpd_set* set, int64_t B, bool by_inst, bool want_ops);
int decode_launch(const vrprpd_set* set, int64_t B, const int32_t* inst, const float* prio, const float* hint,
                  int64_t key_stride, int32_t flags, int64_t* fitness, int32_t* makespan, int32_t* unscheduled,
                  uint32_t* status, uint16_t* ops_out, uint16_t* rt_end_out, void* ws, hipStream_t st);

#define VRP_HIP(call)                                                      \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return ::vrprpd::hip_error(e_, #call);        \
    } while (0)

// Maps a launch's block index to the tile it works on so that consecutive
// tiles land on the same XCD: the hardware deals blocks round-robin over the
// 8 XCDs, so tiles i and i+1 (usually the same instance and base solution)
// would otherwise sit in different L2 caches.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb / kXcds, r = nb % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x * q + (x < r ? x : r) + i;
}

// p[i] for 0 <= i with i * sizeof(T) < 2^32: the byte offset is formed in 32
// bits so that a wave-uniform p becomes the scalar base of the load.
template <typename T>
__device__ __forceinline__ T ld_elem(const T* p, int i)
{
    const uint32_t off = (uint32_t)i * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
}

// fp32 -> bfloat16 bits, round to nearest even (finite inputs).
__host__ __device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Cross-lane helpers over groups of GL consecutive lanes of a wavefront.
template <int GL>
__device__ __forceinline__ uint64_t group_ballot(bool pred)
{
    const uint64_t all = __ballot(pred);
    if constexpr (GL == 64) {
        return all;
    } else {
        const int grp = (threadIdx.x & 63) / GL;
        return (all >> (grp * GL)) & ((1ull << GL) - 1);
    }
}

template <int GL>
__device__ __forceinline__ int group_max(int x)
{
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, GL));
    return x;
}

template <int GL>
__device__ __forceinline__ int group_sum(int x)
{
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, GL);
    return x;
}

template <int GL>
__device__ __forceinline__ long long group_min64(long long x)
{
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) {
        long long y = __shfl_xor(x, o, GL);
        x = y < x ? y : x;
    }
    return x;
}

// LDS loads/stores that other lanes of the same wave may have written since
// the last access: relaxed atomics at wavefront scope compile to plain ds ops
// but keep the compiler from caching or reordering them.
__device__ __forceinline__ int lds_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void lds_store(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Least power of two >= x (x >= 1).
__host__ __device__ inline int pow2_ge(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Block-wide bitonic sort of n (power of two) u64 keys, ascending; key may
// point to LDS or to global memory private to the block.  Every stage goes
// through memory.
__device__ inline void block_sort_u64_mem(unsigned long long* key, int n)
{
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], b = key[l];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// One compare-exchange stage with partner distance J < 8 on the 8 keys
// r[0..7] = key[8t .. 8t+8) that thread t holds in registers.
template <int J>
__device__ __forceinline__ void sort8_stage(unsigned long long (&r)[8], int base, int k)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = e ^ J;
        if (f > e) {
            const unsigned long long a = r[e], b = r[f];
            if ((a > b) == (((base + e) & k) == 0)) {
                r[e] = b;
                r[f] = a;
            }
        }
    }
}

// Compare-exchange toward ascending order when up, descending otherwise.
__device__ __forceinline__ void cx_u64(unsigned long long& a, unsigned long long& b, bool up)
{
    const bool sw = (a > b) == up;
    const unsigned long long x = a;
    a = sw ? b : a;
    b = sw ? x : b;
}

// S consecutive stages of the bitonic merge of size k, partner distances
// j, j/2, ..., q = j / 2^(S-1) (q >= 8), in one pass over memory: each
// thread loads the 2^S keys i0 + e q (i0 with the S distance bits clear, all
// in one run of 2j <= k keys, so one direction), runs the S stages in
// registers and stores them back.
template <int S>
__device__ __forceinline__ void bitonic_group(unsigned long long* key, int n, int k, int j)
{
    constexpr int E = 1 << S;
    const int q = j >> (S - 1);
    const int lq = __ffs(q) - 1;
    for (int g = threadIdx.x; g < n / E; g += blockDim.x) {
        const int i0 = (g & (q - 1)) | ((g >> lq) << (lq + S));
        const bool up = (i0 & k) == 0;
        unsigned long long r[E];
#pragma unroll
        for (int e = 0; e < E; ++e) r[e] = key[i0 + e * q];
#pragma unroll
        for (int d = E / 2; d >= 1; d >>= 1)
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (!(e & d)) cx_u64(r[e], r[e | d], up);
#pragma unroll
        for (int e = 0; e < E; ++e) key[i0 + e * q] = r[e];
    }
    __syncthreads();
}

// The same sort with few passes over memory: the stages of partner distance
// below 8 run in registers on 8 consecutive keys per thread, the others in
// groups of up to three stages per pass (bitonic_group), so a merge of size
// k = 2048 takes three passes and a register pass instead of eight stages.
// n >= 16 (a power of two); smaller n uses the memory-only network.
__device__ inline void block_sort_u64(unsigned long long* key, int n)
{
    if (n < 16) {
        block_sort_u64_mem(key, n);
        return;
    }
    const int T = blockDim.x;
    for (int base = 8 * threadIdx.x; base < n; base += 8 * T) {
        unsigned long long r[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = key[base + e];
        sort8_stage<1>(r, base, 2);
        sort8_stage<2>(r, base, 4);
        sort8_stage<1>(r, base, 4);
        sort8_stage<4>(r, base, 8);
        sort8_stage<2>(r, base, 8);
        sort8_stage<1>(r, base, 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) key[base + e] = r[e];
    }
    __syncthreads();
    for (int k = 16; k <= n; k <<= 1) {
        int j = k >> 1;
        while (j >= 8) {
            if (j >= 32) {
                bitonic_group<3>(key, n, k, j);
                j >>= 3;
            } else if (j >= 16) {
                bitonic_group<2>(key, n, k, j);
                j >>= 2;
            } else {
                bitonic_group<1>(key, n, k, j);
                j >>= 1;
            }
        }
        for (int base = 8 * threadIdx.x; base < n; base += 8 * T) {
            unsigned long long r[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) r[e] = key[base + e];
            sort8_stage<4>(r, base, k);
            sort8_stage<2>(r, base, k);
            sort8_stage<1>(r, base, k);
#pragma unroll
            for (int e = 0; e < 8; ++e) key[base + e] = r[e];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace vrprpd

struct vrprpd_set {
    int device = 0;
    int32_t num_inst = 0, n_max = 0, m_max = 0, dist16 = 1;
    bool uniform_nm = true;
    int64_t time_bound = 0;            // max over instances of (2n+1) * max d + sum p (bounds every time)
    std::vector<vrprpd::InstDev> host;  // same table as d_inst, on the host
    vrprpd::InstDev* d_inst = nullptr;
    void* d_dist = nullptr;            // uint16_t or int32_t, per dist16
    int32_t* d_proc = nullptr;
    // launch shapes of vrprpd_eval chosen by vrprpd_autotune_eval, keyed by
    // (n, m) of the launch: (candidates per wave, ops per lane per sweep
    // step, 1 for the live-leg form)
    std::map<std::pair<int, int>, std::tuple<int, int, int>> eval_tuned;
    // tuples per workgroup of the ALNS repair rounds' insertion scans chosen by
    // alns_autotune, keyed by (n_max, m_max, tuple budget) of the state
    mutable std::map<std::tuple<int, int, int>, int> alns_scan_tuned;
};
