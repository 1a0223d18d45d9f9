// BRKGA population operators (Section 4.4.3 and 4.4.4).
//
// brkga_evolve: rank by (fitness, index), then one block per child:
//   rank < n_elite                 copy of the rank-th individual (elite)
//   n_elite <= i < n_elite+n_mut   fresh U(0,1) genes (mutant)
//   otherwise                      biased uniform crossover of an elite parent
//                                  and a non-elite parent, each gene from the
//                                  elite one with probability rho_e
// Random draws are Philox4x32-10 words indexed by (gene, child, generation),
// so the result does not depend on the launch shape.
//
// brkga_warm_start: seed encoding of a solution (Section 4.4.4): the op at
// 1-based position r of a route of L_v ops gets priority (r-1)/L_v and every
// op of vehicle v gets hint (v + 1/2)/m; n_warm slots cycle through
// n_variants variants of it (variant 0 unperturbed, the others moved by
// U(-0.03, 0.03) per gene and clamped into [0, 1)); the remaining slots are
// fresh U(0,1) individuals.
#include "common.h"
#include "philox.h"
#include "ckpt.h"

namespace vrprpd {

// rank_of[i] = #{ j : (f_j, j) < (f_i, i) }; order[rank_of[i]] = i.
// Population blockIdx.y occupies entries [y Np, (y + 1) Np) of fit and order.
__global__ __launch_bounds__(256) void rank_kernel(const int64_t* __restrict__ fit, int32_t Np,
                                                   int32_t* __restrict__ order)
{
    __shared__ int64_t tile[1024];
    fit += (int64_t)blockIdx.y * Np;
    order += (int64_t)blockIdx.y * Np;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int64_t fi = i < Np ? fit[i] : 0;
    int rank = 0;
    for (int t0 = 0; t0 < Np; t0 += 1024) {
        __syncthreads();
        for (int j = threadIdx.x; j < 1024 && t0 + j < Np; j += 256) tile[j] = fit[t0 + j];
        __syncthreads();
        const int cnt = min(1024, Np - t0);
        for (int j = 0; j < cnt; ++j) {
            const int64_t fj = tile[j];
            rank += (fj < fi) || (fj == fi && t0 + j < i);
        }
    }
    if (i < Np) order[rank] = i;
}

// The same order by sorting: one block per population (Np <= kSortRankMax),
// a bitonic network over (fitness, index) pairs in LDS; the pair order is
// the rank order, so order[r] is the index in place r.
constexpr int kSortRankMax = 4096;
__global__ __launch_bounds__(1024) void rank_sort_kernel(const int64_t* __restrict__ fit, int32_t Np,
                                                         int32_t* __restrict__ order)
{
    __shared__ int64_t f[kSortRankMax];
    __shared__ uint16_t x[kSortRankMax];
    fit += (int64_t)blockIdx.y * Np;
    order += (int64_t)blockIdx.y * Np;
    int np = 1;
    while (np < Np) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        f[i] = i < Np ? fit[i] : INT64_MAX;
        x[i] = (uint16_t)i;                   // padding sorts after every real entry
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int64_t fi = f[i], fl = f[l];
                    const uint16_t xi = x[i], xl = x[l];
                    const bool gt = fi > fl || (fi == fl && xi > xl);
                    if (gt == ((i & k) == 0)) {
                        f[i] = fl;
                        f[l] = fi;
                        x[i] = xl;
                        x[l] = xi;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < Np; r += blockDim.x) order[r] = x[r];
}

// Ranks each of P populations of Np individuals (fitness [P][Np]) into order.
static void launch_rank(const int64_t* fit, int32_t Np, int32_t P, int32_t* order, hipStream_t st)
{
    if (Np <= kSortRankMax)
        hipLaunchKernelGGL(rank_sort_kernel, dim3(1, P), dim3(1024), 0, st, fit, Np, order);
    else
        hipLaunchKernelGGL(rank_kernel, dim3((Np + 255) / 256, P), dim3(256), 0, st, fit, Np, order);
}

struct EvolveArgs {
    const float* prio;
    const float* hint;
    const int32_t* order;
    float* prio_out;
    float* hint_out;
    int64_t stride;
    uint64_t seed;
    int32_t Np, genes, n_elite, n_mutant;
    uint32_t thr24, generation;
    const uint32_t* gen_dev;    // generation read from device memory (batched form), else `generation`
    const int32_t* genes_of;    // genes of each population (batched form), else `genes`
};

// Seed of population p of a batched run (population 0 keeps the seed).
__host__ __device__ inline uint64_t pop_seed(uint64_t seed, int p) { return seed + 0x9E3779B97F4A7C15ull * (uint64_t)p; }

// Block (child, population).
__global__ __launch_bounds__(256) void evolve_kernel(EvolveArgs a)
{
    const int i = blockIdx.x;
    const int pop = blockIdx.y;
    if (pop) {
        const int64_t rows = (int64_t)pop * a.Np;
        a.prio += rows * a.stride;
        a.prio_out += rows * a.stride;
        if (a.hint) {
            a.hint += rows * a.stride;
            a.hint_out += rows * a.stride;
        }
        a.order += rows;
    }
    a.seed = pop_seed(a.seed, pop);
    if (a.gen_dev) a.generation = *a.gen_dev;
    const int G = a.genes_of ? a.genes_of[pop] : a.genes;
    const int total = a.hint ? 2 * G : G;
    float* dp = a.prio_out + (int64_t)i * a.stride;
    float* dh = a.hint ? a.hint_out + (int64_t)i * a.stride : nullptr;
    if (i < a.n_elite) {
        const int s = a.order[i];
        const float* sp = a.prio + (int64_t)s * a.stride;
        const float* sh = a.hint ? a.hint + (int64_t)s * a.stride : nullptr;
        for (int j = threadIdx.x; j < G; j += 256) {
            dp[j] = sp[j];
            if (dh) dh[j] = sh[j];
        }
        return;
    }
    const bool mutant = i < a.n_elite + a.n_mutant;
    const float *ep = nullptr, *eh = nullptr, *xp = nullptr, *xh = nullptr;
    if (!mutant) {
        const uint32_t we = philox_word(a.seed, 0, (uint32_t)i, a.generation, kTagParent);
        const uint32_t wn = philox_word(a.seed, 1, (uint32_t)i, a.generation, kTagParent);
        const int e = a.order[(int)(((uint64_t)we * (uint64_t)a.n_elite) >> 32)];
        const int x = a.order[a.n_elite + (int)(((uint64_t)wn * (uint64_t)(a.Np - a.n_elite)) >> 32)];
        ep = a.prio + (int64_t)e * a.stride;
        xp = a.prio + (int64_t)x * a.stride;
        if (a.hint) {
            eh = a.hint + (int64_t)e * a.stride;
            xh = a.hint + (int64_t)x * a.stride;
        }
    }
    const uint32_t tag = mutant ? kTagMutant : kTagCross;
    for (int blk = threadIdx.x; 4 * blk < total; blk += 256) {
        const Philox4 r = philox4x32_10((uint32_t)blk, (uint32_t)i, a.generation, tag, (uint32_t)a.seed,
                                        (uint32_t)(a.seed >> 32));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * blk + u;
            if (j >= total) break;
            const uint32_t w = r.x[u];
            float g;
            if (mutant) {
                g = unit24(w);
            } else {
                const bool from_elite = (w >> 8) < a.thr24;
                g = j < G ? (from_elite ? ep[j] : xp[j]) : (from_elite ? eh[j - G] : xh[j - G]);
            }
            if (j < G) dp[j] = g;
            else dh[j - G] = g;
        }
    }
}

// Block s encodes source s (ops + s * op_stride, rt + s * rt_stride) into
// p0 / h0 + s * enc_stride.
__global__ __launch_bounds__(256) void warm_encode_kernel(const InstDev* inst_tab, int32_t ii, const uint16_t* ops,
                                                          const uint16_t* rt, float* p0, float* h0,
                                                          int64_t op_stride = 0, int64_t rt_stride = 0,
                                                          int64_t enc_stride = 0)
{
    ops += blockIdx.x * op_stride;
    rt += blockIdx.x * rt_stride;
    p0 += blockIdx.x * enc_stride;
    h0 += blockIdx.x * enc_stride;
    const InstDev I = inst_tab[ii];
    const int G = 2 * I.n, m = I.m;
    for (int o = threadIdx.x; o < G; o += 256) {
        p0[o] = 0.0f;
        h0[o] = 0.0f;
    }
    __syncthreads();
    for (int v = 0; v < m; ++v) {
        const int s = v ? rt[v - 1] : 0, e = rt[v];
        const int L = e - s;
        for (int j = s + threadIdx.x; j < e; j += 256) {
            const int c = ops[j] >> 1, isP = ops[j] & 1;
            if (c < 1 || c > I.n) continue;
            const int o = 2 * (c - 1) + isP;
            p0[o] = (float)((double)(j - s) / (double)L);
            h0[o] = (float)(((double)v + 0.5) / (double)m);
        }
    }
}

// A variant's gene: moved by U(-0.03, 0.03) (fp64) and clamped into [0, 1).
__device__ inline float perturb(float g, uint32_t w)
{
    const double uu = (double)(w >> 8) * (1.0 / 16777216.0);
    double x = (double)g + (uu * 0.06 - 0.03);
    if (x < 0.0) x = 0.0;
    g = (float)x;
    return g >= 1.0f ? 0.99999994f : g;
}

constexpr int kMaxWarmSources = 16;
struct WarmSources {
    int32_t n_src, total;
    int32_t cum[kMaxWarmSources + 1];   // first variant index of each source
};

// Slot i of a population warm-started from several sources: slots below
// n_warm cycle through the sources' variants (source order), the rest are
// fresh U(0,1) individuals.
__global__ __launch_bounds__(256) void warm_multi_fill_kernel(int32_t G, int64_t stride, int32_t n_warm,
                                                              WarmSources src, uint64_t seed, const float* enc_p,
                                                              const float* enc_h, float* prio, float* hint)
{
    const int i = blockIdx.x;
    float* dp = prio + (int64_t)i * stride;
    float* dh = hint + (int64_t)i * stride;
    const bool warm = i < n_warm && src.total > 0;
    int s = 0;
    uint32_t var = 0;
    if (warm) {
        const int q = i % src.total;
        while (q >= src.cum[s + 1]) ++s;
        var = (uint32_t)(q - src.cum[s]);
    }
    const float* p0 = enc_p + (int64_t)s * G;
    const float* h0 = enc_h + (int64_t)s * G;
    for (int blk = threadIdx.x; 4 * blk < 2 * G; blk += 256) {
        const Philox4 r = warm ? philox4x32_10((uint32_t)blk, var, (uint32_t)s, kTagWarm, (uint32_t)seed,
                                               (uint32_t)(seed >> 32))
                               : philox4x32_10((uint32_t)blk, (uint32_t)i, 0u, kTagRandom, (uint32_t)seed,
                                               (uint32_t)(seed >> 32));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * blk + u;
            if (j >= 2 * G) break;
            float g;
            if (warm) {
                g = j < G ? p0[j] : h0[j - G];
                if (var) g = perturb(g, r.x[u]);
            } else {
                g = unit24(r.x[u]);
            }
            if (j < G) dp[j] = g;
            else dh[j - G] = g;
        }
    }
}

__global__ __launch_bounds__(256) void warm_fill_kernel(int32_t G, int64_t stride, int32_t n_warm, int32_t n_var,
                                                        uint64_t seed, float* prio, float* hint)
{
    const int i = blockIdx.x + 1;   // slot 0 holds the encoding itself
    float* dp = prio + (int64_t)i * stride;
    float* dh = hint + (int64_t)i * stride;
    const float* p0 = prio;
    const float* h0 = hint;
    const uint32_t var = i < n_warm ? (uint32_t)(i % n_var) : 0u;
    for (int blk = threadIdx.x; 4 * blk < 2 * G; blk += 256) {
        Philox4 r;
        if (i < n_warm)
            r = philox4x32_10((uint32_t)blk, var, 0u, kTagWarm, (uint32_t)seed, (uint32_t)(seed >> 32));
        else
            r = philox4x32_10((uint32_t)blk, (uint32_t)i, 0u, kTagRandom, (uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * blk + u;
            if (j >= 2 * G) break;
            float g;
            if (i < n_warm) {
                g = j < G ? p0[j] : h0[j - G];
                if (var) g = perturb(g, r.x[u]);
            } else {
                g = unit24(r.x[u]);
            }
            if (j < G) dp[j] = g;
            else dh[j - G] = g;
        }
    }
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" int brkga_evolve(int32_t Np, int32_t genes, int64_t key_stride, const float* prio, const float* hint,
                            const int64_t* fitness, int32_t n_elite, int32_t n_mutant, double rho_e, uint64_t seed,
                            uint32_t generation, float* prio_out, float* hint_out, int32_t* rank_out, void* stream)
{
    if (Np < 1 || genes < 1 || key_stride < genes || !prio || !fitness || !prio_out || !rank_out ||
        (hint && !hint_out))
        return set_error(VRPRPD_EINVAL, "brkga_evolve: need Np >= 1, genes >= 1, key_stride >= genes and "
                                        "prio, fitness, prio_out, rank_out (hint_out with hint)");
    if (n_elite < 0 || n_mutant < 0 || n_elite + n_mutant > Np ||
        (Np - n_elite - n_mutant > 0 && (n_elite < 1 || Np - n_elite < 1)))
        return set_error(VRPRPD_EINVAL, "brkga_evolve: bad elite/mutant sizes %d/%d for Np=%d", n_elite,
                         n_mutant, Np);
    if (!(rho_e >= 0.0 && rho_e <= 1.0)) return set_error(VRPRPD_EINVAL, "brkga_evolve: rho_e outside [0, 1]");
    if (prio == prio_out || (hint && hint == hint_out))
        return set_error(VRPRPD_EINVAL, "brkga_evolve: output must not alias the input population");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    launch_rank(fitness, Np, 1, rank_out, st);
    VRP_HIP(hipGetLastError());
    const uint32_t thr = (uint32_t)std::floor(rho_e * 16777216.0);
    EvolveArgs a{prio, hint, rank_out, prio_out, hint_out, key_stride, seed, Np, genes, n_elite, n_mutant,
                 thr, generation, nullptr, nullptr};
    hipLaunchKernelGGL(evolve_kernel, dim3(Np), dim3(256), 0, st, a);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int brkga_warm_start(const vrprpd_set* set, int32_t inst, const uint16_t* ops, const uint16_t* rt_end,
                                int32_t Np, int32_t n_warm, int32_t n_variants, uint64_t seed, int64_t key_stride,
                                float* prio_out, float* hint_out, void* stream)
{
    if (!set || inst < 0 || inst >= set->num_inst || !ops || !rt_end || !prio_out || !hint_out || Np < 1 ||
        n_warm < 1 || n_warm > Np || n_variants < 1)
        return set_error(VRPRPD_EINVAL, "brkga_warm_start: bad arguments");
    const int G = 2 * set->host[inst].n;
    if (key_stride < G) return set_error(VRPRPD_EINVAL, "brkga_warm_start: key_stride < 2n");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(warm_encode_kernel, dim3(1), dim3(256), 0, st, set->d_inst, inst, ops, rt_end, prio_out,
                       hint_out);
    VRP_HIP(hipGetLastError());
    if (Np > 1) {
        hipLaunchKernelGGL(warm_fill_kernel, dim3(Np - 1), dim3(256), 0, st, G, key_stride, n_warm, n_variants,
                           seed, prio_out, hint_out);
        VRP_HIP(hipGetLastError());
    }
    return VRPRPD_OK;
}

extern "C" int brkga_warm_start_multi(const vrprpd_set* set, int32_t inst, int32_t n_src, const uint16_t* ops,
                                      int64_t op_stride, const uint16_t* rt_end, int64_t rt_stride,
                                      const int32_t* n_var, int32_t Np, int32_t n_warm, uint64_t seed,
                                      int64_t key_stride, float* prio_out, float* hint_out, void* stream)
{
    if (!set || inst < 0 || inst >= set->num_inst || n_src < 1 || n_src > kMaxWarmSources || !ops || !rt_end ||
        !n_var || !prio_out || !hint_out || Np < 1 || n_warm < 0 || n_warm > Np)
        return set_error(VRPRPD_EINVAL, "brkga_warm_start_multi: bad arguments");
    const InstDev& I = set->host[inst];
    const int G = 2 * I.n;
    if (key_stride < G || op_stride < G || rt_stride < I.m)
        return set_error(VRPRPD_EINVAL, "brkga_warm_start_multi: need key_stride, op_stride >= 2n and rt_stride >= m");
    WarmSources src{};
    src.n_src = n_src;
    for (int s = 0; s < n_src; ++s) {
        if (n_var[s] < 0) return set_error(VRPRPD_EINVAL, "brkga_warm_start_multi: n_var[%d] < 0", s);
        src.cum[s + 1] = src.cum[s] + n_var[s];
    }
    for (int s = n_src + 1; s <= kMaxWarmSources; ++s) src.cum[s] = src.cum[n_src];
    src.total = src.cum[n_src];
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    void* enc = nullptr;
    VRP_HIP(hipMallocAsync(&enc, (size_t)2 * n_src * G * sizeof(float), st));
    float* ep = static_cast<float*>(enc);
    float* eh = ep + (size_t)n_src * G;
    hipLaunchKernelGGL(warm_encode_kernel, dim3(n_src), dim3(256), 0, st, set->d_inst, inst, ops, rt_end, ep, eh,
                       op_stride, rt_stride, (int64_t)G);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(warm_multi_fill_kernel, dim3(Np), dim3(256), 0, st, G, key_stride, n_warm, src, seed, ep,
                           eh, prio_out, hint_out);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(enc, st);
    if (e != hipSuccess) return hip_error(e, "brkga_warm_start_multi: launch");
    return VRPRPD_OK;
}

// ============================================================== batched form
// Many instances' populations evolved together (one decode launch over every
// individual, one rank and one evolve launch over every population), one
// generation captured as a HIP graph per population buffer and replayed.
// Population p uses seed pop_seed(seed, p), so it evolves exactly as a
// single-population run of brkga_evolve with that seed would.
namespace vrprpd {

__global__ __launch_bounds__(256) void random_pop_kernel(int64_t stride, const int32_t* genes_of, int32_t Np,
                                                         uint64_t seed, float* prio, float* hint)
{
    const int i = blockIdx.x, pop = blockIdx.y;
    const int G = genes_of[pop];
    const uint64_t sd = pop_seed(seed, pop);
    const int64_t row = (int64_t)pop * Np + i;
    for (int blk = threadIdx.x; 4 * blk < 2 * G; blk += 256) {
        const Philox4 r = philox4x32_10((uint32_t)blk, (uint32_t)i, 0u, kTagRandom, (uint32_t)sd, (uint32_t)(sd >> 32));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * blk + u;
            if (j >= 2 * G) break;
            if (j < G) prio[row * stride + j] = unit24(r.x[u]);
            else hint[row * stride + j - G] = unit24(r.x[u]);
        }
    }
}

// Block per population, after ranking: keep the best individual seen so far.
__global__ __launch_bounds__(256) void best_kernel(int32_t Np, int64_t stride, const int32_t* order, const int64_t* fit,
                                                   const float* prio, const float* hint, int64_t* best_fit,
                                                   float* best_prio, float* best_hint)
{
    const int pop = blockIdx.x;
    const int b = order[(int64_t)pop * Np];
    const int64_t f = fit[(int64_t)pop * Np + b];
    __shared__ int better;
    if (threadIdx.x == 0) better = f < best_fit[pop];
    __syncthreads();
    if (!better) return;
    const int64_t row = (int64_t)pop * Np + b;
    for (int64_t j = threadIdx.x; j < stride; j += 256) {
        best_prio[pop * stride + j] = prio[row * stride + j];
        best_hint[pop * stride + j] = hint[row * stride + j];
    }
    __syncthreads();
    if (threadIdx.x == 0) best_fit[pop] = f;
}

__global__ void gen_tick_kernel(uint32_t* gen)
{
    if (threadIdx.x == 0) *gen += 1u;
}

}  // namespace vrprpd

struct brkga_state {
    const vrprpd_set* set = nullptr;
    int32_t P = 0, Np = 0, ne = 0, nm = 0;
    int32_t dflags = 0;   // decoder flags (VRPRPD_DECODE_*)
    uint32_t thr = 0;
    uint64_t seed = 0;
    int64_t stride = 0;
    int64_t generations = 0;
    float* prio[2] = {nullptr, nullptr};
    float* hint[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t *inst_of_row = nullptr, *genes_of = nullptr, *order = nullptr, *mk = nullptr, *unsch = nullptr;
    uint32_t* status = nullptr;
    int64_t *fit = nullptr, *best_fit = nullptr;
    float *best_prio = nullptr, *best_hint = nullptr;
    uint32_t* gen_dev = nullptr;
    void* dec_ws = nullptr;        // decoder workspace (orders, key flags)
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::vector<void*> allocs;
    std::vector<int32_t> inst_ids;   // host copy (checkpoint check)
};

namespace vrprpd {

// decode + evaluate the population in buffer `from`, keep the best, rank,
// evolve into the other buffer, advance the generation counter
static int brkga_generation(brkga_state* s, int from, hipStream_t st)
{
    const int64_t B = (int64_t)s->P * s->Np;
    int rc = decode_launch(s->set, B, s->inst_of_row, s->prio[from], s->hint[from], s->stride, s->dflags, s->fit, s->mk,
                           s->unsch, s->status, nullptr, nullptr, s->dec_ws, st);
    if (rc) return rc;
    launch_rank(s->fit, s->Np, s->P, s->order, st);
    hipLaunchKernelGGL(best_kernel, dim3(s->P), dim3(256), 0, st, s->Np, s->stride, s->order, s->fit, s->prio[from],
                       s->hint[from], s->best_fit, s->best_prio, s->best_hint);
    EvolveArgs a{s->prio[from], s->hint[from], s->order, s->prio[from ^ 1], s->hint[from ^ 1], s->stride, s->seed,
                 s->Np, 0, s->ne, s->nm, s->thr, 0u, s->gen_dev, s->genes_of};
    hipLaunchKernelGGL(evolve_kernel, dim3(s->Np, s->P), dim3(256), 0, st, a);
    hipLaunchKernelGGL(gen_tick_kernel, dim3(1), dim3(64), 0, st, s->gen_dev);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

}  // namespace vrprpd

extern "C" int brkga_state_destroy(brkga_state* s)
{
    if (!s) return VRPRPD_OK;
    // graphs of this state may still be replaying on the caller's streams
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 2; ++i) {
        if (s->gexec[i]) (void)hipGraphExecDestroy(s->gexec[i]);
        if (s->graph[i]) (void)hipGraphDestroy(s->graph[i]);
    }
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
    return VRPRPD_OK;
}

extern "C" int brkga_state_create(brkga_state** out, const vrprpd_set* set, int32_t n_inst, const int32_t* inst_ids,
                                  int32_t Np, int32_t n_elite, int32_t n_mutant, double rho_e, uint64_t seed,
                                  int32_t decode_flags, const float* prio0, const float* hint0, void* stream)
{
    if (!out) return set_error(VRPRPD_EINVAL, "brkga_state_create: out is NULL");
    *out = nullptr;
    if (!set || n_inst < 1 || !inst_ids || Np < 2 || n_elite < 1 || n_mutant < 0 || n_elite + n_mutant > Np ||
        Np - n_elite < 1 || !(rho_e >= 0.0 && rho_e <= 1.0) || ((prio0 == nullptr) != (hint0 == nullptr)))
        return set_error(VRPRPD_EINVAL, "brkga_state_create: bad arguments");
    if ((int64_t)n_inst * Np > INT32_MAX) return set_error(VRPRPD_EINVAL, "brkga_state_create: too many individuals");
    if (decode_flags & ~VRPRPD_DECODE_HINT_FIRST)
        return set_error(VRPRPD_EINVAL, "brkga_state_create: unknown decoder flags %d", decode_flags);
    int n_max = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (inst_ids[i] < 0 || inst_ids[i] >= set->num_inst)
            return set_error(VRPRPD_EINVAL, "brkga_state_create: instance id %d out of range", inst_ids[i]);
        n_max = std::max(n_max, set->host[inst_ids[i]].n);
    }
    if (n_max != set->n_max)
        return set_error(VRPRPD_EINVAL, "brkga_state_create: the set's largest instance must be among inst_ids "
                                        "(the decoder sizes its keys by the set)");
    brkga_state* s = new brkga_state;
    s->set = set;
    s->dflags = decode_flags;
    s->P = n_inst;
    s->Np = Np;
    s->ne = n_elite;
    s->nm = n_mutant;
    s->thr = (uint32_t)std::floor(rho_e * 16777216.0);
    s->seed = seed;
    s->inst_ids.assign(inst_ids, inst_ids + n_inst);
    s->stride = 2 * (int64_t)set->n_max;
    const int64_t B = (int64_t)n_inst * Np;
    hipError_t e = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(p, bytes ? bytes : 16);
        if (e == hipSuccess) {
            s->allocs.push_back(*p);
            e = hipMemset(*p, 0, bytes ? bytes : 16);
        }
    };
    for (int i = 0; i < 2; ++i) {
        A((void**)&s->prio[i], B * s->stride * 4);
        A((void**)&s->hint[i], B * s->stride * 4);
    }
    A((void**)&s->inst_of_row, B * 4);
    A((void**)&s->genes_of, n_inst * 4);
    A((void**)&s->order, B * 4);
    A((void**)&s->mk, B * 4);
    A((void**)&s->unsch, B * 4);
    A((void**)&s->status, B * 4);
    A((void**)&s->fit, B * 8);
    A((void**)&s->best_fit, n_inst * 8);
    A((void**)&s->best_prio, n_inst * s->stride * 4);
    A((void**)&s->best_hint, n_inst * s->stride * 4);
    A((void**)&s->gen_dev, 4);
    A(&s->dec_ws, (size_t)decode_ws_bytes(set, B, true, false));
    if (e != hipSuccess) {
        brkga_state_destroy(s);
        return set_error(VRPRPD_ENOMEM, "brkga_state_create: %s", hipGetErrorString(e));
    }
    std::vector<int32_t> rows(B), genes(n_inst);
    std::vector<int64_t> bf(n_inst, INT64_MAX);
    for (int p = 0; p < n_inst; ++p) {
        genes[p] = 2 * set->host[inst_ids[p]].n;
        for (int i = 0; i < Np; ++i) rows[(int64_t)p * Np + i] = inst_ids[p];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((e = hipMemcpy(s->inst_of_row, rows.data(), B * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->genes_of, genes.data(), n_inst * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->best_fit, bf.data(), n_inst * 8, hipMemcpyHostToDevice)) != hipSuccess) {
        brkga_state_destroy(s);
        return hip_error(e, "brkga_state_create: upload");
    }
    if (prio0) {
        if ((e = hipMemcpyAsync(s->prio[0], prio0, B * s->stride * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(s->hint[0], hint0, B * s->stride * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess) {
            brkga_state_destroy(s);
            return hip_error(e, "brkga_state_create: copy of the initial population");
        }
    } else {
        hipLaunchKernelGGL(random_pop_kernel, dim3(Np, n_inst), dim3(256), 0, st, s->stride, s->genes_of, Np, seed,
                           s->prio[0], s->hint[0]);
        if ((e = hipGetLastError()) != hipSuccess) {
            brkga_state_destroy(s);
            return hip_error(e, "brkga_state_create: initial population");
        }
    }
    *out = s;
    return VRPRPD_OK;
}

extern "C" int brkga_state_step(brkga_state* s, int32_t generations, int32_t use_graph, void* stream)
{
    if (!s || generations < 0) return set_error(VRPRPD_EINVAL, "brkga_state_step: bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int g = 0; g < generations; ++g) {
        const int from = s->cur;
        if (use_graph) {
            if (!s->gexec[from]) {
                if (!s->cap) VRP_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
                VRP_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
                const int rc = brkga_generation(s, from, s->cap);
                hipGraph_t gr = nullptr;
                const hipError_t e = hipStreamEndCapture(s->cap, &gr);
                if (rc) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return rc;
                }
                if (e != hipSuccess) return hip_error(e, "brkga_state_step: hipStreamEndCapture");
                s->graph[from] = gr;
                VRP_HIP(hipGraphInstantiate(&s->gexec[from], gr, nullptr, nullptr, 0));
            }
            VRP_HIP(hipGraphLaunch(s->gexec[from], st));
        } else {
            const int rc = brkga_generation(s, from, st);
            if (rc) return rc;
        }
        s->cur ^= 1;
        s->generations += 1;
    }
    return VRPRPD_OK;
}

extern "C" int brkga_state_get(const brkga_state* s, int64_t* generations, int64_t* best_fitness, float* best_prio,
                               float* best_hint, float* prio, float* hint, void* stream)
{
    if (!s) return set_error(VRPRPD_EINVAL, "brkga_state_get: state is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t B = (int64_t)s->P * s->Np;
    if (generations) *generations = s->generations;
    if (best_prio) VRP_HIP(hipMemcpyAsync(best_prio, s->best_prio, s->P * s->stride * 4, hipMemcpyDeviceToDevice, st));
    if (best_hint) VRP_HIP(hipMemcpyAsync(best_hint, s->best_hint, s->P * s->stride * 4, hipMemcpyDeviceToDevice, st));
    if (prio) VRP_HIP(hipMemcpyAsync(prio, s->prio[s->cur], B * s->stride * 4, hipMemcpyDeviceToDevice, st));
    if (hint) VRP_HIP(hipMemcpyAsync(hint, s->hint[s->cur], B * s->stride * 4, hipMemcpyDeviceToDevice, st));
    if (best_fitness) {
        VRP_HIP(hipStreamSynchronize(st));
        VRP_HIP(hipMemcpy(best_fitness, s->best_fit, s->P * 8, hipMemcpyDeviceToHost));
    }
    return VRPRPD_OK;
}

// ---------------------------------------------------------------- checkpoint
namespace vrprpd {

struct BrkgaCkptHead {
    char magic[8];           // "VRPBRKG1"
    int32_t P, Np, ne, nm;
    uint32_t thr, pad;
    uint64_t seed;
    int64_t stride, generations;
};

// The population to decode next, the best chromosome and fitness of every
// population so far, and the device generation counter.
static std::vector<DevField> brkga_fields(const brkga_state* s)
{
    const size_t B = (size_t)s->P * s->Np, S = (size_t)s->stride;
    return {{s->prio[s->cur], B * S * 4}, {s->hint[s->cur], B * S * 4}, {s->best_fit, (size_t)s->P * 8},
            {s->best_prio, (size_t)s->P * S * 4}, {s->best_hint, (size_t)s->P * S * 4}, {s->gen_dev, 4}};
}

static BrkgaCkptHead brkga_head(const brkga_state* s)
{
    BrkgaCkptHead h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "VRPBRKG1", 8);
    h.P = s->P;
    h.Np = s->Np;
    h.ne = s->ne;
    h.nm = s->nm;
    h.thr = s->thr;
    h.seed = s->seed;
    h.stride = s->stride;
    h.generations = s->generations;
    return h;
}

}  // namespace vrprpd

extern "C" int brkga_state_save(const brkga_state* s, void* buf, int64_t capacity, int64_t* bytes, void* stream)
{
    using namespace vrprpd;
    if (!s || (!buf && !bytes)) return set_error(VRPRPD_EINVAL, "brkga_state_save: bad arguments");
    std::vector<unsigned char> head(sizeof(BrkgaCkptHead) + s->inst_ids.size() * sizeof(int32_t));
    const BrkgaCkptHead h = brkga_head(s);
    std::memcpy(head.data(), &h, sizeof h);
    std::memcpy(head.data() + sizeof h, s->inst_ids.data(), s->inst_ids.size() * sizeof(int32_t));
    return ckpt_save(head.data(), head.size(), brkga_fields(s), buf, capacity, bytes,
                     reinterpret_cast<hipStream_t>(stream), "brkga_state_save");
}

extern "C" int brkga_state_load(brkga_state* s, const void* buf, int64_t bytes, void* stream)
{
    using namespace vrprpd;
    if (!s || !buf || bytes < (int64_t)sizeof(BrkgaCkptHead))
        return set_error(VRPRPD_EINVAL, "brkga_state_load: bad arguments");
    BrkgaCkptHead h;
    std::memcpy(&h, buf, sizeof h);
    const BrkgaCkptHead mine = brkga_head(s);
    if (std::memcmp(h.magic, "VRPBRKG1", 8) != 0)
        return set_error(VRPRPD_EINVAL, "brkga_state_load: not a BRKGA checkpoint");
    if (h.P != mine.P || h.Np != mine.Np || h.ne != mine.ne || h.nm != mine.nm || h.thr != mine.thr ||
        h.seed != mine.seed || h.stride != mine.stride)
        return set_error(VRPRPD_EINVAL, "brkga_state_load: the checkpoint was taken from a state with other "
                                        "populations, sizes, rho_e or seed");
    const size_t ids_bytes = s->inst_ids.size() * sizeof(int32_t);
    if (bytes < (int64_t)(sizeof h + ids_bytes) ||
        std::memcmp(static_cast<const unsigned char*>(buf) + sizeof h, s->inst_ids.data(), ids_bytes) != 0)
        return set_error(VRPRPD_EINVAL, "brkga_state_load: the checkpoint's populations belong to other instances");
    const int rc = ckpt_load(buf, bytes, sizeof h + ids_bytes, brkga_fields(s), reinterpret_cast<hipStream_t>(stream),
                             "brkga_state_load");
    if (rc) return rc;
    s->generations = h.generations;
    return VRPRPD_OK;
}
