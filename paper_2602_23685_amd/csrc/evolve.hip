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

namespace vrprpd {

// rank_of[i] = #{ j : (f_j, j) < (f_i, i) }; order[rank_of[i]] = i.
__global__ __launch_bounds__(256) void rank_kernel(const int64_t* __restrict__ fit, int32_t Np,
                                                   int32_t* __restrict__ order)
{
    __shared__ int64_t tile[1024];
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
};

__global__ __launch_bounds__(256) void evolve_kernel(EvolveArgs a)
{
    const int i = blockIdx.x;
    const int G = a.genes;
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

__global__ __launch_bounds__(256) void warm_encode_kernel(const InstDev* inst_tab, int32_t ii, const uint16_t* ops,
                                                          const uint16_t* rt, float* p0, float* h0)
{
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
                if (var) {
                    const double uu = (double)(r.x[u] >> 8) * (1.0 / 16777216.0);
                    double x = (double)g + (uu * 0.06 - 0.03);
                    if (x < 0.0) x = 0.0;
                    g = (float)x;
                    if (g >= 1.0f) g = 0.99999994f;
                }
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
    hipLaunchKernelGGL(rank_kernel, dim3((Np + 255) / 256), dim3(256), 0, st, fitness, Np, rank_out);
    VRP_HIP(hipGetLastError());
    const uint32_t thr = (uint32_t)std::floor(rho_e * 16777216.0);
    EvolveArgs a{prio, hint, rank_out, prio_out, hint_out, key_stride, seed, Np, genes, n_elite, n_mutant,
                 thr, generation};
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
