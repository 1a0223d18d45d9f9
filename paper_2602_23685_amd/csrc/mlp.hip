// The learned destroy proposal's scorer network on the GPU: forward,
// backward and a momentum SGD step, all in this file's kernels.
//
// The paper lists learned destroy operators as future work (Section 7.4); the
// network is this library's: per-customer features (64) -> 256 -> 256 -> 256
// -> 1, ReLU after each hidden layer.  A removal set's score is the sum of
// its customers' scores, fitted to the makespan change by mean squared error.
//
// Precision: GEMM operands are bfloat16 (activations, weights and the masked
// upstream gradients, rounded to nearest even), products are accumulated in
// fp32 by the BF16 matrix cores (v_mfma_f32_32x32x16_bf16); biases, the head,
// the loss, gradients and the master weights stay fp32.
//
// GEMM: C[M][N] = sum_k A(m,k) B(n,k) with 128x128 block tiles, 4 waves of
// 64x64 (2x2 MFMA 32x32 tiles each), K in steps of 32 through double-buffered
// LDS.  Operands are read either k-contiguous ([row][k]) or transposed
// ([k][row]); a transposed operand is turned k-contiguous while it is written
// to LDS, so the three products of training need no transposed copies:
//   forward        H_l  = relu(H_{l-1} W_l^T + b_l)       A [m][k], B [n][k]
//   input grads    dZ_l = (dZ_{l+1} W_{l+1}) * [H_l > 0]  A [m][k], B [k][n]
//   weight grads   dW_l = dZ_l^T H_{l-1}  (split over rows) A [k][m], B [k][n]
#include <cstring>
#include <vector>

#include "common.h"
#include "philox.h"

namespace vrprpd {
namespace mlpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kIn = VRPRPD_MLP_IN, kHid = VRPRPD_MLP_HIDDEN;
constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK + 8;          // LDS row stride in bf16 (80 B: 16-byte aligned rows)
constexpr int kSplitRows = 1024;     // rows per block of a weight-gradient product
constexpr int kHeadRows = 256;       // rows per block of the head's backward

// Offsets of the flat parameter vector (W[out][in] then b per layer).
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kHid * kIn;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kHid * kHid;
constexpr int64_t kOffW4 = kOffB3 + kHid;
constexpr int64_t kOffB4 = kOffW4 + kHid;
constexpr int64_t kNumParams = kOffB4 + 1;
static_assert(kNumParams == VRPRPD_MLP_NUM_PARAMS, "parameter layout");

enum { EPI_RELU = 0, EPI_MASK = 1, EPI_PART = 2 };

struct GemmArgs {
    const uint16_t* A;
    int64_t lda;
    const uint16_t* B;
    int64_t ldb;
    int M, N, K, k_chunk;
    const float* bias;        // EPI_RELU: [N]
    uint16_t* out;            // EPI_RELU / EPI_MASK: bf16 [M][ldo]
    int64_t ldo;
    const uint16_t* mask;     // EPI_MASK: bf16 [M][ldm]; the value passes where mask > 0
    int64_t ldm;
    const uint16_t* head_w;   // EPI_RELU: bf16 [N] of the head, or NULL
    float* head_part;         // [N / 64][M]: per 64-column slice, sum_n h * head_w
    float* part;              // EPI_PART: fp32 [gridDim.z][M][N]
    float* colsum;            // EPI_PART with transposed A: [gridDim.z][M], sums of A over k
};

// One 16-byte chunk per thread per half tile: the 128 x 32 tile is 512 chunks.
template <bool kTrans>
__device__ __forceinline__ void load_tile(const uint16_t* X, int64_t ld, int r0, int R, int k0, int ke, int tid,
                                          uint4 (&reg)[2])
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = tid + 256 * h;
        int r, k;
        if constexpr (!kTrans) {
            r = c >> 2;
            k = (c & 3) * 8;
            const bool ok = r0 + r < R && k0 + k < ke;   // ke and k are multiples of 8
            reg[h] = ok ? *reinterpret_cast<const uint4*>(X + (int64_t)(r0 + r) * ld + k0 + k)
                        : make_uint4(0, 0, 0, 0);
        } else {
            k = c >> 4;
            r = (c & 15) * 8;
            const bool ok = k0 + k < ke && r0 + r < R;   // R and r are multiples of 8
            reg[h] = ok ? *reinterpret_cast<const uint4*>(X + (int64_t)(k0 + k) * ld + r0 + r)
                        : make_uint4(0, 0, 0, 0);
        }
    }
}

template <bool kTrans>
__device__ __forceinline__ void store_tile(uint16_t* S, int tid, const uint4 (&reg)[2])
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = tid + 256 * h;
        if constexpr (!kTrans) {
            *reinterpret_cast<uint4*>(S + (c >> 2) * LDK + (c & 3) * 8) = reg[h];
        } else {
            const int k = c >> 4, r = (c & 15) * 8;
            const uint32_t w[4] = {reg[h].x, reg[h].y, reg[h].z, reg[h].w};
#pragma unroll
            for (int e = 0; e < 8; ++e) S[(r + e) * LDK + k] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
        }
    }
}

// Sums of the 8 bf16 values of a chunk into acc (column sums of a transposed A).
__device__ __forceinline__ void add_chunk(float (&acc)[8], const uint4& v)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] += bf2f((uint16_t)(w[e >> 1] >> (16 * (e & 1))));
}

template <bool kAT, bool kBT, int kEpi>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    __shared__ __align__(16) uint16_t As[2][BM * LDK];
    __shared__ __align__(16) uint16_t Bs[2][BN * LDK];
    __shared__ float red[16][BM];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kb = blockIdx.z * g.k_chunk;
    const int ke = min(g.K, kb + g.k_chunk);
    const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const bool do_colsum = kEpi == EPI_PART && kAT && g.colsum && blockIdx.y == 0;

    f32x16 acc[2][2];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[f][h][r] = 0.f;
    float cs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    uint4 ra[2], rb[2];
    if (nk > 0) {
        load_tile<kAT>(g.A, g.lda, m0, g.M, kb, ke, tid, ra);
        load_tile<kBT>(g.B, g.ldb, n0, g.N, kb, ke, tid, rb);
        if (do_colsum) {
            add_chunk(cs, ra[0]);
            add_chunk(cs, ra[1]);
        }
        store_tile<kAT>(As[0], tid, ra);
        store_tile<kBT>(Bs[0], tid, rb);
    }
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        const bool more = t + 1 < nk;
        if (more) {
            load_tile<kAT>(g.A, g.lda, m0, g.M, kb + (t + 1) * BK, ke, tid, ra);
            load_tile<kBT>(g.B, g.ldb, n0, g.N, kb + (t + 1) * BK, ke, tid, rb);
        }
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8 a[2], b[2];
            const int kk = ks + (lane >> 5) * 8;
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int row = wm * 64 + f * 32 + (lane & 31);
                a[f] = *reinterpret_cast<const bf16x8*>(&As[cur][row * LDK + kk]);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int col = wn * 64 + h * 32 + (lane & 31);
                b[h] = *reinterpret_cast<const bf16x8*>(&Bs[cur][col * LDK + kk]);
            }
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    acc[f][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f], b[h], acc[f][h], 0, 0, 0);
        }
        if (more) {
            if (do_colsum) {
                add_chunk(cs, ra[0]);
                add_chunk(cs, ra[1]);
            }
            store_tile<kAT>(As[cur ^ 1], tid, ra);
            store_tile<kBT>(Bs[cur ^ 1], tid, rb);
        }
        __syncthreads();
    }

    // Accumulator element r of tile (f, h) of this lane:
    //   row m0 + wm*64 + f*32 + (r/4)*8 + (lane/32)*4 + r%4,  col n0 + wn*64 + h*32 + lane%32
    const int lrow = (lane >> 5) * 4;
    if constexpr (kEpi == EPI_PART) {
        float* P = g.part + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int col = n0 + wn * 64 + h * 32 + (lane & 31);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + f * 32 + (r >> 2) * 8 + lrow + (r & 3);
                    if (row < g.M && col < g.N) P[(int64_t)row * g.N + col] = acc[f][h][r];
                }
            }
        if (do_colsum) {
            // thread tid holds sums for columns (tid & 15) * 8 .. +7 over k rows tid/16 (mod 16)
#pragma unroll
            for (int e = 0; e < 8; ++e) red[tid >> 4][(tid & 15) * 8 + e] = cs[e];
            __syncthreads();
            if (tid < BM && m0 + tid < g.M) {
                float s = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) s += red[i][tid];
                g.colsum[(int64_t)blockIdx.z * g.M + m0 + tid] = s;
            }
        }
    } else {
        float hs[2][16];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int r = 0; r < 16; ++r) hs[f][r] = 0.f;
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int col = n0 + wn * 64 + h * 32 + (lane & 31);
                const bool cok = col < g.N;
                float bias = 0.f, hw = 0.f;
                if constexpr (kEpi == EPI_RELU) {
                    bias = cok ? g.bias[col] : 0.f;
                    hw = (cok && g.head_w) ? bf2f(g.head_w[col]) : 0.f;
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + f * 32 + (r >> 2) * 8 + lrow + (r & 3);
                    const bool ok = cok && row < g.M;
                    float v = acc[f][h][r];
                    if constexpr (kEpi == EPI_RELU) {
                        v += bias;
                        v = v > 0.f ? v : 0.f;
                    } else {
                        const float mk = ok ? bf2f(g.mask[(int64_t)row * g.ldm + col]) : 0.f;
                        v = mk > 0.f ? v : 0.f;
                    }
                    const uint16_t hb = f2bf(v);
                    if (ok) g.out[(int64_t)row * g.ldo + col] = hb;
                    if constexpr (kEpi == EPI_RELU) hs[f][r] += bf2f(hb) * hw;
                }
            }
        if constexpr (kEpi == EPI_RELU) {
            if (g.head_w) {
                // sum over the 32 columns held by the lanes of this half-wave
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        float s = hs[f][r];
#pragma unroll
                        for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
                        hs[f][r] = s;
                    }
                if ((lane & 31) == 0) {
                    float* HP = g.head_part + (int64_t)(blockIdx.y * 2 + wn) * g.M;
#pragma unroll
                    for (int f = 0; f < 2; ++f)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int row = m0 + wm * 64 + f * 32 + (r >> 2) * 8 + lrow + (r & 3);
                            if (row < g.M) HP[row] = hs[f][r];
                        }
                }
            }
        }
    }
}

// Head backward: dz3 = bf16(dy * w4 * [h3 > 0]); per block partial sums of
// dw4[n] = sum_m dy[m] h3[m][n] and db4 = sum_m dy[m].  Thread = column.
__global__ __launch_bounds__(256) void head_bwd_kernel(int M, const float* dy, const uint16_t* h3,
                                                       const uint16_t* w4, uint16_t* dz3, float* dw4_part,
                                                       float* db4_part)
{
    const int n = threadIdx.x;
    const int r0 = blockIdx.x * kHeadRows, r1 = min(M, r0 + kHeadRows);
    const float w = bf2f(w4[n]);
    float sw = 0.f, sb = 0.f;
    for (int r = r0; r < r1; ++r) {
        const float d = dy[r];
        const float h = bf2f(h3[(int64_t)r * kHid + n]);
        dz3[(int64_t)r * kHid + n] = f2bf(h > 0.f ? d * w : 0.f);
        sw += d * h;
        sb += d;
    }
    dw4_part[(int64_t)blockIdx.x * kHid + n] = sw;
    if (n == 0) db4_part[blockIdx.x] = sb;
}

// y[m] = b4 + sum of the head partials; per set s: err_s = sum_{m in s} y[m]
// - target[s], sq[s] = err_s^2, dy[m] = 2 err_s / S.  One wave per set.
// Without a target, score[s] = sum_{m in s} y[m].
__global__ __launch_bounds__(256) void set_loss_kernel(int M, int S, int nparts, const float* head_part,
                                                       const float* b4, const int64_t* seg, const float* target,
                                                       float* y, float* dy, float* sq, float* score)
{
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= S) return;
    // offsets are clamped to the rows so that bad ones cannot read out of bounds
    int64_t a = seg[s], e = seg[s + 1];
    a = a < 0 ? 0 : (a > M ? M : a);
    e = e < a ? a : (e > M ? M : e);
    float sum = 0.f;
    for (int64_t m = a + lane; m < e; m += 64) {
        float v = *b4;
        for (int p = 0; p < nparts; ++p) v += head_part[(int64_t)p * M + m];
        if (y) y[m] = v;
        sum += v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (score && lane == 0) score[s] = sum;
    if (target) {
        const float err = sum - target[s];
        if (lane == 0 && sq) sq[s] = err * err;
        const float d = 2.f * err / (float)S;
        for (int64_t m = a + lane; m < e; m += 64) dy[m] = d;
    }
}

// y[m] = b4 + the four 64-column partial sums of the head.
__global__ __launch_bounds__(256) void head_sum_kernel(int M, const float* head_part, const float* b4, float* y)
{
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    float v = *b4;
#pragma unroll
    for (int p = 0; p < 4; ++p) v += head_part[(int64_t)p * M + m];
    y[m] = v;
}

// Flat gradient from the partial sums of each product.
struct GradArgs {
    float* grad;
    const float* part1;
    const float* part2;
    const float* part3;
    const float* cs1;
    const float* cs2;
    const float* cs3;
    const float* dw4_part;
    const float* db4_part;
    int splits, head_blocks;
};

__global__ __launch_bounds__(256) void grad_reduce_kernel(GradArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= kNumParams) return;
    const float* src;
    int64_t stride, j;
    int cnt = a.splits;
    if (i < kOffB1) {
        src = a.part1, stride = (int64_t)kHid * kIn, j = i - kOffW1;
    } else if (i < kOffW2) {
        src = a.cs1, stride = kHid, j = i - kOffB1;
    } else if (i < kOffB2) {
        src = a.part2, stride = (int64_t)kHid * kHid, j = i - kOffW2;
    } else if (i < kOffW3) {
        src = a.cs2, stride = kHid, j = i - kOffB2;
    } else if (i < kOffB3) {
        src = a.part3, stride = (int64_t)kHid * kHid, j = i - kOffW3;
    } else if (i < kOffW4) {
        src = a.cs3, stride = kHid, j = i - kOffB3;
    } else if (i < kOffB4) {
        src = a.dw4_part, stride = kHid, j = i - kOffW4, cnt = a.head_blocks;
    } else {
        src = a.db4_part, stride = 1, j = 0, cnt = a.head_blocks;
    }
    float s = 0.f;
    for (int z = 0; z < cnt; ++z) s += src[z * stride + j];
    a.grad[i] = s;
}

// v <- mu v + g; p <- p - lr v; refresh the bf16 copy.
__global__ __launch_bounds__(256) void sgd_kernel(float* p, float* v, const float* g, uint16_t* pb, float lr,
                                                  float mu)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= kNumParams) return;
    const float vn = mu * v[i] + g[i];
    const float pn = p[i] - lr * vn;
    v[i] = vn;
    p[i] = pn;
    pb[i] = f2bf(pn);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* p, uint16_t* pb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) pb[i] = f2bf(p[i]);
}

__global__ __launch_bounds__(256) void fill_kernel(float* p, float v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace mlpk
}  // namespace vrprpd

using namespace vrprpd;
using namespace vrprpd::mlpk;

struct vrprpd_mlp {
    int device = 0;
    int64_t max_rows = 0;
    int max_splits = 0, max_head_blocks = 0;
    float* p = nullptr;       // fp32 master parameters (flat)
    float* v = nullptr;       // momentum
    float* grad = nullptr;    // last backward's gradient
    uint16_t* pb = nullptr;   // bf16 copy
    uint16_t* h[3] = {nullptr, nullptr, nullptr};   // hidden activations [rows][256]
    uint16_t* dz[2] = {nullptr, nullptr};           // masked upstream gradients
    const uint16_t* x = nullptr;                    // features of the last forward (caller's)
    int64_t rows = 0;                               // rows of the last forward
    float* head_part = nullptr;   // [4][rows]
    float* dy = nullptr;          // [rows]
    float* part[3] = {nullptr, nullptr, nullptr};
    float* cs[3] = {nullptr, nullptr, nullptr};
    float* dw4_part = nullptr;
    float* db4_part = nullptr;
    std::vector<void*> allocs;
};

namespace {

int mlp_alloc(vrprpd_mlp* h, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) return set_error(VRPRPD_ENOMEM, "vrprpd_mlp: hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    h->allocs.push_back(*p);
    return VRPRPD_OK;
}

template <bool kAT, bool kBT, int kEpi>
int launch_gemm(const GemmArgs& g, int splits, hipStream_t st)
{
    dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN, splits);
    hipLaunchKernelGGL((gemm_kernel<kAT, kBT, kEpi>), grid, dim3(256), 0, st, g);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

// Glorot-uniform hidden weights, U(-a, a) with a = sqrt(6 / (in + out)),
// from Philox words (counter = parameter index, tag "MLPI"); zero biases and
// a zero head, so an untrained network predicts no change for every set.
void init_params(std::vector<float>& v, uint64_t seed)
{
    const int dims[5] = {kIn, kHid, kHid, kHid, 1};
    const int64_t offW[4] = {kOffW1, kOffW2, kOffW3, kOffW4};
    std::fill(v.begin(), v.end(), 0.f);
    for (int l = 0; l < 3; ++l) {
        const double a = std::sqrt(6.0 / (dims[l] + dims[l + 1]));
        const int64_t cnt = (int64_t)dims[l] * dims[l + 1];
        for (int64_t i = 0; i < cnt; ++i) {
            const uint32_t w = philox_word(seed, (uint32_t)((offW[l] + i) & 0xFFFFFFFFu), 0, 0, 0x4D4C5049u);
            const double u = (double)(w >> 8) * (1.0 / 16777216.0);
            v[offW[l] + i] = (float)((2.0 * u - 1.0) * a);
        }
    }
}

}  // namespace

extern "C" int vrprpd_mlp_create(vrprpd_mlp** out, int64_t max_rows, const float* params, uint64_t seed)
{
    if (!out) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_create: out is NULL");
    *out = nullptr;
    if (max_rows < 1 || max_rows > (int64_t)1 << 26)
        return set_error(VRPRPD_EINVAL, "vrprpd_mlp_create: max_rows = %lld (need 1..2^26)", (long long)max_rows);
    vrprpd_mlp* h = new vrprpd_mlp;
    VRP_HIP(hipGetDevice(&h->device));
    h->max_rows = max_rows;
    h->max_splits = (int)((max_rows + kSplitRows - 1) / kSplitRows);
    h->max_head_blocks = (int)((max_rows + kHeadRows - 1) / kHeadRows);
    const size_t R = (size_t)max_rows;
    int rc = VRPRPD_OK;
    auto A = [&](void** p, size_t bytes) {
        if (rc == VRPRPD_OK) rc = mlp_alloc(h, p, bytes);
    };
    A((void**)&h->p, kNumParams * 4);
    A((void**)&h->v, kNumParams * 4);
    A((void**)&h->grad, kNumParams * 4);
    A((void**)&h->pb, kNumParams * 2);
    for (int l = 0; l < 3; ++l) A((void**)&h->h[l], R * kHid * 2);
    for (int l = 0; l < 2; ++l) A((void**)&h->dz[l], R * kHid * 2);
    A((void**)&h->head_part, 4 * R * 4);
    A((void**)&h->dy, R * 4);
    A((void**)&h->part[0], (size_t)h->max_splits * kHid * kIn * 4);
    A((void**)&h->part[1], (size_t)h->max_splits * kHid * kHid * 4);
    A((void**)&h->part[2], (size_t)h->max_splits * kHid * kHid * 4);
    for (int l = 0; l < 3; ++l) A((void**)&h->cs[l], (size_t)h->max_splits * kHid * 4);
    A((void**)&h->dw4_part, (size_t)h->max_head_blocks * kHid * 4);
    A((void**)&h->db4_part, (size_t)h->max_head_blocks * 4);
    if (rc != VRPRPD_OK) {
        vrprpd_mlp_destroy(h);
        return rc;
    }
    std::vector<float> host(kNumParams);
    if (params)
        std::memcpy(host.data(), params, kNumParams * 4);
    else
        init_params(host, seed);
    std::vector<uint16_t> hb(kNumParams);
    for (int64_t i = 0; i < kNumParams; ++i) hb[i] = f2bf(host[i]);
    hipError_t e;
    if ((e = hipMemcpy(h->p, host.data(), kNumParams * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->pb, hb.data(), kNumParams * 2, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(h->v, 0, kNumParams * 4)) != hipSuccess ||
        (e = hipMemset(h->grad, 0, kNumParams * 4)) != hipSuccess) {
        vrprpd_mlp_destroy(h);
        return hip_error(e, "vrprpd_mlp_create: upload");
    }
    *out = h;
    return VRPRPD_OK;
}

int64_t vrprpd::mlp_max_rows(const vrprpd_mlp* h) { return h ? h->max_rows : 0; }

extern "C" int vrprpd_mlp_destroy(vrprpd_mlp* h)
{
    if (!h) return VRPRPD_OK;
    for (void* p : h->allocs) (void)hipFree(p);
    delete h;
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_get_params(const vrprpd_mlp* h, float* params, float* grad, void* stream)
{
    if (!h) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_get_params: handle is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (params) VRP_HIP(hipMemcpyAsync(params, h->p, kNumParams * 4, hipMemcpyDeviceToDevice, st));
    if (grad) VRP_HIP(hipMemcpyAsync(grad, h->grad, kNumParams * 4, hipMemcpyDeviceToDevice, st));
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_set_params(vrprpd_mlp* h, const float* params, void* stream)
{
    if (!h || !params) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_set_params: NULL argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    VRP_HIP(hipMemcpyAsync(h->p, params, kNumParams * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, h->p, h->pb,
                       (int64_t)kNumParams);
    hipLaunchKernelGGL(fill_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, h->v, 0.f,
                       (int64_t)kNumParams);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_forward(vrprpd_mlp* h, int64_t rows, const uint16_t* x, float* y, void* stream)
{
    if (!h) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_forward: handle is NULL");
    if (rows < 0 || rows > h->max_rows)
        return set_error(VRPRPD_EINVAL, "vrprpd_mlp_forward: rows = %lld outside [0, %lld]", (long long)rows,
                         (long long)h->max_rows);
    if (rows > 0 && !x) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_forward: x is NULL");
    if (((uintptr_t)x & 15) != 0) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_forward: x must be 16-byte aligned");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    h->x = x;
    h->rows = rows;
    if (rows == 0) return VRPRPD_OK;
    const int M = (int)rows;
    const uint16_t* in = x;
    int64_t ld = kIn;
    const int64_t offW[3] = {kOffW1, kOffW2, kOffW3}, offB[3] = {kOffB1, kOffB2, kOffB3};
    for (int l = 0; l < 3; ++l) {
        GemmArgs g{};
        g.A = in, g.lda = ld, g.B = h->pb + offW[l], g.ldb = l == 0 ? kIn : kHid;
        g.M = M, g.N = kHid, g.K = l == 0 ? kIn : kHid, g.k_chunk = g.K;
        g.bias = h->p + offB[l], g.out = h->h[l], g.ldo = kHid;
        if (l == 2) g.head_w = h->pb + kOffW4, g.head_part = h->head_part;
        const int rc = launch_gemm<false, false, EPI_RELU>(g, 1, st);
        if (rc) return rc;
        in = h->h[l], ld = kHid;
    }
    if (y) {
        hipLaunchKernelGGL(head_sum_kernel, dim3((M + 255) / 256), dim3(256), 0, st, M, h->head_part,
                           h->p + kOffB4, y);
        VRP_HIP(hipGetLastError());
    }
    return VRPRPD_OK;
}

static int check_sets(const vrprpd_mlp* h, int32_t S, const int64_t* seg_off, const char* who)
{
    if (!h) return set_error(VRPRPD_EINVAL, "%s: handle is NULL", who);
    if (S < 1 || !seg_off) return set_error(VRPRPD_EINVAL, "%s: need num_sets >= 1 and seg_off", who);
    if (h->rows < 1) return set_error(VRPRPD_EINVAL, "%s: no forward pass with rows >= 1 before", who);
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_set_scores(vrprpd_mlp* h, int32_t num_sets, const int64_t* seg_off, float* set_score,
                                     void* stream)
{
    int rc = check_sets(h, num_sets, seg_off, "vrprpd_mlp_set_scores");
    if (rc) return rc;
    if (!set_score) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_set_scores: set_score is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(set_loss_kernel, dim3((num_sets + 3) / 4), dim3(256), 0, st, (int)h->rows, num_sets, 4,
                       h->head_part, h->p + kOffB4, seg_off, nullptr, nullptr, nullptr, nullptr, set_score);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_loss(vrprpd_mlp* h, int32_t num_sets, const int64_t* seg_off, const float* target,
                               float* sq_err, void* stream)
{
    int rc = check_sets(h, num_sets, seg_off, "vrprpd_mlp_loss");
    if (rc) return rc;
    if (!target) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_loss: target is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // rows outside every set get no gradient
    hipLaunchKernelGGL(fill_kernel, dim3((h->rows + 255) / 256), dim3(256), 0, st, h->dy, 0.f, h->rows);
    hipLaunchKernelGGL(set_loss_kernel, dim3((num_sets + 3) / 4), dim3(256), 0, st, (int)h->rows, num_sets, 4,
                       h->head_part, h->p + kOffB4, seg_off, target, nullptr, h->dy, sq_err, nullptr);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_backward(vrprpd_mlp* h, const float* dy, void* stream)
{
    if (!h) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_backward: handle is NULL");
    if (h->rows < 1) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_backward: no forward pass with rows >= 1 before");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int M = (int)h->rows;
    const int splits = (M + kSplitRows - 1) / kSplitRows;
    const int hblocks = (M + kHeadRows - 1) / kHeadRows;
    const float* d = dy ? dy : h->dy;
    hipLaunchKernelGGL(head_bwd_kernel, dim3(hblocks), dim3(256), 0, st, M, d, h->h[2], h->pb + kOffW4, h->dz[0],
                       h->dw4_part, h->db4_part);
    VRP_HIP(hipGetLastError());
    // layer l = 3, 2, 1 (index 2, 1, 0): dz of layer l sits in dz[cur]
    int cur = 0;
    const int64_t offW[3] = {kOffW1, kOffW2, kOffW3};
    for (int l = 2; l >= 0; --l) {
        const uint16_t* a_in = l == 0 ? h->x : h->h[l - 1];
        const int kin = l == 0 ? kIn : kHid;
        GemmArgs g{};
        g.A = h->dz[cur], g.lda = kHid;        // A(j, row) = dz[row][j]
        g.B = a_in, g.ldb = kin;               // B(i, row) = a[row][i]
        g.M = kHid, g.N = kin, g.K = M, g.k_chunk = kSplitRows;
        g.part = h->part[l], g.colsum = h->cs[l];
        int rc = launch_gemm<true, true, EPI_PART>(g, splits, st);
        if (rc) return rc;
        if (l > 0) {
            GemmArgs q{};
            q.A = h->dz[cur], q.lda = kHid;          // A(row, j) = dz[row][j]
            q.B = h->pb + offW[l], q.ldb = kin;      // B(i, j) = W_l[j][i]
            q.M = M, q.N = kin, q.K = kHid, q.k_chunk = kHid;
            q.mask = h->h[l - 1], q.ldm = kHid;
            q.out = h->dz[cur ^ 1], q.ldo = kHid;
            rc = launch_gemm<false, true, EPI_MASK>(q, 1, st);
            if (rc) return rc;
            cur ^= 1;
        }
    }
    GradArgs ga{h->grad, h->part[0], h->part[1], h->part[2], h->cs[0], h->cs[1], h->cs[2], h->dw4_part,
                h->db4_part, splits, hblocks};
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, ga);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_sgd_step(vrprpd_mlp* h, float lr, float momentum, void* stream)
{
    if (!h) return set_error(VRPRPD_EINVAL, "vrprpd_mlp_sgd_step: handle is NULL");
    if (!(lr >= 0.f) || !(momentum >= 0.f && momentum < 1.f))
        return set_error(VRPRPD_EINVAL, "vrprpd_mlp_sgd_step: lr = %g, momentum = %g", lr, momentum);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(sgd_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, h->p, h->v, h->grad, h->pb, lr,
                       momentum);
    VRP_HIP(hipGetLastError());
    return VRPRPD_OK;
}

extern "C" int vrprpd_mlp_hidden(const vrprpd_mlp* h, int32_t layer, uint16_t* out, void* stream)
{
    if (!h || !out || layer < 0 || layer > 4)
        return set_error(VRPRPD_EINVAL, "vrprpd_mlp_hidden: bad argument");
    if (h->rows < 1) return VRPRPD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const uint16_t* src = layer < 3 ? h->h[layer] : h->dz[layer - 3];
    VRP_HIP(hipMemcpyAsync(out, src, (size_t)h->rows * kHid * 2, hipMemcpyDeviceToDevice, st));
    return VRPRPD_OK;
}
