// Instance sets and error reporting of the C-ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.h"

namespace vrprpd {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_error(hipError_t e, const char* what)
{
    return set_error(e == hipErrorOutOfMemory ? VRPRPD_ENOMEM : VRPRPD_EHIP, "%s: %s", what,
                     hipGetErrorString(e));
}

}  // namespace vrprpd

using namespace vrprpd;

extern "C" const char* vrprpd_last_error(void) { return g_last_error.c_str(); }

extern "C" int vrprpd_set_create(vrprpd_set** out, int32_t num_inst, const vrprpd_instance_desc* desc)
{
    if (!out) return set_error(VRPRPD_EINVAL, "vrprpd_set_create: out is NULL");
    *out = nullptr;
    if (num_inst < 1 || !desc) return set_error(VRPRPD_EINVAL, "vrprpd_set_create: need num_inst >= 1 and desc");
    auto* s = new vrprpd_set();
    s->num_inst = num_inst;
    s->host.resize(num_inst);
    int64_t dsz = 0, psz = 0;
    for (int i = 0; i < num_inst; ++i) {
        const vrprpd_instance_desc& D = desc[i];
        if (D.n < 1 || D.n > kMaxN || D.m < 1 || D.m > kMaxM || D.k < 1 || D.R < 0 ||
            (D.load_model != VRPRPD_MIN_PRELOAD && D.load_model != VRPRPD_FULL_START) || !D.dist ||
            !D.proc) {
            delete s;
            return set_error(VRPRPD_EINVAL,
                             "instance %d: need 1<=n<=%d, 1<=m<=%d, k>=1, R>=0, a load model and host "
                             "dist/proc (got n=%d m=%d k=%d R=%d)",
                             i, kMaxN, kMaxM, D.n, D.m, D.k, D.R);
        }
        const int64_t N1 = D.n + 1;
        int64_t dmax = 0, psum = 0;
        for (int64_t a = 0; a < N1; ++a)
            for (int64_t b = 0; b < N1; ++b) {
                const int32_t x = D.dist[a * N1 + b];
                if (x < 0 || (a == b && x != 0)) {
                    delete s;
                    return set_error(VRPRPD_EINVAL, "instance %d: d[%lld][%lld] = %d (need >= 0, zero diagonal)",
                                     i, (long long)a, (long long)b, x);
                }
                if (x > dmax) dmax = x;
            }
        if (D.proc[0] != 0) {
            delete s;
            return set_error(VRPRPD_EINVAL, "instance %d: proc[0] must be 0", i);
        }
        for (int64_t c = 1; c < N1; ++c) {
            if (D.proc[c] < 0) {
                delete s;
                return set_error(VRPRPD_EINVAL, "instance %d: proc[%lld] < 0", i, (long long)c);
            }
            psum += D.proc[c];
        }
        // A longest path in the op graph has at most one incoming edge per op
        // (a travel time or a processing time) plus the return leg.
        if ((2 * (int64_t)D.n + 1) * dmax + psum >= (int64_t)INT32_MAX - 1) {
            delete s;
            return set_error(VRPRPD_ERANGE, "instance %d: (2n+1)*max d + sum p = %lld overflows int32 times", i,
                             (long long)((2 * (int64_t)D.n + 1) * dmax + psum));
        }
        const int64_t tb = (2 * (int64_t)D.n + 1) * dmax + psum;
        if (tb > s->time_bound) s->time_bound = tb;
        if (dmax > 65535) s->dist16 = 0;
        int ashift = 0;
        while ((dmax >> ashift) >= (1 << 14)) ++ashift;
        InstDev& h = s->host[i];
        h = InstDev{D.n, D.m, D.k, D.R, D.load_model, ashift, dsz, psz};
        dsz += N1 * N1;
        psz += (N1 + 3) & ~int64_t(3);   // 16-byte aligned rows: kernels read p in int4 vectors
        if (D.n > s->n_max) s->n_max = D.n;
        if (D.m > s->m_max) s->m_max = D.m;
        if (D.n != desc[0].n || D.m != desc[0].m) s->uniform_nm = false;
    }
    // Pack on the host, then one copy per buffer.
    const size_t esz = s->dist16 ? 2 : 4;
    std::vector<unsigned char> dbuf(dsz * esz);
    std::vector<int32_t> pbuf(psz);
    for (int i = 0; i < num_inst; ++i) {
        const InstDev& h = s->host[i];
        const int64_t N1 = h.n + 1;
        for (int64_t e = 0; e < N1 * N1; ++e) {
            if (s->dist16)
                reinterpret_cast<uint16_t*>(dbuf.data())[h.d_off + e] = (uint16_t)desc[i].dist[e];
            else
                reinterpret_cast<int32_t*>(dbuf.data())[h.d_off + e] = desc[i].dist[e];
        }
        std::memcpy(pbuf.data() + h.p_off, desc[i].proc, N1 * sizeof(int32_t));
    }
    hipError_t e;
    if ((e = hipGetDevice(&s->device)) != hipSuccess ||
        (e = hipMalloc(&s->d_dist, dbuf.size())) != hipSuccess ||
        (e = hipMalloc(&s->d_proc, pbuf.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&s->d_inst, s->host.size() * sizeof(InstDev))) != hipSuccess ||
        (e = hipMemcpy(s->d_dist, dbuf.data(), dbuf.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->d_proc, pbuf.data(), pbuf.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(s->d_inst, s->host.data(), s->host.size() * sizeof(InstDev), hipMemcpyHostToDevice)) !=
            hipSuccess) {
        vrprpd_set_destroy(s);
        return hip_error(e, "vrprpd_set_create");
    }
    *out = s;
    return VRPRPD_OK;
}

extern "C" int vrprpd_set_destroy(vrprpd_set* s)
{
    if (!s) return VRPRPD_OK;
    if (s->d_dist) (void)hipFree(s->d_dist);
    if (s->d_proc) (void)hipFree(s->d_proc);
    if (s->d_inst) (void)hipFree(s->d_inst);
    delete s;
    return VRPRPD_OK;
}

extern "C" int vrprpd_set_info(const vrprpd_set* s, int32_t* num_inst, int32_t* n_max, int32_t* m_max,
                               int32_t* dist16)
{
    if (!s) return set_error(VRPRPD_EINVAL, "vrprpd_set_info: set is NULL");
    if (num_inst) *num_inst = s->num_inst;
    if (n_max) *n_max = s->n_max;
    if (m_max) *m_max = s->m_max;
    if (dist16) *dist16 = s->dist16;
    return VRPRPD_OK;
}
