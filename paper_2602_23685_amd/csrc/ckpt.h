// Checkpoint blobs of the search states: a fixed header written by the
// caller, then a list of device arrays copied back to back into a host
// buffer.  Saving and loading order themselves on the caller's stream and
// return after the copies are complete.
#pragma once

#include <cstring>
#include <vector>

#include "common.h"

namespace vrprpd {

struct DevField {
    void* dev;
    size_t bytes;
};

inline size_t fields_bytes(const std::vector<DevField>& f)
{
    size_t b = 0;
    for (const DevField& x : f) b += x.bytes;
    return b;
}

// Writes head (head_bytes) and then every field into buf.  With buf NULL
// only *bytes is set.  EINVAL when capacity is too small.
inline int ckpt_save(const void* head, size_t head_bytes, const std::vector<DevField>& f, void* buf,
                     int64_t capacity, int64_t* bytes, hipStream_t st, const char* who)
{
    const size_t total = head_bytes + fields_bytes(f);
    if (bytes) *bytes = (int64_t)total;
    if (!buf) return VRPRPD_OK;
    if (capacity < (int64_t)total)
        return set_error(VRPRPD_EINVAL, "%s: buffer holds %lld bytes, the checkpoint needs %zu", who,
                         (long long)capacity, total);
    unsigned char* out = static_cast<unsigned char*>(buf);
    std::memcpy(out, head, head_bytes);
    size_t off = head_bytes;
    for (const DevField& x : f) {
        VRP_HIP(hipMemcpyAsync(out + off, x.dev, x.bytes, hipMemcpyDeviceToHost, st));
        off += x.bytes;
    }
    VRP_HIP(hipStreamSynchronize(st));
    return VRPRPD_OK;
}

// Copies the fields back from buf (whose header the caller has checked).
inline int ckpt_load(const void* buf, int64_t bytes, size_t head_bytes, const std::vector<DevField>& f,
                     hipStream_t st, const char* who)
{
    const size_t total = head_bytes + fields_bytes(f);
    if (bytes != (int64_t)total)
        return set_error(VRPRPD_EINVAL, "%s: checkpoint has %lld bytes, this state's needs %zu", who,
                         (long long)bytes, total);
    const unsigned char* in = static_cast<const unsigned char*>(buf);
    size_t off = head_bytes;
    VRP_HIP(hipStreamSynchronize(st));
    for (const DevField& x : f) {
        VRP_HIP(hipMemcpyAsync(x.dev, in + off, x.bytes, hipMemcpyHostToDevice, st));
        off += x.bytes;
    }
    VRP_HIP(hipStreamSynchronize(st));
    return VRPRPD_OK;
}

}  // namespace vrprpd
