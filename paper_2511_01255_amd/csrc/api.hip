// api.hip -- status strings, per-thread error text, device check.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "common.hpp"

namespace qpm {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

qpm_status check_device()
{
    int dev = 0;
    QPM_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QPM_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
        return QPM_ENOTSUP;
    }
    return QPM_OK;
}

struct ScratchCache {
    struct Slot {
        hipStream_t s = nullptr;
        void *p = nullptr;
        size_t bytes = 0;
        bool taken = false;
    };
    std::mutex m;
    Slot slot[kScratchSlots];
};

ScratchCache *scratch_cache_create() { return new (std::nothrow) ScratchCache(); }

void scratch_cache_destroy(ScratchCache *c)
{
    if (!c) return;
    bool any = false;
    for (auto &sl : c->slot) any = any || sl.p != nullptr;
    // the last uses were enqueued on streams that may be gone by now
    if (any) (void)hipDeviceSynchronize();
    for (auto &sl : c->slot)
        if (sl.p) (void)hipFree(sl.p);
    delete c;
}

qpm_status ScratchLease::begin(size_t bytes, void **p)
{
    *p = nullptr;
    if (bytes == 0) return QPM_OK;
    // a slot belongs to one stream handle for the cache's lifetime; uses on
    // one stream are ordered by the stream. A handle value can come back
    // for a new stream only after hipStreamDestroy, which drains the old
    // stream's work first, so the new stream's uses cannot overlap the old.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusActive;
    if (hipStreamIsCapturing(s_, &cap) != hipSuccess) {
        // unknown: take the allocator (the call's own launches report
        // whatever is wrong with the stream)
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;
    }
    if (c_ != nullptr && cap == hipStreamCaptureStatusNone) {
        c_->m.lock();
        locked_ = true;
        int k = -1;
        for (int j = 0; j < kScratchSlots && k < 0; ++j)
            if (c_->slot[j].taken && c_->slot[j].s == s_) k = j;
        for (int j = 0; j < kScratchSlots && k < 0; ++j)
            if (!c_->slot[j].taken) k = j;
        if (k >= 0) {
            auto &sl = c_->slot[k];
            if (sl.bytes < bytes) {
                // grow: the old buffer's uses (all on this stream) end first
                if (sl.p) {
                    const hipError_t e = hipStreamSynchronize(s_);
                    if (e != hipSuccess) {
                        end();
                        set_error("hipStreamSynchronize failed: %s", hipGetErrorString(e));
                        return QPM_EHIP;
                    }
                    (void)hipFree(sl.p);
                    sl.p = nullptr;
                    sl.bytes = 0;
                }
                const hipError_t e = hipMalloc(&sl.p, bytes);
                if (e != hipSuccess) {
                    sl.p = nullptr;
                    end();
                    set_error("scratch allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
                    return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
                }
                sl.bytes = bytes;
            }
            sl.s = s_;
            sl.taken = true;
            *p = sl.p;
            return QPM_OK;
        }
        c_->m.unlock();
        locked_ = false;
    }
    QPM_TRY_HIP(hipMallocAsync(&owned_, bytes, s_));
    *p = owned_;
    return QPM_OK;
}

qpm_status ScratchLease::end()
{
    qpm_status st = QPM_OK;
    if (locked_) {
        c_->m.unlock();
        locked_ = false;
    }
    if (owned_) {
        const hipError_t e = hipFreeAsync(owned_, s_);
        owned_ = nullptr;
        if (e != hipSuccess) {
            set_error("hipFreeAsync failed: %s", hipGetErrorString(e));
            st = QPM_EHIP;
        }
    }
    return st;
}

}  // namespace qpm

QPM_API const char *qpm_status_string(qpm_status s)
{
    switch (s) {
    case QPM_OK: return "ok";
    case QPM_EINVAL: return "invalid argument";
    case QPM_ERANGE: return "size out of range";
    case QPM_ENOMEM: return "out of device memory";
    case QPM_EHIP: return "HIP runtime error";
    case QPM_ENOTSUP: return "unsupported device";
    default: return "unknown status";
    }
}

QPM_API const char *qpm_last_error(void) { return qpm::g_last_error; }
