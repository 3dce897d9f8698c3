// noalloc.hip -- qpm_eval_fitness_noalloc: the fitness of a population
// (qpm_eval_fitness) for callers that cannot allocate device memory (code
// under stream capture, tight serving loops, harnesses that forbid
// hipMalloc). Its segment partials live in a fixed device array of this
// file instead of per-call or per-design scratch.
#include <mutex>

#include "common.hpp"

namespace qpm {

constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;  // 16 MiB per device

// The segment partials of every call on a device: each device that runs the
// library holds its own copy until the process ends. Host code reaches it
// only through the per-device address from hipGetSymbolAddress (the name
// itself is a host-side stand-in). Every partial a call reads was written
// by the same call, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The address of this device's copy of `scratch`, looked up once per device
// with that device current.
qpm_status scratch_address(void **out)
{
    int dev = 0;
    QPM_TRY_HIP(hipGetDevice(&dev));
    QPM_REQUIRE(dev >= 0 && dev < kMaxDevices, QPM_ENOTSUP, "device %d is beyond the %d supported", dev,
                kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hipGetSymbolAddress of the fitness scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return QPM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QPM_OK;
}

}  // namespace

}  // namespace qpm

using namespace qpm;

QPM_API qpm_status qpm_eval_fitness_noalloc(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                            void *fitness, int32_t kernel, qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(kernel == QPM_FIT_AUTO || kernel == QPM_FIT_SEGMENTED || kernel == QPM_FIT_PER_GENOME ||
                    kernel == QPM_FIT_TABLE,
                QPM_EINVAL, "unknown fitness kernel %d", (int)kernel);
    QPM_REQUIRE(!(kernel == QPM_FIT_PER_GENOME && p != QPM_PREC_F64), QPM_EINVAL,
                "the per-genome kernel computes in FP64 only");
    QPM_REQUIRE(d && bits && fitness, QPM_EINVAL, "design, bits and fitness must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(np >= 1, QPM_EINVAL, "np must be >= 1 (got %lld)", (long long)np);
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np (%lld) and a multiple of 64",
                (long long)ld, (long long)np);
    QPM_REQUIRE((reinterpret_cast<uintptr_t>(bits) & 3u) == 0, QPM_EINVAL, "bits must be 4-byte aligned");
    QPM_REQUIRE(np <= (int64_t(1) << 31) && d->words * ld <= (int64_t(1) << 40), QPM_ERANGE,
                "population too large");
    const FitPlan pl = plan_fitness(*d, p, np, kernel);
    QPM_REQUIRE(pl.gy <= 65535, QPM_ERANGE, "too many workgroup segments (%d)", pl.gy);
    const size_t bytes = fitness_workspace_bytes(pl, ld);
    QPM_REQUIRE(bytes <= kNoAllocScratchBytes, QPM_ERANGE,
                "this population needs %zu bytes of segment partials, more than the %zu of the fixed scratch "
                "(use qpm_eval_fitness)",
                bytes, kNoAllocScratchBytes);
    void *ws = nullptr;
    if (bytes > 0) {
        const qpm_status st = scratch_address(&ws);
        if (st != QPM_OK) return st;
    }
    return launch_fitness(*d, p, bits, np, ld, fitness, pl, static_cast<double *>(ws), static_cast<hipStream_t>(sv));
}
