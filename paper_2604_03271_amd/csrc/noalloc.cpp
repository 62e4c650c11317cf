// noalloc.cpp -- smc_kernel_resample_noalloc: systematic resampling for callers that
// cannot allocate device memory.  The same kernels as smc_kernel_resample, with the
// descriptor, the group state, the integer CDF and the stage scratch in `scratch`, a static
// device array (one copy per GPU, held until the process ends).  Host code never passes
// the array's name to a kernel or a copy: the address of this GPU's copy comes from
// hipGetSymbolAddress, once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_common.hpp"

using namespace smc;

namespace {
constexpr int kNoallocMaxP = SMC_NOALLOC_MAX_P;
constexpr size_t al256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }
constexpr size_t kNoallocChunks = (kNoallocMaxP + kStageChunk - 1) / kStageChunk;
constexpr size_t kNoallocBytes =
    al256(sizeof(GroupDesc)) + al256(sizeof(GroupState)) + al256(sizeof(unsigned long long) * kNoallocMaxP) +
    al256(sizeof(double) * 2 * kNoallocChunks * kStagePartVals) + al256(sizeof(StageNewton) * 2) +
    al256(sizeof(unsigned long long) * kNoallocChunks);
constexpr int kNoallocMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first call per device).
smc_status noalloc_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoallocMaxDevices) return SMC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SMC_EDEVICE;
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return SMC_OK;
}

// The descriptor and a cleared group state, written by a kernel from its by-value arguments
// (no host buffer, no memset).
__global__ void k_put_group(GroupDesc g, GroupDesc* dst) {
    *dst = g;
    *g.st = GroupState{};
}
}  // namespace

extern "C" smc_status smc_kernel_resample_noalloc(const double* weights, int32_t P, int32_t M, uint32_t r,
                                                  int32_t* ancestors, void* stream) {
    if (!weights || !ancestors || P < 1 || M < 1 || P > kNoallocMaxP) return SMC_EINVAL;
    if (!device_ok()) return SMC_EDEVICE;
    void* base = nullptr;
    smc_status st = noalloc_scratch(&base);
    if (st != SMC_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a{base, kNoallocBytes, 0};
    GroupDesc* d_group = static_cast<GroupDesc*>(a.take(sizeof(GroupDesc)));
    GroupDesc g{};
    g.st = static_cast<GroupState*>(a.take(sizeof(GroupState)));
    g.cdf = static_cast<unsigned long long*>(a.take(sizeof(unsigned long long) * P));
    if (!d_group || !g.st || !g.cdf || !carve_stage_scratch(a, P, g)) return SMC_EINVAL;
    g.P = P;
    g.M = M;
    g.n_moves = 1;
    g.max_stages = 1;
    if (hipMemcpyAsync(g.cdf, weights, sizeof(double) * P, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMC_EDEVICE;
    hipLaunchKernelGGL(k_put_group, dim3(1), dim3(1), 0, s, g, d_group);
    if (hipGetLastError() != hipSuccess || launch_resample_hook(d_group, P, M, r, ancestors, s) != hipSuccess)
        return SMC_EDEVICE;
    return SMC_OK;
}
