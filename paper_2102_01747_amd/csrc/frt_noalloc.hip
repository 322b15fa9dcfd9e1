// frt_noalloc.hip -- the library's own device scratch for callers that cannot
// allocate (frt_render_batch_noalloc), and the argument-carried upload that
// fills it without a staging buffer.
//
// `scratch` is a file-scope device array: every GPU the library runs on
// holds its own copy, at its own address, for the life of the process.  In
// host code the array's name is only a host-side stand-in, so the address
// kernels are given is looked up with hipGetSymbolAddress once per device
// (with that device current) and kept; the name itself is never passed to a
// kernel, a copy or a fill.
#include <hip/hip_runtime.h>

#include <mutex>

#include "frt_internal.hpp"

namespace frt {
namespace {

// header + FRT_NOALLOC_MAX_JOBS jobs, laid out as frt_workspace_bytes() does
constexpr size_t kScratchBytes =
    (sizeof(WorkspaceHeader) + size_t(FRT_NOALLOC_MAX_JOBS) * kWorkspaceBytesPerJob + 255) / 256 * 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

struct alignas(16) UploadArgs {
    uint4* dst;
    int words;          // 16-byte words to write
    int pad[3];
    uint4 data[kUploadBytes / 16];
};

// One thread per 16-byte word; the payload travels in the kernel arguments.
__global__ void __launch_bounds__(256) upload_kernel(const UploadArgs a) {
    for (int i = threadIdx.x; i < a.words; i += blockDim.x) a.dst[i] = a.data[i];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void* noalloc_scratch(hipError_t& err) {
    err = hipSuccess;
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p) {
            if (err == hipSuccess) err = hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

hipError_t launch_upload(void* dst, const void* src, int bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    if (bytes > kUploadBytes || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return hipErrorInvalidValue;
    UploadArgs a;
    a.dst = static_cast<uint4*>(dst);
    a.words = bytes / 16;
    a.pad[0] = a.pad[1] = a.pad[2] = 0;
    __builtin_memcpy(a.data, src, size_t(bytes));
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace frt
