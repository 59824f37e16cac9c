// Bandwidth probes: a streaming copy and a streaming read of a device buffer,
// timed by the caller; the measured HBM ceilings reported beside the 8 TB/s
// peak when the recurrence's bandwidth is rated (Sec. 2.4's sparse products
// are memory-bound).  Each thread keeps four 16-byte loads in flight; the read
// folds what it loads into one word per workgroup so no load is dead.
#include "common.hpp"

namespace tbk {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;
constexpr int kProbeBlocksPerCu = 8;

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const u32x4 *__restrict__ src,
                                                              u32x4 *__restrict__ dst, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * kProbeThreads * kProbeUnroll;
    for (int64_t i0 = (int64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x; i0 < n; i0 += step) {
        u32x4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kProbeThreads;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kProbeThreads;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const u32x4 *__restrict__ src, int64_t n,
                                                              uint32_t *__restrict__ out) {
    __shared__ uint32_t red[kProbeThreads];
    const int64_t step = (int64_t)gridDim.x * kProbeThreads * kProbeUnroll;
    uint32_t acc = 0;
    for (int64_t i0 = (int64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x; i0 < n; i0 += step) {
        u32x4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kProbeThreads;
            v[u] = i < n ? __builtin_nontemporal_load(src + i) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kProbeThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace
}  // namespace tbk

using namespace tbk;

extern "C" tbk_status tbk_bandwidth_probe(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream) {
    clear_error();
    TBK_CHECK(mode == 0 || mode == 1, TBK_ERR_INVALID_ARG, "mode must be 0 (read) or 1 (copy)");
    TBK_CHECK(bytes >= 16 && bytes % 16 == 0, TBK_ERR_INVALID_ARG, "bytes = %lld: a positive multiple of 16",
              (long long)bytes);
    TBK_CHECK(src && dst, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0, TBK_ERR_INVALID_ARG,
              "src and dst must be 16-byte aligned");
    int dev = 0, cus = 0;
    TBK_HIP(hipGetDevice(&dev));
    TBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t n = bytes / 16;
    const int64_t want = ceil_div(n, (int64_t)kProbeThreads * kProbeUnroll);
    const unsigned G = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * kProbeBlocksPerCu));
    hipStream_t s = as_stream(stream);
    if (mode == 1)
        k_probe_copy<<<G, kProbeThreads, 0, s>>>(static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n);
    else
        k_probe_read<<<G, kProbeThreads, 0, s>>>(static_cast<const u32x4 *>(src), n, static_cast<uint32_t *>(dst));
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" int64_t tbk_bandwidth_probe_words(void) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return (int64_t)cus * kProbeBlocksPerCu;
}
