// A plain streaming copy: the achievable HBM bandwidth reference next to
// which the operator kernels are measured, and the kernel of known traffic
// that scales the hardware byte counters.
#include <functional>

#include "common.h"
#include "hts.h"

namespace hts {
hts_status guard_call(const std::function<void()> &f);

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// 16-byte vector loads and stores, four per thread per pass, grid-stride
// over the whole buffer (n16 16-byte words); the tail below 16 bytes is
// copied bytewise by the first threads.
__global__ __launch_bounds__(256) void k_stream_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                     int64_t n16, const uint8_t *__restrict__ s8,
                                                     uint8_t *__restrict__ d8, int64_t tail0, int64_t nbytes)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const v4u a = __builtin_nontemporal_load(src + i);
        const v4u b = __builtin_nontemporal_load(src + i + stride);
        const v4u c = __builtin_nontemporal_load(src + i + 2 * stride);
        const v4u d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nbytes - tail0) d8[tail0 + t] = s8[tail0 + t];
}

}  // namespace
}  // namespace hts

using namespace hts;

extern "C" hts_status hts_stream_copy(const void *src, void *dst, int64_t bytes, int32_t reps, void *stream,
                                      double *ms_per_copy)
{
    return guard_call([&] {
        if (bytes < 0 || reps < 0 || (bytes > 0 && (!src || !dst))) throw Error(HTS_ERR_ARG, "bad arguments");
        if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
            throw Error(HTS_ERR_ARG, "buffers must be 16-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        const int64_t n16 = bytes / 16;
        int dev = 0, ncu = 0;
        HTS_HIP(hipGetDevice(&dev));
        HTS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        // enough 256-thread blocks for 16 waves per compute unit
        const int64_t want = (int64_t)std::max(ncu, 1) * 16;
        const int64_t need = std::max<int64_t>(1, (n16 + 255) / 256);
        const unsigned grid = (unsigned)std::min(want, need);
        hipEvent_t a = nullptr, b = nullptr;
        HTS_HIP(hipEventCreate(&a));
        HTS_HIP(hipEventCreate(&b));
        auto launch = [&] {
            k_stream_copy<<<dim3(grid), dim3(256), 0, s>>>(static_cast<const v4u *>(src), static_cast<v4u *>(dst),
                                                           n16, static_cast<const uint8_t *>(src),
                                                           static_cast<uint8_t *>(dst), n16 * 16, bytes);
            HTS_LAUNCH_CHECK();
        };
        try {
            if (bytes > 0) launch();   // untimed first pass
            HTS_HIP(hipEventRecord(a, s));
            for (int r = 0; r < reps && bytes > 0; r++) launch();
            HTS_HIP(hipEventRecord(b, s));
            HTS_HIP(hipEventSynchronize(b));
            float ms = 0.0f;
            HTS_HIP(hipEventElapsedTime(&ms, a, b));
            if (ms_per_copy) *ms_per_copy = reps > 0 ? (double)ms / reps : 0.0;
        } catch (...) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            throw;
        }
        HTS_HIP(hipEventDestroy(a));
        HTS_HIP(hipEventDestroy(b));
    });
}
