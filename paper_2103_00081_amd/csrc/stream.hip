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

// One 16-byte word per thread, one short-lived block per 4 KiB (measured
// on MI355X over 1 GiB: 6.2 TB/s, against 4.2-5.1 TB/s for grid-stride
// loops of 1024-16384 blocks with 1-8 words per thread and iteration); the
// tail below 16 bytes is copied bytewise by the first threads.
__global__ __launch_bounds__(256) void k_stream_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                     int64_t n16, const uint8_t *__restrict__ s8,
                                                     uint8_t *__restrict__ d8, int64_t tail0, int64_t nbytes)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
    if (i < nbytes - tail0) d8[tail0 + i] = s8[tail0 + i];
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
        const int64_t blocks = std::max<int64_t>(1, (n16 + 255) / 256);
        if (blocks > INT32_MAX) throw Error(HTS_ERR_ARG, "copy too large");
        const unsigned grid = (unsigned)blocks;
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
