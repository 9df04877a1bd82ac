// probe.hip -- attainable HBM bandwidth of the device: a plain copy kernel of known size,
// the denominator the step's achieved bandwidth is compared with besides the vendor peak.
//
// Each lane moves 16 bytes per access (buffer-width vector loads), several accesses in
// flight per lane, with the non-temporal cache policy on loads and stores: the copy streams
// through L2 without keeping lines, as the populations do in the single-pass step. A few
// launch shapes are timed with HIP events and the fastest is reported.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm2p.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ __launch_bounds__(256) void k_copy(const f4 *__restrict__ src, f4 *__restrict__ dst, long long m) {
    const long long stride = (long long)gridDim.x * 256;
    long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    for (; k + (U - 1) * stride < m; k += U * stride) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + k + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + k + u * stride);
    }
    for (; k < m; k += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

struct Shape {
    int unroll, blocks;
};
constexpr Shape kShapes[] = {{1, 1024}, {2, 512}, {2, 1024}, {4, 512}, {1, 4096}};

void launch(const Shape &sh, hipStream_t s, const f4 *src, f4 *dst, long long m) {
    switch (sh.unroll) {
    case 1: hipLaunchKernelGGL(k_copy<1>, dim3(sh.blocks), dim3(256), 0, s, src, dst, m); break;
    case 2: hipLaunchKernelGGL(k_copy<2>, dim3(sh.blocks), dim3(256), 0, s, src, dst, m); break;
    default: hipLaunchKernelGGL(k_copy<4>, dim3(sh.blocks), dim3(256), 0, s, src, dst, m); break;
    }
}

}  // namespace

extern "C" int lbm_copy_probe(void *dst, const void *src, int64_t bytes, int reps, void *hip_stream, double out[3]) {
    if (!dst || !src || !out || bytes < 16 || bytes % 16 || reps < 1) return LBM_E_INVAL;
    const hipStream_t s = (hipStream_t)hip_stream;
    const long long m = bytes / 16;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_E_HIP;
    }
    double best_ms = 0.0;
    int best = -1;
    int rc = LBM_OK;
    for (int i = 0; i < (int)(sizeof(kShapes) / sizeof(kShapes[0])) && rc == LBM_OK; ++i) {
        launch(kShapes[i], s, (const f4 *)src, (f4 *)dst, m);   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = LBM_E_HIP; break; }
        for (int r = 0; r < reps; ++r) launch(kShapes[i], s, (const f4 *)src, (f4 *)dst, m);
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) {
            rc = LBM_E_HIP;
            break;
        }
        const double per = ms / reps;
        if (best < 0 || per < best_ms) {
            best_ms = per;
            best = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    out[0] = 2.0 * (double)bytes / (best_ms * 1e-3) / 1e9;   // GB/s, bytes read + written
    out[1] = best_ms;
    out[2] = (double)(kShapes[best].unroll * 100000 + kShapes[best].blocks);
    return LBM_OK;
}
