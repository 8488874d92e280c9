// fm_bench.hip -- LDS read-bandwidth probe for the benchmark (not part of the
// rendering path).  Two access patterns:
//   mode 0: every lane reads its own 16-byte word, consecutive lanes
//           consecutive words (ds_read_b128 without bank conflicts): the
//           LDS data rate of the compute unit;
//   mode 1: all lanes of a wave read the same 16-byte word (a broadcast),
//           the pattern in which the blend kernels read staged records.
// Each thread accumulates what it reads and stores one float, so the reads
// cannot be dropped.
#include "fm_internal.h"

namespace fm {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 2048;  // 32 KiB of float4 in LDS: five workgroups per CU

template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(int iters, float *__restrict__ sink) {
    __shared__ float4 buf[kProbeWords];
    for (int i = threadIdx.x; i < kProbeWords; i += kProbeThreads)
        buf[i] = make_float4((float)i, 1.f, 2.f, 3.f);
    __syncthreads();
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const int wave = threadIdx.x >> 6;
    int idx = MODE == 0 ? (int)threadIdx.x : wave * 64;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 v = buf[(idx + u * 256) & (kProbeWords - 1)];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        idx = (idx + 576) & (kProbeWords - 1);
    }
    sink[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

hipError_t launch_lds_probe(int mode, int blocks, int iters, float *sink, hipStream_t st) {
    if (mode == 0)
        hipLaunchKernelGGL(k_lds_probe<0>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, sink);
    else
        hipLaunchKernelGGL(k_lds_probe<1>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, sink);
    return hipGetLastError();
}

int64_t lds_probe_bytes(int blocks, int iters) { return (int64_t)blocks * kProbeThreads * iters * 8 * 16; }

}  // namespace fm
