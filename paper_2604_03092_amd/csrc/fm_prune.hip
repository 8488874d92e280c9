// fm_prune.hip -- removal of the primitives that map fusion prunes (Sec. 3.3,
// "Map Fusion"): the surfels whose error-attributed score exceeds a cut are
// dropped and the others are written, in their original order, to the
// output planes.  Three launches: per-chunk counts of kept surfels, one
// exclusive scan of the chunk counts, and the scatter (a block-wide scan of
// each chunk, then 13 floats per kept surfel).
#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

constexpr int kChunk = 1024;  // surfels per block of the count and scatter kernels

// Kept when the score does not exceed the cut (a NaN score is kept, the
// comparison being false).
__device__ __forceinline__ bool kept(const float *score, int64_t i, float tau) { return !(score[i] > tau); }

__global__ __launch_bounds__(kChunk) void k_prune_count(const float *__restrict__ score, int64_t n, float tau,
                                                         uint32_t *__restrict__ chunk) {
    __shared__ uint32_t wsum[kChunk / 64];
    const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    const bool k = i < n && kept(score, i, tau);
    const uint32_t c = (uint32_t)__popcll(ballot64(k));
    if (lane_id() == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kChunk / 64; ++w) t += wsum[w];
        chunk[blockIdx.x] = t;
    }
}

// Exclusive scan of the chunk counts in place (one block); *count receives
// the number of kept surfels.
__global__ __launch_bounds__(1024) void k_prune_scan(uint32_t *__restrict__ chunk, int nc,
                                                      int32_t *__restrict__ count) {
    __shared__ uint32_t part[1024];
    const int per = (nc + 1023) / 1024;
    const int beg = threadIdx.x * per, end = beg + per < nc ? beg + per : nc;
    uint32_t s = 0;
    for (int i = beg; i < end; ++i) s += chunk[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = beg; i < end; ++i) {
        const uint32_t c = chunk[i];
        chunk[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *count = (int32_t)part[1023];
}

__global__ __launch_bounds__(kChunk) void k_prune_write(fm_surfels in, const float *__restrict__ score, float tau,
                                                         const uint32_t *__restrict__ chunk_off,
                                                         fm_surfel_buffer out) {
    __shared__ uint32_t wsum[kChunk / 64];
    const int64_t n = in.n;
    const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    const bool k = i < n && kept(score, i, tau);
    const uint64_t b = ballot64(k);
    const int lane = lane_id(), w = (int)threadIdx.x >> 6;
    if (lane == 0) wsum[w] = (uint32_t)__popcll(b);
    __syncthreads();
    if (!k) return;
    uint32_t o = chunk_off[blockIdx.x] + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    for (int j = 0; j < w; ++j) o += wsum[j];
    const int64_t C = out.capacity;
    if ((int64_t)o >= C) return;
    out.mean[o] = in.mean[i];
    out.mean[C + o] = in.mean[n + i];
    out.mean[2 * C + o] = in.mean[2 * n + i];
    out.quat[o] = in.quat[i];
    out.quat[C + o] = in.quat[n + i];
    out.quat[2 * C + o] = in.quat[2 * n + i];
    out.quat[3 * C + o] = in.quat[3 * n + i];
    out.scale[o] = in.scale[i];
    out.scale[C + o] = in.scale[n + i];
    out.opacity[o] = in.opacity[i];
    out.color[o] = in.color[i];
    out.color[C + o] = in.color[n + i];
    out.color[2 * C + o] = in.color[2 * n + i];
}

int64_t chunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

}  // namespace

size_t prune_compact_workspace_bytes(int64_t n) { return (size_t)(chunks(n) > 0 ? chunks(n) : 1) * 4; }

hipError_t launch_prune_compact(const fm_surfels &in, const float *score, float tau, const fm_surfel_buffer &out,
                                int32_t *count, void *ws, hipStream_t st) {
    const int64_t nc = chunks(in.n);
    uint32_t *chunk = static_cast<uint32_t *>(ws);
    if (nc == 0) {
        hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, st, chunk, 0, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_prune_count, dim3((unsigned)nc), dim3(kChunk), 0, st, score, (int64_t)in.n, tau, chunk);
    hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, st, chunk, (int)nc, count);
    hipLaunchKernelGGL(k_prune_write, dim3((unsigned)nc), dim3(kChunk), 0, st, in, score, tau, chunk, out);
    return hipGetLastError();
}

}  // namespace fm
