// fm_warp.hip -- loop correction of the map (Sec. 3.3): every primitive is
// bound to the keyframe that created it; when loop closure moves keyframes,
// each bound primitive is moved by its keyframe's Delta T = T_new T_old^-1,
// a similarity (s, q, t): mu <- s R(q) mu + t, r <- q r, scales <- s scales.
// One thread per primitive; the keyframes' transforms (rotation matrices
// formed once per workgroup into LDS) are read from a device array, so the
// call is graph-capturable.
#include "fm_internal.h"

namespace fm {

namespace {

constexpr int kWarpLds = 256;  // keyframe transforms staged in LDS per workgroup (17 KB)

struct Sim3x {
    float s, R[9], q[4], t[3];
};

__device__ __forceinline__ Sim3x make_sim(const fm_sim3 &d) {
#pragma clang fp contract(off)
    Sim3x x;
    const float n = sqrtf(d.q[0] * d.q[0] + d.q[1] * d.q[1] + d.q[2] * d.q[2] + d.q[3] * d.q[3]);
    const float w = d.q[0] / n, a = d.q[1] / n, b = d.q[2] / n, c = d.q[3] / n;
    x.s = d.s;
    x.q[0] = w; x.q[1] = a; x.q[2] = b; x.q[3] = c;
    x.R[0] = 1.f - 2.f * (b * b + c * c); x.R[1] = 2.f * (a * b - w * c); x.R[2] = 2.f * (a * c + w * b);
    x.R[3] = 2.f * (a * b + w * c); x.R[4] = 1.f - 2.f * (a * a + c * c); x.R[5] = 2.f * (b * c - w * a);
    x.R[6] = 2.f * (a * c - w * b); x.R[7] = 2.f * (b * c + w * a); x.R[8] = 1.f - 2.f * (a * a + b * b);
    x.t[0] = d.t[0]; x.t[1] = d.t[1]; x.t[2] = d.t[2];
    return x;
}

__global__ __launch_bounds__(256) void k_warp(float *__restrict__ mean, float *__restrict__ quat,
                                               float *__restrict__ scale, const int32_t *__restrict__ kf,
                                               int64_t n, const fm_sim3 *__restrict__ deltas, int32_t K) {
#pragma clang fp contract(off)
    __shared__ Sim3x sd[kWarpLds];
    const bool staged = K <= kWarpLds;
    if (staged)
        for (int k = threadIdx.x; k < K; k += 256) sd[k] = make_sim(deltas[k]);
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t k = kf[i];
        if (k < 0 || k >= K) continue;
        const Sim3x T = staged ? sd[k] : make_sim(deltas[k]);
        const float x = mean[i], y = mean[n + i], z = mean[2 * n + i];
        mean[i] = T.s * (T.R[0] * x + T.R[1] * y + T.R[2] * z) + T.t[0];
        mean[n + i] = T.s * (T.R[3] * x + T.R[4] * y + T.R[5] * z) + T.t[1];
        mean[2 * n + i] = T.s * (T.R[6] * x + T.R[7] * y + T.R[8] * z) + T.t[2];
        const float bw = quat[i], bx = quat[n + i], by = quat[2 * n + i], bz = quat[3 * n + i];
        quat[i] = T.q[0] * bw - T.q[1] * bx - T.q[2] * by - T.q[3] * bz;
        quat[n + i] = T.q[0] * bx + T.q[1] * bw + T.q[2] * bz - T.q[3] * by;
        quat[2 * n + i] = T.q[0] * by - T.q[1] * bz + T.q[2] * bw + T.q[3] * bx;
        quat[3 * n + i] = T.q[0] * bz + T.q[1] * by - T.q[2] * bx + T.q[3] * bw;
        scale[i] *= T.s;
        scale[n + i] *= T.s;
    }
}

}  // namespace

hipError_t launch_warp(float *mean, float *quat, float *scale, const int32_t *kf, int64_t n,
                       const fm_sim3 *deltas, int32_t K, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_warp, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, st, mean, quat, scale,
                       kf, n, deltas, K);
    return hipGetLastError();
}

}  // namespace fm
