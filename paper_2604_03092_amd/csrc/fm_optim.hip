// fm_optim.hip -- fused Adam step over the surfel parameter tensors (the
// optimizer of the map refinement, Sec. 3.3; the paper names none, Adam as
// defined by Kingma & Ba, Algorithm 1, is used).
//
// Each tensor is updated in the space its parameterisation names: theta = p,
// log p (tangent scales) or log(p / (1 - p)) (opacity).  The rasterizer takes
// and returns the activated values p, so the kernel maps p and dL/dp to
// theta and dL/dtheta, takes the bias-corrected step there and maps back.
// Four elements per thread, all tensors of a call in one launch; everything
// per element stays in registers (reads p, g, m, v; writes p, m, v, and a
// cleared g when asked).  The step counter lives in device
// memory and is advanced by a one-thread kernel first, so a captured graph
// replays consecutive steps.
#include "fm_internal.h"

namespace fm {

namespace {

constexpr float kLogitClamp = 1e-6f;   // logit parameters are kept in [1e-6, 1 - 1e-6]
constexpr float kLogFloor = 1e-30f;    // log parameters are kept >= 1e-30

__global__ void k_step_advance(int32_t *step) { *step += 1; }

// Up to kAdamTable tensors per launch.  Block b works on 1024 consecutive
// elements of one tensor, four per thread: tensor k owns blocks
// [first[k], first[k + 1]).  A tensor whose four buffers are all 16-byte
// aligned (vec[k]) is read and written as float4; the others, and a ragged
// tail, element by element.  The arithmetic per element is the same either way.
constexpr int kAdamTable = 16;
constexpr int kAdamPerThread = 4;
constexpr int kAdamBlock = 256 * kAdamPerThread;
struct AdamTable {
    fm_adam_tensor t[kAdamTable];
    int32_t first[kAdamTable + 1];
    uint8_t vec[kAdamTable];
    int32_t count;
};

struct AdamConst {
    float b1, b2, eps, bc1, bc2;
};

// One element: p, g the activated value and dL/dp; m, v updated in place.
__device__ __forceinline__ float adam_elem(int kind, float lr, const AdamConst &c, float p, float g, float &m,
                                           float &v) {
    float th, gt;
    if (kind == FM_PARAM_LOG) {
        p = fmaxf(p, kLogFloor);
        th = logf(p);
        gt = g * p;
    } else if (kind == FM_PARAM_LOGIT) {
        p = fminf(fmaxf(p, kLogitClamp), 1.f - kLogitClamp);
        th = logf(p) - log1pf(-p);
        gt = g * p * (1.f - p);
    } else {
        th = p;
        gt = g;
    }
    m = c.b1 * m + (1.f - c.b1) * gt;
    v = c.b2 * v + (1.f - c.b2) * gt * gt;
    th -= lr * (m / c.bc1) / (sqrtf(v / c.bc2) + c.eps);
    if (kind == FM_PARAM_LOG) return expf(th);
    if (kind == FM_PARAM_LOGIT) return 1.f / (1.f + expf(-th));
    return th;
}

__global__ __launch_bounds__(256) void k_adam(AdamTable tab, const int32_t *__restrict__ step, float b1,
                                               float b2, float eps, int zero_grad) {
    int k = 0;
    while (k + 1 < tab.count && (int32_t)blockIdx.x >= tab.first[k + 1]) ++k;  // uniform over the block
    const fm_adam_tensor &t = tab.t[k];
    const int64_t i0 = ((int64_t)((int32_t)blockIdx.x - tab.first[k]) * 256 + threadIdx.x) * kAdamPerThread;
    if (i0 >= t.n) return;
    const float tf = (float)*step;
    const AdamConst c{b1, b2, eps, 1.f - powf(b1, tf), 1.f - powf(b2, tf)};
    const int kind = t.kind;
    if (tab.vec[k] && i0 + kAdamPerThread <= t.n) {
        float4 p = *reinterpret_cast<const float4 *>(t.param + i0);
        const float4 g = *reinterpret_cast<const float4 *>(t.grad + i0);
        float4 m = *reinterpret_cast<const float4 *>(t.m + i0);
        float4 v = *reinterpret_cast<const float4 *>(t.v + i0);
        p.x = adam_elem(kind, t.lr, c, p.x, g.x, m.x, v.x);
        p.y = adam_elem(kind, t.lr, c, p.y, g.y, m.y, v.y);
        p.z = adam_elem(kind, t.lr, c, p.z, g.z, m.z, v.z);
        p.w = adam_elem(kind, t.lr, c, p.w, g.w, m.w, v.w);
        *reinterpret_cast<float4 *>(t.m + i0) = m;
        *reinterpret_cast<float4 *>(t.v + i0) = v;
        *reinterpret_cast<float4 *>(t.param + i0) = p;
        if (zero_grad) *reinterpret_cast<float4 *>(t.grad + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    for (int64_t i = i0; i < i0 + kAdamPerThread && i < t.n; ++i) {
        float m = t.m[i], v = t.v[i];
        t.param[i] = adam_elem(kind, t.lr, c, t.param[i], t.grad[i], m, v);
        t.m[i] = m;
        t.v[i] = v;
        if (zero_grad) t.grad[i] = 0.f;
    }
}

}  // namespace

hipError_t launch_adam(const fm_adam_tensor *ts, int count, const fm_adam_config &cfg, int32_t *step,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, st, step);
    AdamTable tab;
    tab.count = 0;
    tab.first[0] = 0;
    for (int k = 0; k < count; ++k) {
        if (ts[k].n > 0) {
            tab.t[tab.count] = ts[k];
            tab.first[tab.count + 1] = tab.first[tab.count] + (int32_t)((ts[k].n + kAdamBlock - 1) / kAdamBlock);
            const auto a16 = [](const float *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
            tab.vec[tab.count] = a16(ts[k].param) && a16(ts[k].grad) && a16(ts[k].m) && a16(ts[k].v) ? 1 : 0;
            ++tab.count;
        }
        if (tab.count > 0 && (tab.count == kAdamTable || k + 1 == count)) {
            hipLaunchKernelGGL(k_adam, dim3((unsigned)tab.first[tab.count]), dim3(256), 0, st, tab, step,
                               cfg.beta1, cfg.beta2, cfg.eps, cfg.zero_grad ? 1 : 0);
            tab.count = 0;
        }
    }
    return hipGetLastError();
}

}  // namespace fm
