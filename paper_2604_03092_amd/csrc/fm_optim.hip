// fm_optim.hip -- fused Adam step over the surfel parameter tensors (the
// optimizer of the map refinement, Sec. 3.3; the paper names none, Adam as
// defined by Kingma & Ba, Algorithm 1, is used).
//
// Each tensor is updated in the space its parameterisation names: theta = p,
// log p (tangent scales) or log(p / (1 - p)) (opacity).  The rasterizer takes
// and returns the activated values p, so the kernel maps p and dL/dp to
// theta and dL/dtheta, takes the bias-corrected step there and maps back.
// One thread per element, all tensors of a call in one launch; everything
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

// Up to kAdamTable tensors per launch.  Block b works on 256 consecutive
// elements of one tensor: tensor k owns blocks [first[k], first[k + 1]).
constexpr int kAdamTable = 16;
struct AdamTable {
    fm_adam_tensor t[kAdamTable];
    int32_t first[kAdamTable + 1];
    int32_t count;
};

__global__ __launch_bounds__(256) void k_adam(AdamTable tab, const int32_t *__restrict__ step, float b1,
                                               float b2, float eps, int zero_grad) {
    int k = 0;
    while (k + 1 < tab.count && (int32_t)blockIdx.x >= tab.first[k + 1]) ++k;  // uniform over the block
    const fm_adam_tensor &t = tab.t[k];
    const int64_t i = (int64_t)((int32_t)blockIdx.x - tab.first[k]) * 256 + threadIdx.x;
    if (i >= t.n) return;
    const float tf = (float)*step;
    const float bc1 = 1.f - powf(b1, tf);
    const float bc2 = 1.f - powf(b2, tf);
    float p = t.param[i];
    const float g = t.grad[i];
    float th, gt;
    if (t.kind == FM_PARAM_LOG) {
        p = fmaxf(p, kLogFloor);
        th = logf(p);
        gt = g * p;
    } else if (t.kind == FM_PARAM_LOGIT) {
        p = fminf(fmaxf(p, kLogitClamp), 1.f - kLogitClamp);
        th = logf(p) - log1pf(-p);
        gt = g * p * (1.f - p);
    } else {
        th = p;
        gt = g;
    }
    const float m = b1 * t.m[i] + (1.f - b1) * gt;
    const float v = b2 * t.v[i] + (1.f - b2) * gt * gt;
    t.m[i] = m;
    t.v[i] = v;
    th -= t.lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    if (t.kind == FM_PARAM_LOG)
        p = expf(th);
    else if (t.kind == FM_PARAM_LOGIT)
        p = 1.f / (1.f + expf(-th));
    else
        p = th;
    t.param[i] = p;
    if (zero_grad) t.grad[i] = 0.f;
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
            tab.first[tab.count + 1] = tab.first[tab.count] + (int32_t)((ts[k].n + 255) / 256);
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
