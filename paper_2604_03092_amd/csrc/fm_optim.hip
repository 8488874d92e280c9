// fm_optim.hip -- fused Adam step over the surfel parameter tensors (the
// optimizer of the map refinement, Sec. 3.3; the paper names none, Adam as
// defined by Kingma & Ba, Algorithm 1, is used).
//
// Each tensor is updated in the space its parameterisation names: theta = p,
// log p (tangent scales) or log(p / (1 - p)) (opacity).  The rasterizer takes
// and returns the activated values p, so the kernel maps p and dL/dp to
// theta and dL/dtheta, takes the bias-corrected step there and maps back.
// One thread per element; everything per element stays in registers
// (reads p, g, m, v; writes p, m, v).  The step counter lives in device
// memory and is advanced by a one-thread kernel first, so a captured graph
// replays consecutive steps.
#include "fm_internal.h"

namespace fm {

namespace {

constexpr float kLogitClamp = 1e-6f;   // logit parameters are kept in [1e-6, 1 - 1e-6]
constexpr float kLogFloor = 1e-30f;    // log parameters are kept >= 1e-30

__global__ void k_step_advance(int32_t *step) { *step += 1; }

__global__ __launch_bounds__(256) void k_adam(fm_adam_tensor t, const int32_t *__restrict__ step, float b1,
                                               float b2, float eps) {
    const float tf = (float)*step;
    const float bc1 = 1.f - powf(b1, tf);
    const float bc2 = 1.f - powf(b2, tf);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < t.n; i += (int64_t)gridDim.x * 256) {
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
    }
}

}  // namespace

hipError_t launch_adam(const fm_adam_tensor *ts, int count, const fm_adam_config &cfg, int32_t *step,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, st, step);
    for (int k = 0; k < count; ++k) {
        if (ts[k].n == 0) continue;
        const int64_t blocks = (ts[k].n + 255) / 256;
        hipLaunchKernelGGL(k_adam, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, st, ts[k], step,
                           cfg.beta1, cfg.beta2, cfg.eps);
    }
    return hipGetLastError();
}

}  // namespace fm
