// adam.h -- the optimizer arithmetic shared by the separate optimizer kernels
// and the backward projection that applies Adam where the gradient is formed
// (Sec. 3.3: Adam on the raw parameters, the opacity loss beta_o mean(o) and
// the size loss beta_s mean(2 / |(v1 - v0) x (v2 - v0)|)).  One definition,
// so both paths take the same FP32 steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ts {

struct AdamK {
    float b1, b2, bc1, bc2, eps;   // betas and the bias corrections 1 - beta^t
};

// One bias-corrected Adam step of parameter p with gradient g; m and s are
// the first and second moments, updated in place.
__device__ __forceinline__ float adam_update(float p, float g, float& m, float& s, float lr,
                                             const AdamK& k)
{
    m = fmaf(k.b1, m, (1.f - k.b1) * g);
    s = fmaf(k.b2, s, (1.f - k.b2) * g * g);
    return p - lr * (m / k.bc1) / (sqrtf(s / k.bc2) + k.eps);
}

// Activation chains: act 1 is the opacity logit (o = sigmoid(a); add is the
// opacity loss's dL/do = beta_o / N), act 2 the log of sigma (sigma = exp(b)).
// y is the activated value before the step.
__device__ __forceinline__ float act_grad(float g, int act, float add, float y)
{
    if (act == 1) return (g + add) * y * (1.f - y);
    if (act == 2) return g * y;
    return g;
}

__device__ __forceinline__ float act_value(float p, int act)
{
    return act == 1 ? 1.f / (1.f + expf(-p)) : expf(p);
}

// Adds the size loss's gradient for one triangle to its vertex gradient row:
// L = beta_s / N sum 2 / |c|, c = (v1 - v0) x (v2 - v0), so dL/dc = -2 beta_s
// / N c / |c|^3, and c = e1 x e2 gives dL/de1 = e2 x dL/dc, dL/de2 = dL/dc x e1.
__device__ __forceinline__ void size_loss_grad(const float* p, float* g, float beta_s, int64_t N)
{
    const float e1[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
    const float e2[3] = {p[6] - p[0], p[7] - p[1], p[8] - p[2]};
    const float c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
    const float n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (!(n2 > 0.f)) return;
    const float inv = rsqrtf(n2);
    const float kk = -2.f * beta_s / (float)N * inv * inv * inv;   // dL/dc = kk c
    const float gc[3] = {kk * c[0], kk * c[1], kk * c[2]};
    const float g1[3] = {e2[1] * gc[2] - e2[2] * gc[1], e2[2] * gc[0] - e2[0] * gc[2],
                         e2[0] * gc[1] - e2[1] * gc[0]};
    const float g2[3] = {gc[1] * e1[2] - gc[2] * e1[1], gc[2] * e1[0] - gc[0] * e1[2],
                         gc[0] * e1[1] - gc[1] * e1[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g[a] -= g1[a] + g2[a];
        g[3 + a] += g1[a];
        g[6 + a] += g2[a];
    }
}

}  // namespace ts
