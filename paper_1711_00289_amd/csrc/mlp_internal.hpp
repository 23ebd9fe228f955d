// mlp_internal.hpp -- what the network kernels (mlp.hip) and the surrogate's fused inference
// (surrogate.hip) share: the activation function, BF16 rounding, and a view of a network's device
// parameters.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace mlpk {

// h(z) = Phi(-|z|) = erfc(|z| / sqrt 2) / 2, with erfc in the Chebyshev-fitted exponential form of
// Press et al., Numerical Recipes (erfcc: erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + x / 2),
// fractional error below 1.2e-7 for every x >= 0, so the negative tail keeps its relative
// accuracy).  Evaluated with the base-2 exponential: the coefficients of P are those of erfcc times
// log2(e), and the constant term also carries the factor 1/2 (as -1), so
//   h = t exp2(log2(e) P(t) - 1 - log2(e) z^2 / 2),  t = 1 / (1 + |z| / (2 sqrt 2)).
__device__ __forceinline__ float phi_tail(float z) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(az, 0.35355339f, 1.0f));
    float p = 0.2465173f;
    p = fmaf(p, t, -1.1861149f);
    p = fmaf(p, t, 2.1474745f);
    p = fmaf(p, t, -1.6377531f);
    p = fmaf(p, t, 0.40232158f);
    p = fmaf(p, t, -0.26875687f);
    p = fmaf(p, t, 0.13963005f);
    p = fmaf(p, t, 0.53970063f);
    p = fmaf(p, t, 1.4427292f);
    p = fmaf(p, t, -2.8257482f);
    return t * __builtin_amdgcn_exp2f(fmaf(z * z, -0.72134752f, p));
}

// GELU(z) = z Phi(z) (Hendrycks & Gimpel 2016, the erf form) = max(z, 0) - |z| h(z): z (1 - h) for
// z >= 0 and z h for z < 0, one fused multiply-add.
__device__ __forceinline__ float gelu(float z) {
    return fmaf(-fabsf(z), phi_tail(z), fmaxf(z, 0.0f));
}

// GELU'(z) = Phi(z) + z phi(z), phi the standard normal density.
__device__ __forceinline__ float gelu_grad(float z) {
    const float h = phi_tail(z);
    const float Phi = z >= 0.0f ? 1.0f - h : h;
    return fmaf(z * 0.39894228f, __builtin_amdgcn_exp2f(z * z * -0.72134752f), Phi);
}

// Round two floats to BF16 (nearest, ties to even) and pack them, lo in the low half: one
// v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t bf16x2(float lo, float hi) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    const bf2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

struct NetView {
    int n;                                 // layers
    int32_t w[MLP_MAX_LAYERS + 1];         // widths
    const uint16_t *wb[MLP_MAX_LAYERS];    // BF16 weights of layer i, [w[i+1]][w[i]] row-major
    const float *bias[MLP_MAX_LAYERS];     // FP32 biases of layer i, [w[i+1]]
};

NetView net_view(const mlp_t *m);

}  // namespace mlpk
