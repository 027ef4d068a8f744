// mlp.hpp -- the drift surrogate: layout, activation and MFMA helpers.
//
// The network maps (t, rate state, rate index) to the part of the coupling
// term of the drift (paper Section 2, eq. (LIBOR-drift-PT)) that the
// first-order product expansion of Section 3.2 (eq. (drifta)) misses:
//     C_i = C'_i + sigma * net(features_i),
//     C'_i = sum_{l>i} ell_l [kappa(lambda_i + lambda_l) - kappa(lambda_i) - kappa(lambda_l)],
// where C_i is the 64-node quadrature coupling.  C'_i is evaluated exactly
// (FP32, from an FP64 table); the network only carries the O(ell^2) rest.
//
// Features (96 wide, 81 used): [0] = t_k / T_N; [1 + l] = X_l = log L_l - log L_l(0)
// for rates l > i, else 0; [41 + i] = 1 (rate index one-hot); the rest 0.
// Network: 96 -> 64 -> 64 -> 64 -> 1, tanh-form GELU, BF16 operands with FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), FP32 master
// weights.  Parameter vector (FP32):
//     W1[64][96] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lll {
namespace mlp {

constexpr int kIn = 96;
constexpr int kHid = 64;
constexpr int kRates = 40;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kHid;
constexpr int kParams = kOffB4 + 1;  // 14593

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// tanh-form GELU: 0.5 x (1 + tanh(u)), u = sqrt(2/pi) (x + 0.044715 x^3),
// = x / (1 + e^{-2u}) = x / (1 + 2^{x (a + b x^2)}) with a = -2 sqrt(2/pi) / ln 2
// and b = 0.044715 a folded into one polynomial for the hardware base-2
// exponential (which saturates to +inf / 0, giving 0 / x in the tails).
__device__ __forceinline__ float gelu(float x) {
    constexpr float a = -2.302208198144325f;
    constexpr float b = -0.1029432395800235f;
    const float p = x * fmaf(b, x * x, a);
    return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(p));
}

// d gelu / dx for the same form.
__device__ __forceinline__ float gelu_grad(float x) {
    const float x2 = x * x;
    const float u = 0.7978845608028654f * fmaf(0.044715f * x, x2, x);
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * u));  // (1 + tanh u) / 2
    const float du = 0.7978845608028654f * fmaf(3.0f * 0.044715f, x2, 1.0f);
    // d/dx [x s(u)] = s + x * 2 s (1 - s) du
    return fmaf(x * 2.0f * s * (1.0f - s), du, s);
}

__device__ __forceinline__ floatx4 mfma16(const bf16x8 &a, const bf16x8 &b, const floatx4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

}  // namespace mlp
}  // namespace lll
