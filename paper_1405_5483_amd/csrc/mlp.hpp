// The parameter-selector network: 16 features -> 64 ReLU -> 64 ReLU -> 64
// predicted costs (one per candidate (q, k, sigma') triple), FP32. Parameters
// are one flat vector: W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [64][64],
// b3 [64], rows are output units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mag_internal.hpp"

namespace mag {

constexpr int kSelIn = 16;
constexpr int kSelHid = 64;
constexpr int kSelOut = 64;
constexpr int kSelChoices = 32;   // outputs 0..31 predict cost, 32..63 verifications
constexpr int kSelW1 = 0;
constexpr int kSelB1 = kSelW1 + kSelHid * kSelIn;
constexpr int kSelW2 = kSelB1 + kSelHid;
constexpr int kSelB2 = kSelW2 + kSelHid * kSelHid;
constexpr int kSelW3 = kSelB2 + kSelHid;
constexpr int kSelB3 = kSelW3 + kSelOut * kSelHid;
constexpr int kSelParams = kSelB3 + kSelOut;
constexpr int kSelGradGroups = 32;        // workgroups that each sum part of a batch's gradient

// y [B][64] = network(x [B][16]).
mag_status launch_mlp_forward(const float *params, const float *x, uint32_t B, float *y,
                              hipStream_t stream);
// Gradient of the masked mean squared error sum M (y - t)^2 / sum M over the
// batch into grad [kSelParams] and the loss into *loss. partials holds
// kSelGradGroups * (kSelParams + 2) floats.
mag_status launch_mlp_grad(const float *params, const float *x, const float *t, const uint8_t *mask,
                           uint32_t B, float *partials, float *grad, float *loss, hipStream_t stream);
// One Adam step with bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
mag_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2,
                           hipStream_t stream);
// pick[b] = feasible candidate with the smallest output (lowest index on
// ties), -1 if none.
mag_status launch_mlp_select(const float *params, const float *x, const uint8_t *feasible, uint32_t B,
                             int32_t *pick, hipStream_t stream);

}  // namespace mag
