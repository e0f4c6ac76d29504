// Forward, gradient, Adam and selection kernels of the parameter-selector
// network (shapes in mlp.hpp).
//
// A workgroup is one wave; lane j owns unit j of every layer. The parameters
// (37 KB) are staged in LDS once per workgroup and a workgroup walks a
// strided share of the batch, one sample at a time: activations pass between
// lanes through LDS. Row reads start at column (i + j) mod width so that the
// lanes of a step touch different LDS banks. The gradient kernel sums its
// samples' gradients in LDS (each lane only updates its own units' rows, so
// no atomics) and writes one partial per workgroup; a second kernel adds the
// partials in a fixed order and divides by the number of labelled entries.
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace mag {
namespace {

constexpr int kWave = 64;
static_assert(kSelHid == kWave && kSelOut == kWave, "one lane per unit");

__device__ __forceinline__ void stage_params(float *s_p, const float *p) {
    const float4 *src = reinterpret_cast<const float4 *>(p);
    float4 *dst = reinterpret_cast<float4 *>(s_p);
    for (int i = threadIdx.x; i < kSelParams / 4; i += kWave) dst[i] = src[i];
}

struct Act {
    float z1, z2, y;
};

// Forward pass of one sample: s_x, s_h1, s_h2 receive the input and the
// hidden activations; returns this lane's pre-activations and output.
__device__ __forceinline__ Act forward_one(const float *s_p, const float *x, float *s_x, float *s_h1,
                                           float *s_h2) {
    const int j = threadIdx.x;
    if (j < kSelIn) s_x[j] = x[j];
    __syncthreads();
    Act a;
    float z = s_p[kSelB1 + j];
    for (int i = 0; i < kSelIn; ++i) {
        const int c = (i + j) & (kSelIn - 1);
        z = fmaf(s_p[kSelW1 + j * kSelIn + c], s_x[c], z);
    }
    a.z1 = z;
    s_h1[j] = z > 0.0f ? z : 0.0f;
    __syncthreads();
    z = s_p[kSelB2 + j];
    for (int i = 0; i < kSelHid; ++i) {
        const int c = (i + j) & (kSelHid - 1);
        z = fmaf(s_p[kSelW2 + j * kSelHid + c], s_h1[c], z);
    }
    a.z2 = z;
    s_h2[j] = z > 0.0f ? z : 0.0f;
    __syncthreads();
    z = s_p[kSelB3 + j];
    for (int i = 0; i < kSelHid; ++i) {
        const int c = (i + j) & (kSelHid - 1);
        z = fmaf(s_p[kSelW3 + j * kSelHid + c], s_h2[c], z);
    }
    a.y = z;
    return a;
}

__global__ __launch_bounds__(kWave) void k_mlp_forward(const float *p, const float *x, uint32_t B,
                                                       float *y) {
    __shared__ __align__(16) float s_p[kSelParams];
    __shared__ float s_x[kSelIn], s_h1[kSelHid], s_h2[kSelHid];
    stage_params(s_p, p);
    __syncthreads();
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const Act a = forward_one(s_p, x + (size_t)b * kSelIn, s_x, s_h1, s_h2);
        y[(size_t)b * kSelOut + threadIdx.x] = a.y;
        __syncthreads();       // s_x / s_h* are rewritten by the next sample
    }
}

__global__ __launch_bounds__(kWave) void k_mlp_select(const float *p, const float *x,
                                                      const uint8_t *feasible, uint32_t B,
                                                      int32_t *pick) {
    __shared__ __align__(16) float s_p[kSelParams];
    __shared__ float s_x[kSelIn], s_h1[kSelHid], s_h2[kSelHid];
    stage_params(s_p, p);
    __syncthreads();
    const int j = threadIdx.x;
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const Act a = forward_one(s_p, x + (size_t)b * kSelIn, s_x, s_h1, s_h2);
        const bool ok = feasible[(size_t)b * kSelOut + j] != 0;
        // (value, index) minimum over the wave; infeasible lanes never win
        float best = ok ? a.y : 0.0f;
        int idx = ok ? j : kSelOut;
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(idx, off);
            const bool take = oi < kSelOut && (idx == kSelOut || ob < best || (ob == best && oi < idx));
            if (take) {
                best = ob;
                idx = oi;
            }
        }
        if (j == 0) pick[b] = idx == kSelOut ? -1 : idx;
        __syncthreads();
    }
}

// Per workgroup: the unnormalized gradient sum over its samples of
// M (y - t)^2, that sum itself and the number of labelled entries, into
// partials[wg * (kSelParams + 2) ...].
__global__ __launch_bounds__(kWave) void k_mlp_grad(const float *p, const float *x, const float *t,
                                                    const uint8_t *mask, uint32_t B, float *partials) {
    extern __shared__ __align__(16) float smem[];
    float *s_p = smem;                       // kSelParams
    float *s_g = smem + kSelParams;          // kSelParams
    __shared__ float s_x[kSelIn], s_h1[kSelHid], s_h2[kSelHid], s_d[kSelOut], s_dz[kSelHid];
    const int j = threadIdx.x;
    stage_params(s_p, p);
    for (int i = j; i < kSelParams; i += kWave) s_g[i] = 0.0f;
    __syncthreads();
    float loss = 0.0f, cnt = 0.0f;
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const Act a = forward_one(s_p, x + (size_t)b * kSelIn, s_x, s_h1, s_h2);
        const bool lab = mask[(size_t)b * kSelOut + j] != 0;
        const float e = lab ? a.y - t[(size_t)b * kSelOut + j] : 0.0f;
        loss = fmaf(e, e, loss);
        cnt += lab ? 1.0f : 0.0f;
        const float d = 2.0f * e;            // d(sum M e^2) / dy
        s_d[j] = d;
        __syncthreads();
        // output layer: row j of W3 and b3
        s_g[kSelB3 + j] += d;
        for (int i = 0; i < kSelHid; ++i) {
            const int c = (i + j) & (kSelHid - 1);
            s_g[kSelW3 + j * kSelHid + c] = fmaf(d, s_h2[c], s_g[kSelW3 + j * kSelHid + c]);
        }
        // back to hidden unit j of layer 2
        float dh = 0.0f;
        for (int o = 0; o < kSelOut; ++o) dh = fmaf(s_p[kSelW3 + o * kSelHid + j], s_d[o], dh);
        const float dz2 = a.z2 > 0.0f ? dh : 0.0f;
        s_dz[j] = dz2;
        __syncthreads();
        s_g[kSelB2 + j] += dz2;
        for (int i = 0; i < kSelHid; ++i) {
            const int c = (i + j) & (kSelHid - 1);
            s_g[kSelW2 + j * kSelHid + c] = fmaf(dz2, s_h1[c], s_g[kSelW2 + j * kSelHid + c]);
        }
        dh = 0.0f;
        for (int o = 0; o < kSelHid; ++o) dh = fmaf(s_p[kSelW2 + o * kSelHid + j], s_dz[o], dh);
        const float dz1 = a.z1 > 0.0f ? dh : 0.0f;
        s_g[kSelB1 + j] += dz1;
        for (int i = 0; i < kSelIn; ++i) {
            const int c = (i + j) & (kSelIn - 1);
            s_g[kSelW1 + j * kSelIn + c] = fmaf(dz1, s_x[c], s_g[kSelW1 + j * kSelIn + c]);
        }
        __syncthreads();                     // s_x, s_h*, s_d, s_dz are rewritten next
    }
    for (int off = 32; off > 0; off >>= 1) {
        loss += __shfl_xor(loss, off);
        cnt += __shfl_xor(cnt, off);
    }
    float *out = partials + (size_t)blockIdx.x * (kSelParams + 2);
    for (int i = j; i < kSelParams; i += kWave) out[i] = s_g[i];
    if (j == 0) {
        out[kSelParams] = loss;
        out[kSelParams + 1] = cnt;
    }
}

// grad[i] = sum over workgroups of the partials / labelled count; the loss likewise.
__global__ void k_mlp_reduce(const float *partials, int groups, float *grad, float *loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = kSelParams + 2;
    float n = 0.0f;
    for (int g = 0; g < groups; ++g) n += partials[(size_t)g * stride + kSelParams + 1];
    const float inv = n > 0.0f ? 1.0f / n : 0.0f;
    if (i < kSelParams) {
        float s = 0.0f;
        for (int g = 0; g < groups; ++g) s += partials[(size_t)g * stride + i];
        grad[i] = s * inv;
    } else if (i == kSelParams) {
        float s = 0.0f;
        for (int g = 0; g < groups; ++g) s += partials[(size_t)g * stride + kSelParams];
        *loss = s * inv;
    }
}

__global__ void k_mlp_adam(float *p, const float *g, float *m, float *v, float lr, float beta1,
                           float beta2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kSelParams) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

uint32_t groups_for(uint32_t B, uint32_t cap) { return B < cap ? (B ? B : 1) : cap; }

}  // namespace

mag_status launch_mlp_forward(const float *params, const float *x, uint32_t B, float *y,
                              hipStream_t stream) {
    if (!B) return MAG_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3(groups_for(B, 512)), dim3(kWave), 0, stream, params, x, B, y);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "selector forward launch");
}

mag_status launch_mlp_select(const float *params, const float *x, const uint8_t *feasible, uint32_t B,
                             int32_t *pick, hipStream_t stream) {
    if (!B) return MAG_OK;
    hipLaunchKernelGGL(k_mlp_select, dim3(groups_for(B, 512)), dim3(kWave), 0, stream, params, x,
                       feasible, B, pick);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "selector launch");
}

mag_status launch_mlp_grad(const float *params, const float *x, const float *t, const uint8_t *mask,
                           uint32_t B, float *partials, float *grad, float *loss, hipStream_t stream) {
    static bool configured = false;
    const size_t shmem = 2 * (size_t)kSelParams * sizeof(float);
    if (!configured) {
        (void)hipFuncSetAttribute((const void *)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem);
        (void)hipGetLastError();
        configured = true;
    }
    const uint32_t G = groups_for(B, kSelGradGroups);
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(kWave), shmem, stream, params, x, t, mask, B, partials);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kSelParams + 1 + 255) / 256), dim3(256), 0, stream,
                       (const float *)partials, (int)G, grad, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "selector gradient launch");
}

mag_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kSelParams + 255) / 256), dim3(256), 0, stream, params, grad,
                       m, v, lr, beta1, beta2, eps, bc1, bc2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "selector Adam launch");
}

}  // namespace mag
