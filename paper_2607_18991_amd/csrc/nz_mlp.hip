// nz_mlp.hip -- the small MLP of the learned prefill: (7 zone-mask bits,
// standardised size variable L^(-1/nu)) -> 64 -> 64 -> (u, v), tanh after the
// hidden layers; u, v
// estimate ln mean and ln std of n*/N.  Weights are stored as bfloat16 and
// widened exactly to float; every product and sum is FP32.  The network is
// about 5k parameters and is evaluated for a few hundred rows, so the kernels
// are latency-bound single-pass loops rather than matrix-core tiles.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nz.h"

#define NZ_API extern "C" __attribute__((visibility("default")))

namespace nzmlp {

constexpr int IN = 8, H = 64, OUT = 2;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + IN * H;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H * OUT;
constexpr int NPARAM = OFF_B3 + OUT;
static_assert(NPARAM == NZ_MLP_NPARAM, "parameter layout");
static_assert(NZ_MLP_NACT == 2 * H, "activation cache layout");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

// Round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    return static_cast<uint16_t>((u + 0x7FFFu + lsb) >> 16);
}

// One workgroup of 64 threads per row; thread j owns hidden unit j.
__global__ __launch_bounds__(64) void mlp_forward_kernel(const uint16_t *__restrict__ p, const float *__restrict__ x,
                                                         float *__restrict__ y, float *__restrict__ act, int32_t B)
{
    __shared__ float h1[H], h2[H], xin[IN];
    const int b = blockIdx.x;
    if (b >= B) return;
    const int j = threadIdx.x;
    if (j < IN) xin[j] = x[b * IN + j];
    __syncthreads();
    float a = bf16_to_f32(p[OFF_B1 + j]);
    for (int i = 0; i < IN; ++i) a = fmaf(xin[i], bf16_to_f32(p[OFF_W1 + i * H + j]), a);
    h1[j] = tanhf(a);
    __syncthreads();
    a = bf16_to_f32(p[OFF_B2 + j]);
    for (int k = 0; k < H; ++k) a = fmaf(h1[k], bf16_to_f32(p[OFF_W2 + k * H + j]), a);
    h2[j] = tanhf(a);
    act[b * NZ_MLP_NACT + j] = h1[j];
    act[b * NZ_MLP_NACT + H + j] = h2[j];
    __syncthreads();
    if (j < OUT) {
        a = bf16_to_f32(p[OFF_B3 + j]);
        for (int k = 0; k < H; ++k) a = fmaf(h2[k], bf16_to_f32(p[OFF_W3 + k * OUT + j]), a);
        y[b * OUT + j] = a;
    }
}

// One workgroup of 256 threads for the whole batch, rows taken in tiles of 32:
// the tile's pre-activation gradients are formed in LDS, then every thread adds
// the tile's contribution to the parameter gradients it owns.  The summation
// order is fixed, so results are deterministic.
constexpr int BT = 256;
constexpr int TILE = 32;

__global__ __launch_bounds__(BT) void mlp_backward_kernel(const uint16_t *__restrict__ p, const float *__restrict__ x,
                                                          const float *__restrict__ act, const float *__restrict__ dy,
                                                          float *__restrict__ grad, int32_t B)
{
    __shared__ float sx[TILE][IN], sh1[TILE][H], sh2[TILE][H], sdy[TILE][OUT], dz2[TILE][H], dz1[TILE][H];
    constexpr int PER = (NPARAM + BT - 1) / BT;
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.0f;
    const int t = threadIdx.x;

    for (int r0 = 0; r0 < B; r0 += TILE) {
        const int rows = min(TILE, B - r0);
        for (int e = t; e < TILE * H; e += BT) {
            const int r = e / H, k = e % H;
            const bool ok = r < rows;
            sh1[r][k] = ok ? act[(r0 + r) * NZ_MLP_NACT + k] : 0.0f;
            sh2[r][k] = ok ? act[(r0 + r) * NZ_MLP_NACT + H + k] : 0.0f;
        }
        for (int e = t; e < TILE * IN; e += BT) {
            const int r = e / IN, i = e % IN;
            sx[r][i] = r < rows ? x[(r0 + r) * IN + i] : 0.0f;
        }
        for (int e = t; e < TILE * OUT; e += BT) {
            const int r = e / OUT, o = e % OUT;
            sdy[r][o] = r < rows ? dy[(r0 + r) * OUT + o] : 0.0f;
        }
        __syncthreads();
        // dz2 = (dy W3^T) * (1 - h2^2)
        for (int e = t; e < TILE * H; e += BT) {
            const int r = e / H, k = e % H;
            float g = 0.0f;
            for (int o = 0; o < OUT; ++o) g = fmaf(sdy[r][o], bf16_to_f32(p[OFF_W3 + k * OUT + o]), g);
            dz2[r][k] = g * (1.0f - sh2[r][k] * sh2[r][k]);
        }
        __syncthreads();
        // dz1 = (dz2 W2^T) * (1 - h1^2)
        for (int e = t; e < TILE * H; e += BT) {
            const int r = e / H, k = e % H;
            float g = 0.0f;
            for (int j = 0; j < H; ++j) g = fmaf(dz2[r][j], bf16_to_f32(p[OFF_W2 + k * H + j]), g);
            dz1[r][k] = g * (1.0f - sh1[r][k] * sh1[r][k]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = t + q * BT;
            if (idx >= NPARAM) break;
            float g = 0.0f;
            if (idx < OFF_B1) {
                const int i = idx / H, j = idx % H;
                for (int r = 0; r < rows; ++r) g = fmaf(sx[r][i], dz1[r][j], g);
            } else if (idx < OFF_W2) {
                const int j = idx - OFF_B1;
                for (int r = 0; r < rows; ++r) g += dz1[r][j];
            } else if (idx < OFF_B2) {
                const int k = (idx - OFF_W2) / H, j = (idx - OFF_W2) % H;
                for (int r = 0; r < rows; ++r) g = fmaf(sh1[r][k], dz2[r][j], g);
            } else if (idx < OFF_W3) {
                const int j = idx - OFF_B2;
                for (int r = 0; r < rows; ++r) g += dz2[r][j];
            } else if (idx < OFF_B3) {
                const int k = (idx - OFF_W3) / OUT, o = (idx - OFF_W3) % OUT;
                for (int r = 0; r < rows; ++r) g = fmaf(sh2[r][k], sdy[r][o], g);
            } else {
                const int o = idx - OFF_B3;
                for (int r = 0; r < rows; ++r) g += sdy[r][o];
            }
            acc[q] += g;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = t + q * BT;
        if (idx < NPARAM) grad[idx] = acc[q];
    }
}

// Adam with decoupled weight decay; FP32 master weights, BF16 copy rewritten.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ w, uint16_t *__restrict__ wb,
                                                       const float *__restrict__ g, float *__restrict__ m,
                                                       float *__restrict__ v, float lr, float b1, float b2, float eps,
                                                       float wd, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1;
    const float vh = vi / c2;
    const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
    w[i] = wi;
    wb[i] = f32_to_bf16(wi);
}

// Weighted squared error and its gradient; one workgroup, fixed summation order.
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                                       const float *__restrict__ w, float *__restrict__ dy,
                                                       float *__restrict__ loss, int32_t B)
{
    __shared__ float red[256];
    float sw = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) sw += w[b];
    red[threadIdx.x] = sw;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const float inv = 1.0f / red[0];
    __syncthreads();
    float acc = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float wn = w[b] * inv;
        for (int o = 0; o < OUT; ++o) {
            const float r = y[b * OUT + o] - t[b * OUT + o];
            acc = fmaf(wn * r, r, acc);
            dy[b * OUT + o] = 2.0f * wn * r;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

}  // namespace nzmlp

namespace nz {
int set_error(int code, const char *msg);
}

namespace {
int mlp_fail(hipError_t e)
{
    return e == hipSuccess ? NZ_OK : nz::set_error(NZ_EDEVICE, hipGetErrorString(e));
}
}  // namespace

NZ_API int nz_mlp_forward(const uint16_t *params_bf16, const float *x, float *y, float *act, int32_t B, void *stream)
{
    if (!params_bf16 || !x || !y || !act || B < 1) return nz::set_error(NZ_EINVAL, "nz_mlp_forward: NULL pointer or B < 1");
    hipLaunchKernelGGL(nzmlp::mlp_forward_kernel, dim3(B), dim3(64), 0, static_cast<hipStream_t>(stream), params_bf16,
                       x, y, act, B);
    return mlp_fail(hipGetLastError());
}

NZ_API int nz_mlp_backward(const uint16_t *params_bf16, const float *x, const float *act, const float *dy, float *grad,
                           int32_t B, void *stream)
{
    if (!params_bf16 || !x || !act || !dy || !grad || B < 1) return nz::set_error(NZ_EINVAL, "nz_mlp_backward: NULL pointer or B < 1");
    hipLaunchKernelGGL(nzmlp::mlp_backward_kernel, dim3(1), dim3(nzmlp::BT), 0, static_cast<hipStream_t>(stream),
                       params_bf16, x, act, dy, grad, B);
    return mlp_fail(hipGetLastError());
}

NZ_API int nz_mlp_adam(float *params_fp32, uint16_t *params_bf16, const float *grad, float *adam_m, float *adam_v,
                       const float hyper[5], int32_t step, void *stream)
{
    if (!params_fp32 || !params_bf16 || !grad || !adam_m || !adam_v || !hyper || step < 1)
        return nz::set_error(NZ_EINVAL, "nz_mlp_adam: NULL pointer or step < 1");
    const float lr = hyper[0], b1 = hyper[1], b2 = hyper[2], eps = hyper[3], wd = hyper[4];
    if (!(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f) || !(wd >= 0.0f))
        return nz::set_error(NZ_EINVAL, "nz_mlp_adam: hyper-parameters out of range");
    const float c1 = 1.0f - powf(b1, static_cast<float>(step));
    const float c2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(nzmlp::mlp_adam_kernel, dim3((nzmlp::NPARAM + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params_fp32, params_bf16, grad, adam_m, adam_v, lr, b1, b2,
                       eps, wd, c1, c2);
    return mlp_fail(hipGetLastError());
}

NZ_API int nz_mlp_loss(const float *y, const float *target, const float *weight, float *dy, float *loss, int32_t B,
                       void *stream)
{
    if (!y || !target || !weight || !dy || !loss || B < 1)
        return nz::set_error(NZ_EINVAL, "nz_mlp_loss: NULL pointer or B < 1");
    hipLaunchKernelGGL(nzmlp::mlp_loss_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), y, target,
                       weight, dy, loss, B);
    return mlp_fail(hipGetLastError());
}
