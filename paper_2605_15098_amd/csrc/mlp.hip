// k7: the schedule cost model, a multilayer perceptron in -> 64 -> 64 -> 1
// with ReLU after the two hidden layers, in FP32. It maps features of a
// (circuit, candidate schedule) pair to a predicted log run time; the tuner
// takes the candidate with the smallest prediction. Training minimises the
// mean squared error with Adam (Kingma and Ba, 2015).
//
// Parameters are one flat float array (offsets in mlp_layout):
//   W1[64][in], b1[64], W2[64][64], b2[64], w3[64], b3.
// Inputs are standardised inside the kernels: x' = (x - mean) * inv_std with
// norm = {mean[in], inv_std[in]} (norm may be null: identity).
//
// Every reduction runs in a fixed order (per sample in hidden-unit order, per
// work-group in sample order, across work-groups in group order), so results
// are deterministic for a given grid.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mlp.h"

namespace svk {

namespace {

constexpr int H = kMlpHidden;
constexpr int TILE = 64;           // samples per work-group step
constexpr int GRAD_THREADS = 256;  // threads of the gradient kernel
constexpr int PAD = H + 1;         // LDS row stride (odd: no bank conflicts on columns)

__device__ __forceinline__ float relu(float x) { return x > 0.f ? x : 0.f; }

// Parameters and standardisation, staged in LDS by the whole work-group.
__device__ void stage_params(float *sp, float *snorm, const float *P, const float *norm, int in, int count)
{
    for (int e = threadIdx.x; e < count; e += blockDim.x) sp[e] = P[e];
    for (int i = threadIdx.x; i < in; i += blockDim.x) {
        snorm[i] = norm ? norm[i] : 0.f;
        snorm[in + i] = norm ? norm[in + i] : 1.f;
    }
}

// One sample's forward pass from standardised inputs x[in]; fills h1, h2.
__device__ __forceinline__ float forward_one(const float *sp, const MlpLayout &L, const float *x, float *h1,
                                             float *h2)
{
    for (int k = 0; k < H; ++k) {
        float a = sp[L.b1 + k];
        for (int i = 0; i < L.in; ++i) a = fmaf(sp[L.w1 + k * L.in + i], x[i], a);
        h1[k] = relu(a);
    }
    for (int j = 0; j < H; ++j) {
        float a = sp[L.b2 + j];
        for (int k = 0; k < H; ++k) a = fmaf(sp[L.w2 + j * H + k], h1[k], a);
        h2[j] = relu(a);
    }
    float y = sp[L.b3];
    for (int j = 0; j < H; ++j) y = fmaf(sp[L.w3 + j], h2[j], y);
    return y;
}

// Forward: one thread per sample, one wave per work-group.
__global__ void __launch_bounds__(TILE) k7_forward_kernel(const float *P, int in, const float *norm,
                                                          const float *X, int batch, float *y, int *argmin)
{
    extern __shared__ float lds[];
    const MlpLayout L = mlp_layout(in);
    float *sp = lds;
    float *snorm = sp + L.count;
    float *sy = snorm + 2 * in;
    float *h1 = sy + TILE + threadIdx.x * 2 * H;  // per-thread rows
    float *h2 = h1 + H;
    stage_params(sp, snorm, P, norm, in, L.count);
    __syncthreads();
    const int s = blockIdx.x * TILE + threadIdx.x;
    float out = 0.f;
    if (s < batch) {
        float x[kMlpMaxIn];
        for (int i = 0; i < in; ++i) x[i] = (X[(size_t)s * in + i] - snorm[i]) * snorm[in + i];
        out = forward_one(sp, L, x, h1, h2);
        y[s] = out;
    }
    sy[threadIdx.x] = out;
    __syncthreads();
    if (argmin && gridDim.x == 1 && threadIdx.x == 0) {
        int best = 0;
        for (int k = 1; k < batch; ++k)
            if (sy[k] < sy[best]) best = k;
        *argmin = best;
    }
}

// Gradient of the mean squared error over the batch. Each work-group takes
// tiles of 64 samples (grid-stride), keeps its share of the gradient in
// registers and writes one partial row of count + 1 floats (last: loss).
constexpr int kMaxPerThread = (kMlpMaxParams + GRAD_THREADS - 1) / GRAD_THREADS;

__global__ void __launch_bounds__(GRAD_THREADS) k7_grad_kernel(const float *P, int in, const float *norm,
                                                              const float *X, const float *T, int batch,
                                                              float *partial)
{
    extern __shared__ float lds[];
    const MlpLayout L = mlp_layout(in);
    float *sp = lds;
    float *snorm = sp + L.count;
    float *xs = snorm + 2 * in;    // [TILE][in]
    float *h1 = xs + TILE * in;    // [TILE][PAD]
    float *h2 = h1 + TILE * PAD;
    float *d1 = h2 + TILE * PAD;
    float *d2 = d1 + TILE * PAD;
    float *dy = d2 + TILE * PAD;   // [TILE]
    float *sq = dy + TILE;         // [TILE]
    stage_params(sp, snorm, P, norm, in, L.count);
    const int tid = threadIdx.x;
    const float inv_b = 1.f / (float)batch;
    float acc[kMaxPerThread];
#pragma unroll
    for (int k = 0; k < kMaxPerThread; ++k) acc[k] = 0.f;
    float loss = 0.f;
    const int tiles = (batch + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        __syncthreads();
        if (tid < TILE) {
            const int s = tile * TILE + tid;
            float *x = xs + tid * in;
            float *a1 = h1 + tid * PAD, *a2 = h2 + tid * PAD, *g1 = d1 + tid * PAD, *g2 = d2 + tid * PAD;
            if (s < batch) {
                for (int i = 0; i < in; ++i) x[i] = (X[(size_t)s * in + i] - snorm[i]) * snorm[in + i];
                const float yv = forward_one(sp, L, x, a1, a2);
                const float r = yv - T[s];
                const float g = 2.f * r * inv_b;
                dy[tid] = g;
                sq[tid] = r * r;
                for (int j = 0; j < H; ++j) g2[j] = a2[j] > 0.f ? g * sp[L.w3 + j] : 0.f;
                for (int k = 0; k < H; ++k) {
                    float a = 0.f;
                    for (int j = 0; j < H; ++j) a = fmaf(sp[L.w2 + j * H + k], g2[j], a);
                    g1[k] = a1[k] > 0.f ? a : 0.f;
                }
            } else {
                for (int i = 0; i < in; ++i) x[i] = 0.f;
                for (int j = 0; j < H; ++j) a1[j] = a2[j] = g1[j] = g2[j] = 0.f;
                dy[tid] = 0.f;
                sq[tid] = 0.f;
            }
        }
        __syncthreads();
        if (tid == 0) {
            float t = 0.f;
            for (int s = 0; s < TILE; ++s) t += sq[s];
            loss += t * inv_b;
        }
#pragma unroll
        for (int k = 0; k < kMaxPerThread; ++k) {
            const int e = tid + k * GRAD_THREADS;
            if (e >= L.count) break;
            const float *A;
            const float *B = nullptr;
            int sa, sb = 0;
            if (e < L.b1) {            // W1[r][c] = sum d1[s][r] x[s][c]
                const int r = (e - L.w1) / in, c = (e - L.w1) % in;
                A = d1 + r; sa = PAD; B = xs + c; sb = in;
            } else if (e < L.w2) {     // b1[r]
                A = d1 + (e - L.b1); sa = PAD;
            } else if (e < L.b2) {     // W2[r][c] = sum d2[s][r] h1[s][c]
                const int r = (e - L.w2) / H, c = (e - L.w2) % H;
                A = d2 + r; sa = PAD; B = h1 + c; sb = PAD;
            } else if (e < L.w3) {     // b2[r]
                A = d2 + (e - L.b2); sa = PAD;
            } else if (e < L.b3) {     // w3[r] = sum dy[s] h2[s][r]
                A = dy; sa = 1; B = h2 + (e - L.w3); sb = PAD;
            } else {                   // b3
                A = dy; sa = 1;
            }
            float t = 0.f;
            if (B) {
                for (int s = 0; s < TILE; ++s) t = fmaf(A[s * sa], B[s * sb], t);
            } else {
                for (int s = 0; s < TILE; ++s) t += A[s * sa];
            }
            acc[k] += t;
        }
    }
    float *row = partial + (size_t)blockIdx.x * (L.count + 1);
#pragma unroll
    for (int k = 0; k < kMaxPerThread; ++k) {
        const int e = tid + k * GRAD_THREADS;
        if (e < L.count) row[e] = acc[k];
    }
    if (tid == 0) row[L.count] = loss;
}

// Sum of the partial rows in group order: grad[e] and, at e == count, loss.
__global__ void __launch_bounds__(256) k7_reduce_kernel(const float *partial, int groups, int count, float *grad,
                                                        float *loss)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > count) return;
    float t = 0.f;
    for (int g = 0; g < groups; ++g) t += partial[(size_t)g * (count + 1) + e];
    if (e < count) grad[e] = t;
    else if (loss) *loss = t;
}

// Adam with bias correction; step is the 1-based update count.
__global__ void __launch_bounds__(256) k7_adam_kernel(float *P, float *m, float *v, const float *g, int count,
                                                      float lr, float beta1, float beta2, float eps, int step)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const double c1 = 1.0 - pow((double)beta1, (double)step);
    const double c2 = 1.0 - pow((double)beta2, (double)step);
    const float ge = g[e];
    const float me = beta1 * m[e] + (1.f - beta1) * ge;
    const float ve = beta2 * v[e] + (1.f - beta2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float mh = (float)(me / c1);
    const float vh = (float)(ve / c2);
    P[e] -= lr * mh / (sqrtf(vh) + eps);
}

size_t forward_lds(int in) { return sizeof(float) * (mlp_layout(in).count + 2 * in + TILE + TILE * 2 * H); }

size_t grad_lds(int in)
{
    return sizeof(float) * (mlp_layout(in).count + 2 * in + TILE * in + 4 * TILE * PAD + 2 * TILE);
}

bool in_ok(int in) { return in >= 1 && in <= kMlpMaxIn; }

}  // namespace

int mlp_grad_groups(int batch)
{
    const int tiles = (batch + TILE - 1) / TILE;
    return tiles < 128 ? tiles : 128;
}

hipError_t mlp_forward(const float *P, int in, const float *norm, const float *X, int batch, float *y,
                       int *argmin, hipStream_t st)
{
    if (!in_ok(in) || batch < 1) return hipErrorInvalidValue;
    if (argmin && batch > TILE) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k7_forward_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const unsigned grid = (unsigned)((batch + TILE - 1) / TILE);
    k7_forward_kernel<<<grid, TILE, forward_lds(in), st>>>(P, in, norm, X, batch, y, argmin);
    return hipGetLastError();
}

hipError_t mlp_grad(const float *P, int in, const float *norm, const float *X, const float *T, int batch,
                    float *grad, float *loss, float *workspace, hipStream_t st)
{
    if (!in_ok(in) || batch < 1) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k7_grad_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const MlpLayout L = mlp_layout(in);
    const int groups = mlp_grad_groups(batch);
    k7_grad_kernel<<<groups, GRAD_THREADS, grad_lds(in), st>>>(P, in, norm, X, T, batch, workspace);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k7_reduce_kernel<<<(L.count + 1 + 255) / 256, 256, 0, st>>>(workspace, groups, L.count, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, float *m, float *v, const float *g, int count, float lr, float beta1, float beta2,
                    float eps, int step, hipStream_t st)
{
    if (count < 1 || step < 1) return hipErrorInvalidValue;
    k7_adam_kernel<<<(count + 255) / 256, 256, 0, st>>>(P, m, v, g, count, lr, beta1, beta2, eps, step);
    return hipGetLastError();
}

}  // namespace svk
