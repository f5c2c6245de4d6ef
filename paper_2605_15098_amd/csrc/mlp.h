// The schedule cost model's network (k7, mlp.hip): layout of its flat
// parameter array and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace svk {

constexpr int kMlpHidden = 64;
constexpr int kMlpMaxIn = 32;

// Offsets (in floats) of each tensor in the flat parameter array.
struct MlpLayout {
    int in, w1, b1, w2, b2, w3, b3, count;
};

__host__ __device__ constexpr MlpLayout mlp_layout(int in)
{
    return MlpLayout{in,
                     0,
                     kMlpHidden * in,
                     kMlpHidden * in + kMlpHidden,
                     kMlpHidden * in + kMlpHidden + kMlpHidden * kMlpHidden,
                     kMlpHidden * in + 2 * kMlpHidden + kMlpHidden * kMlpHidden,
                     kMlpHidden * in + 3 * kMlpHidden + kMlpHidden * kMlpHidden,
                     kMlpHidden * in + 3 * kMlpHidden + kMlpHidden * kMlpHidden + 1};
}

constexpr int kMlpMaxParams = mlp_layout(kMlpMaxIn).count;

// Work-groups of the gradient kernel for a batch; the workspace holds one
// row of count + 1 floats per group.
int mlp_grad_groups(int batch);

// y[s] = network(standardised X[s]) for s < batch. With argmin non-null
// (batch <= 64 only) the index of the smallest prediction, lowest index on
// ties, is written to *argmin.
hipError_t mlp_forward(const float *P, int in, const float *norm, const float *X, int batch, float *y,
                       int *argmin, hipStream_t st);
// grad = d/dP of mean_s (network(X[s]) - T[s])^2; *loss = that mean.
hipError_t mlp_grad(const float *P, int in, const float *norm, const float *X, const float *T, int batch,
                    float *grad, float *loss, float *workspace, hipStream_t st);
// One Adam update of P (moments m, v) with gradient g; step counts from 1.
hipError_t mlp_adam(float *P, float *m, float *v, const float *g, int count, float lr, float beta1, float beta2,
                    float eps, int step, hipStream_t st);

}  // namespace svk
