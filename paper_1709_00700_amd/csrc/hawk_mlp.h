// Cost-model kernels (hk_mlp.hip): sizes and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_IN 12
#define MLP_HIDDEN 64
#define MLP_NPARAMS (MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1)

hipError_t hk_mlp_forward(hipStream_t st, const float* p, const float* mu, const float* sd, const float* X, int64_t m,
                          float* out);
// partial rows needed by hk_mlp_grad for a batch of m samples
int64_t hk_mlp_grad_rows(int64_t m);
// gradient of mean((yhat - y)^2) over samples idx[0..m) (idx NULL: rows 0..m) and the loss;
// partial/partial_loss hold partial_cap_rows rows, which must be >= hk_mlp_grad_rows(m)
// (hipErrorInvalidValue otherwise, nothing launched)
hipError_t hk_mlp_grad(hipStream_t st, const float* p, const float* mu, const float* sd, const float* X, const float* y,
                       const int32_t* idx, int64_t m, float* partial, float* partial_loss, int64_t partial_cap_rows,
                       float* grad, float* loss);
hipError_t hk_adam(hipStream_t st, float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2);
hipError_t hk_argmin_rows(hipStream_t st, const float* v, int64_t rows, int64_t cols, int32_t* out);
