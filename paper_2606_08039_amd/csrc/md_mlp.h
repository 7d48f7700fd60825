// md_mlp.h -- internal constants and helpers of the surrogate network.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "md.h"

namespace md {

constexpr int MLP_IN = 64;    // 60 features, zero padded
constexpr int MLP_H = 128;    // three hidden layers
constexpr int MLP_OUT = 6;    // body-frame force (3) and torque (3)
constexpr int MLP_NPARAMS = 42118;
constexpr int MLP_NORM = 2 * MLP_IN + 2 * MLP_OUT;  // x_mean, x_inv_std, y_mean, y_std
extern const int kParamOff[8];

std::string hip_msg(const char *what, hipError_t e);
hipError_t mlp_destandardize(const float *Y, const float *ymean_std, float *out, int B, hipStream_t st);
const float *mlp_device_params(const md_mlp *m);
const float *mlp_device_norm(const md_mlp *m);

}  // namespace md
