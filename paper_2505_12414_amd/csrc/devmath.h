// Per-event arithmetic of the two precisions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace uml {

// FP32: single hardware instructions (v_exp_f32, v_log_f32, v_rcp_f32,
// v_sqrt_f32, v_sin_f32, v_cos_f32), each correct to about one ulp.
static __device__ __forceinline__ float k_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
static __device__ __forceinline__ float k_log2(float x) { return __builtin_amdgcn_logf(x); }
static __device__ __forceinline__ float k_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
static __device__ __forceinline__ float k_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
static __device__ __forceinline__ void k_sincos(float phi, float& s, float& c) {
  // the hardware sine and cosine take their argument in revolutions:
  // t = phi / (2 pi) with 1/(2 pi) as an FP32 pair (its nearest FP32 value
  // alone is 4e-8 small, a scale error that every event would share)
  const float t = fmaf(phi, 0x1.45f306p-3f, phi * 0x1.b9391p-28f);
  s = __builtin_amdgcn_sinf(t);
  c = __builtin_amdgcn_cosf(t);
}
// FP64: the device math library.
static __device__ __forceinline__ double k_exp2(double x) { return exp2(x); }
static __device__ __forceinline__ double k_log2(double x) { return log2(x); }
static __device__ __forceinline__ double k_rcp(double x) { return 1.0 / x; }
static __device__ __forceinline__ double k_sqrt(double x) { return sqrt(x); }
static __device__ __forceinline__ void k_sincos(double phi, double& s, double& c) { sincos(phi, &s, &c); }

}  // namespace uml
