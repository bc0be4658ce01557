// BF16 storage type of the stored factors (ACR_MIXED_BF16).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace acr {

// A stored factor entry in BF16: the upper 16 bits of its FP32 value.
struct bf16s {
  uint16_t b;
  __host__ __device__ explicit operator float() const {
    union {
      uint32_t u;
      float f;
    } v;
    v.u = (uint32_t)b << 16;
    return v.f;
  }
  __host__ __device__ explicit operator double() const { return (double)(float)*this; }
};

}  // namespace acr
