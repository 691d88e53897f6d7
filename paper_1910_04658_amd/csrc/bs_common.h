// Internal helpers shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binsketch.h"

namespace bs {

constexpr int kWave = 64;  // CDNA wavefront width

// T(x) = ln(1 - x/N) / ln(1 - 1/N) for x in [0, N] in FP64, with x = N taken as
// N - 1 (the saturation clamp). Every table of T is built from this one
// expression, so the FP32 tables of all kernels hold the same bits.
__device__ __forceinline__ double t_value(int32_t x, int32_t N) {
  const int32_t xc = x < N ? x : N - 1;
  return xc == 0 ? 0.0 : log1p(-(double)xc / (double)N) / log1p(-1.0 / (double)N);
}

// Returns BS_OK if the current device is a gfx950, else BS_ERR_DEVICE.
bs_status check_device();

// LDS bytes a block may use and the compute-unit count of the current device
// (cached per device; zeros if the runtime cannot say).
void device_limits(int* lds_max, int* n_cu);

inline bool valid_width(int32_t N) { return N >= 64 && N <= BS_MAX_N && N % 64 == 0; }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline bs_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BS_OK : BS_ERR_HIP;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Records a pair of HIP events around the launches in its scope when timing
// is enabled (bs_timing_enable); otherwise does nothing.
class ScopedTiming {
 public:
  ScopedTiming(const char* name, hipStream_t s);
  ~ScopedTiming();

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr;
  hipEvent_t stop_ = nullptr;
};

// ---- device helpers -------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// View of read-only global data through the constant address space, so that
// wave-uniform loads from it become scalar (s_load) loads feeding SGPR
// operands. Only for data no kernel writes while the reading kernel runs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}

__device__ __forceinline__ uint32_t popc32(uint32_t x) { return __builtin_popcount(x); }

// acc + popcount(x) as one v_bcnt_u32_b32 (bit count with accumulate). The
// compiler otherwise may split long count chains into separate counts plus
// three-input adds, half an instruction more per word.
__device__ __forceinline__ uint32_t bcnt_add(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// Order-preserving map float -> uint32 (larger float -> larger key). -0.0 is
// first turned into +0.0 so that the two zeros compare equal, as IEEE says.
__device__ __forceinline__ uint32_t float_key(float f) {
  f = f + 0.0f;
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

// The estimators of Algorithms 1-4 in FP32 from table values T(x_a), T(x_b),
// T(x_u), with Hamming as |a|+|b|-2 IP, in the canonical operation order:
// s = Ta + Tb, ip = s - Tu, ham = s - 2 ip, js = ip / (ip + ham),
// cos = ip / sqrt(Ta Tb); zero denominators give 0.
template <int M>
__device__ __forceinline__ float score_f32(float Ta, float Tb, float Tu) {
  const float s = Ta + Tb;
  const float ip = s - Tu;
  if (M == BS_IP) return ip;
  const float ham = s - (ip + ip);
  if (M == BS_HAMMING) return ham;
  if (M == BS_JACCARD) {
    const float den = ip + ham;
    return den == 0.0f ? 0.0f : ip / den;
  }
  const float pr = Ta * Tb;
  return pr == 0.0f ? 0.0f : ip / sqrtf(pr);
}

}  // namespace bs
