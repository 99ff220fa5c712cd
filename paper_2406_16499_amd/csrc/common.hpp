// Shared definitions of liblsq's HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <stddef.h>

namespace lsq {

// ---------------------------------------------------------------- errors --
struct HipError {
  hipError_t code;
  const char* where;
};

#define LSQ_HIP(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) throw ::lsq::HipError{e_, #expr};             \
  } while (0)

#define LSQ_LAUNCH_CHECK() LSQ_HIP(hipGetLastError())

// --------------------------------------------------- LDS poisoning (debug) --
// In builds with LSQ_POISON_LDS every work-group fills its LDS buffers with
// all-ones bit patterns (NaN in FP32 and FP64) before first use, so that a
// read of an LDS element no thread has written turns into a NaN in the
// results instead of a plausible stale value.  Every thread of the
// work-group must reach the call (it ends with a barrier).
#ifdef LSQ_POISON_LDS
template <typename T>
__device__ __forceinline__ void lds_poison(T* p, size_t bytes) {
  unsigned* w = reinterpret_cast<unsigned*>(p);
  const size_t nt = (size_t)blockDim.x * blockDim.y * blockDim.z;
  const size_t t = threadIdx.x + (size_t)blockDim.x * (threadIdx.y + (size_t)blockDim.y * threadIdx.z);
  for (size_t i = t; i < bytes / 4; i += nt) w[i] = 0xFFFFFFFFu;
  __syncthreads();
}
#define LSQ_LDS_POISON(arr) ::lsq::lds_poison(&(arr), sizeof(arr))
#else
#define LSQ_LDS_POISON(arr) ((void)0)
#endif

// ------------------------------------------------------------- constants --
constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kMaxNb = 64;              // widest panel of the blocked QR

// MFMA input precision used for the trailing updates of the factorization.
enum class Mma : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3, F8 = 4 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------ device utilities --
__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
  return __shfl_xor(v, mask, kWave);
}
__device__ __forceinline__ float shfl_xor_f(float v, int mask) {
  return __shfl_xor(v, mask, kWave);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over a whole work-group; `red` is LDS of at least blockDim.x/64 entries.
// Every thread receives the total.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Maximum over a whole work-group (every thread receives it); `red` as for block_sum.
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
  for (int i = 0; i < nw; ++i) m = fmax(m, red[i]);
  __syncthreads();
  return m;
}

template <typename T> struct Conv;
template <> struct Conv<float> {
  __device__ static float from(double v) { return (float)v; }
};
template <> struct Conv<double> {
  __device__ static double from(double v) { return v; }
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace lsq
