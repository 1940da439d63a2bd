// Internal helpers shared by the HIP translation units of librtucker.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rt {

// Status codes mirror include/rtucker.h.
enum : int {
  kOk = 0,
  kErrInvalid = -1,
  kErrUnsupported = -2,
  kErrWorkspace = -3,
  kErrNonfinite = -4,
  kErrNumerical = -5,
  kErrHip = -6,
  kErrNoDevice = -7
};

void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define RT_LAUNCH_CHECK(what)                                   \
  do {                                                          \
    hipError_t _e = hipGetLastError();                          \
    if (_e != hipSuccess) return ::rt::hip_fail(_e, what);      \
  } while (0)

#define RT_TRY(x)                      \
  do {                                 \
    int _rc = (x);                     \
    if (_rc != ::rt::kOk) return _rc;  \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace.  Every carve is 256-byte
// aligned; `need` accumulates the total so the same planning code answers
// the *_workspace queries (base == nullptr).
struct Arena {
  char* base;
  size_t need = 0;
  explicit Arena(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = align_up(need, 256);
    need = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// ---------------------------------------------------------------- device

// bf16 bit pattern <-> float, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    return static_cast<uint16_t>((u >> 16) | 0x0040u);
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

template <typename T>
__device__ __forceinline__ double to_double(T x) { return static_cast<double>(x); }

// Wavefront (64 lanes) sum via shuffles.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

// Block-wide sum; `scratch` holds one T per wave.  All threads get the sum.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T s = 0;
  for (int w = 0; w < nw; ++w) s += scratch[w];  // fixed order
  return s;
}

}  // namespace rt
