// Shared definitions of the slab solver's HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

// ---------------------------------------------------------------------------
// Error reporting (thread-local message, status codes of slab.h).
// ---------------------------------------------------------------------------
namespace slab {

void set_error(const std::string& msg);

#define SLAB_HIP_CHECK(expr)                                                   \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::slab::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_)); \
      return SLAB_E_HIP;                                                       \
    }                                                                          \
  } while (0)

// Launch-error check after a kernel launch.
#define SLAB_LAUNCH_CHECK()                                                    \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) {                                                    \
      ::slab::set_error(std::string("kernel launch failed at ") + __FILE__ +    \
                        ":" + std::to_string(__LINE__) + ": " +                 \
                        hipGetErrorString(e_));                                \
      return SLAB_E_HIP;                                                       \
    }                                                                          \
  } while (0)

// ---------------------------------------------------------------------------
// MFMA 16x16x4 wrappers.  One wave computes D(16x16) += A(16x4) B(4x16):
//   lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   lane l = 16 g + c holds D[acc_row(g, i)][c] in accumulator element i, with
//   acc_row(g, i) = 4 g + i for the FP32 instruction and g + 4 i for the FP64
//   instruction (measured on gfx950: the FP64 result rows are interleaved).
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct acc4;
template <> struct acc4<double> { typedef d4 type; };
template <> struct acc4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __host__ __device__ __forceinline__ int acc_row(int g, int i);
template <> __host__ __device__ __forceinline__ int acc_row<float>(int g, int i) { return 4 * g + i; }
template <> __host__ __device__ __forceinline__ int acc_row<double>(int g, int i) { return g + 4 * i; }
// Inverse of acc_row within a 16-row tile: lane group and element holding row r16.
template <typename T> __host__ __device__ __forceinline__ int acc_group(int r16);
template <typename T> __host__ __device__ __forceinline__ int acc_elem(int r16);
template <> __host__ __device__ __forceinline__ int acc_group<float>(int r16) { return r16 >> 2; }
template <> __host__ __device__ __forceinline__ int acc_elem<float>(int r16) { return r16 & 3; }
template <> __host__ __device__ __forceinline__ int acc_group<double>(int r16) { return r16 & 3; }
template <> __host__ __device__ __forceinline__ int acc_elem<double>(int r16) { return r16 >> 2; }

// Global-memory views of pointers.  Pointers read from descriptor tables are
// generic to the compiler, which then emits flat memory instructions; those
// share the LDS wait counter, so every wait for an LDS read would also wait
// for all prefetches in flight.  Kernels convert descriptor pointers once with
// gp() and work with g_t<T>* (global address space) from there on.
// Reciprocal for pivots on the critical path of sequential eliminations: the
// hardware estimate refined by Newton steps r <- r + r (1 - x r) (two for
// FP64, one for FP32), a few dependent instructions instead of the IEEE
// division sequence; the result is within about one ulp of 1/x.
__device__ __forceinline__ double fast_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float fast_recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// v if c else 0, by masking the bits (keeps a select on a just-loaded value
// out of divergent control flow, where the compiler would wait for every
// outstanding load)
__device__ __forceinline__ float keep_if(bool c, float v) {
  return __builtin_bit_cast(float, __builtin_bit_cast(int, v) & -(int)c);
}
__device__ __forceinline__ double keep_if(bool c, double v) {
  return __builtin_bit_cast(double, __builtin_bit_cast(long long, v) & -(long long)c);
}

template <class T> using g_t = __attribute__((address_space(1))) T;
template <class T> __device__ __forceinline__ g_t<T>* gp(T* p) { return (g_t<T>*)p; }

// Padded slab-block order: BP in {16, 32, 64} >= b.
inline int padded_block(int b) { return b <= 16 ? 16 : (b <= 32 ? 32 : 64); }

// Position of element (row, col) of a BP x BP propagator in the fragment-major
// layout read by the Schur kernel.  Fragment (mt, ks) for ks = 4*mt2 + i holds,
// in lane l = 16 g + n, the element (16 mt + n, 16 mt2 + acc_row(g, i)); the
// k index is permuted so that an MFMA result can be fed back as the next
// step's B operand without moving data between lanes.
template <typename T>
__host__ __device__ __forceinline__ int swz_index(int row, int col, int BP) {
  const int NK = BP / 4;
  const int mt = row >> 4, n = row & 15;
  const int mt2 = col >> 4, g = acc_group<T>(col & 15), i = acc_elem<T>(col & 15);
  const int ks = 4 * mt2 + i;
  return (mt * NK + ks) * 64 + 16 * g + n;
}

// LDS exchange between the lanes of one wave: a wave's LDS operations are
// performed in order, so only the compiler has to keep them in order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// Workgroup barrier, or the wave-level ordering when the workgroup is one wave.
template <int NT> __device__ __forceinline__ void group_sync() {
  if constexpr (NT == 64) wave_lds_sync();
  else __syncthreads();
}

inline unsigned int ceil_div(long long a, long long b) { return (unsigned int)((a + b - 1) / b); }

}  // namespace slab
