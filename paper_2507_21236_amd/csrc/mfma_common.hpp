// Device helpers shared by the gfx950 kernel sources: MFMA wrappers, the
// accumulator layouts of the 16 x 16 x 4 FP64 / FP32 and 16 x 16 x 32 BF16
// products (checked on the device by a probe of each instruction), and
// loads through the global address space.
#pragma once
#include <hip/hip_runtime.h>

namespace attn {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct V4;
template <> struct V4<double> { typedef d4 type; };
template <> struct V4<float> { typedef f4 type; };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// accumulator row of item i in lane group g = lane / 16
template <typename T> __device__ __forceinline__ int drow(int g, int i);
template <> __device__ __forceinline__ int drow<double>(int g, int i) { return g + 4 * i; }
template <> __device__ __forceinline__ int drow<float>(int g, int i) { return 4 * g + i; }

// accumulator row of item i in lane group g for the 16x16x32 BF16 product
__device__ __forceinline__ int drow_bf(int g, int i) { return 4 * g + i; }
// column held at position pos of a permuted 32-wide chunk, and its inverse
__device__ __forceinline__ int bf_perm(int pos) {
  const int j = pos & 7, g = (pos >> 3) & 3;
  return (pos & ~31) + 16 * (j >> 2) + drow_bf(g, j & 3);
}
__device__ __forceinline__ int bf_pinv(int a) {
  const int r = a & 15, h = (a >> 4) & 1;
  return (a & ~31) + 8 * (r >> 2) + 4 * h + (r & 3);
}

// Loads of operator blocks through the global address space: the blocks
// arrive as generic pointers, and flat loads would make every wait for them
// also wait for LDS traffic (full drains instead of counted partial waits).
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// The rows of Y_s owned by this wave for items [i0, i1), written to y.
// Column order of a 16-wide tile as the products see it: tile row m of both
// MFMA stages stands for column colperm(m).  FP64: the accumulator rows of a
// lane, l/16 + 4 i, become the columns 2 (l/16) + {0, 1, 8, 9}, so that each
// lane ends up with two pairs of adjacent columns and stores them as 16-byte
// writes; FP32 lanes already hold 4 adjacent columns.
template <typename T> __device__ __forceinline__ int colperm(int m);
template <> __device__ __forceinline__ int colperm<double>(int m) { return 2 * (m & 3) + ((m >> 2) & 1) + 8 * (m >> 3); }
template <> __device__ __forceinline__ int colperm<float>(int m) { return m; }

}  // namespace attn
