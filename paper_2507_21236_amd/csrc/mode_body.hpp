// Mode-product bodies shared by the kernel sources (the staged launches and
// the persistent batched matvec run the same code, so both give the same
// results bit for bit).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mfma_common.hpp"

namespace attn {

// ============================================================================ mode product
// Element (i, f) of a (d0, d1, d2) tensor contracted on leg j, where f runs over
// the two other legs in order.
__device__ __forceinline__ int64_t mode_addr(int j, int d0, int d1, int d2, int i, int64_t f) {
  if (j == 0) return (int64_t)i * d1 * d2 + f;
  if (j == 1) {
    const int64_t a = f / d2, c = f - a * d2;
    return a * d1 * d2 + (int64_t)i * d2 + c;
  }
  return f * d2 + i;
}

// out (+)= sum_jobs coef * A x_j in.  wu = (task, f-tile of 64).  LDS holds the
// input tile [i'][f]; wave w owns f in [16 w, +16) and every i.
// workgroups per 64-wide free block of the LDS-staged mode product
constexpr int mode_qs(int NI) { return NI == 4 ? 4 : (NI == 2 ? 2 : 1); }

template <typename T, int NI, int QS = 1>
__device__ __forceinline__ void mode_mfma(const MPTask& t, const MPJob* __restrict__ jobs,
                                          const int2 wu, const T* __restrict__ xbase,
                                          unsigned char* smem_raw) {
  // QS > 1: the 64-wide free block of the work unit is split over blockIdx.y
  // into QS parts, and the four waves take (4 / QS) tiles of 16 free indices
  // times QS groups of output rows; every output entry keeps its summation order
  typedef typename V4<T>::type v4;
  constexpr int mj = 16 * NI, NQ = NI / QS, FW = 64 / QS;   // rows per wave, free width per WG
  constexpr int ld = 64 + 2;
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int j = t.j, d0 = t.d0, d1 = t.d1, d2 = t.d2;
  const int64_t f0 = (int64_t)wu.y * 64 + (QS > 1 ? FW * (int64_t)blockIdx.y : 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int tile = wave / QS, q0 = (wave % QS) * NQ;
  v4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) acc[q] = v4{0, 0, 0, 0};
  for (int jb = t.job0; jb < t.job0 + t.njob; jb++) {
    const T* in = jobs[jb].in ? (const T*)jobs[jb].in : xbase;
    const T* A = (const T*)jobs[jb].A;
    const T coef = (T)jobs[jb].coef;
    __syncthreads();
    if (j == 2) {
      for (int e = threadIdx.x; e < FW * mj; e += 256) {
        const int fl = e / mj, i = e - fl * mj;
        lds[i * ld + fl] = in[mode_addr(j, d0, d1, d2, i, f0 + fl)];
      }
    } else {
      for (int e = threadIdx.x; e < FW * mj; e += 256) {
        const int i = e / FW, fl = e - i * FW;
        lds[i * ld + fl] = in[mode_addr(j, d0, d1, d2, i, f0 + fl)];
      }
    }
    __syncthreads();
    const T* Ap = A + 16 * q0 + l16;
    for (int k0 = 0; k0 < mj; k0 += 4) {
      const T bop = lds[(k0 + l4) * ld + 16 * tile + l16] * coef;
      const T* Ak = Ap + (int64_t)(k0 + l4) * mj;
#pragma unroll
      for (int q = 0; q < NQ; q++) acc[q] = mfma16(Ak[16 * q], bop, acc[q]);
    }
  }
  T* out = (T*)t.out;
  const int64_t f = f0 + 16 * tile + l16;
#pragma unroll
  for (int q = 0; q < NQ; q++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t ad = mode_addr(j, d0, d1, d2, 16 * (q0 + q) + drow<T>(l4, i), f);
      if (t.accumulate) out[ad] += acc[q][i];
      else out[ad] = acc[q][i];
    }
}

// Generic mode product: one thread per output element.  wu = (task, first element).
template <typename T>
__device__ __forceinline__ void mode_gen_elem(const MPTask& t, const MPJob* __restrict__ jobs,
                                              int64_t e, const T* __restrict__ xbase) {
  const int j = t.j, d0 = t.d0, d1 = t.d1, d2 = t.d2;
  const int mj = j == 0 ? d0 : (j == 1 ? d1 : d2);
  const int64_t total = (int64_t)d0 * d1 * d2;
  if (e >= total) return;
  const int64_t F = total / mj;
  const int i = (int)(e / F);
  const int64_t f = e - (int64_t)i * F;
  T acc = 0;
  for (int jb = t.job0; jb < t.job0 + t.njob; jb++) {
    const T* in = jobs[jb].in ? (const T*)jobs[jb].in : xbase;
    const T* A = (const T*)jobs[jb].A;
    T sum = 0;
    for (int k = 0; k < mj; k++) sum += A[(int64_t)k * mj + i] * in[mode_addr(j, d0, d1, d2, k, f)];
    acc += (T)jobs[jb].coef * sum;
  }
  T* out = (T*)t.out;
  const int64_t ad = mode_addr(j, d0, d1, d2, i, f);
  if (t.accumulate) out[ad] += acc;
  else out[ad] = acc;
}

}  // namespace attn
