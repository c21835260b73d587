// gfx950 sandwich kernels of the hot path: Y_s += c A X_s B^T over the
// spectator slices s of a node tensor, for the H_eff matvec (two-leg terms and
// local operators) and the effective-operator updates; FP64 / FP32 on the
// 16 x 16 x 4 matrix cores, split BF16 on the 16 x 16 x 32 ones, a generic
// form for legs that are not multiples of 16, and the mixed-shape and
// persistent launches of the batched form.
//
// This file is compiled with the MFMA accumulators in ordinary VGPRs (the
// build passes -amdgpu-mfma-vgpr-form for it alone): with accumulation
// registers the compiler copied the stage-1 accumulators out and back at
// every K step.  The other kernels keep the default form.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"
#include "mfma_common.hpp"
#include "mode_body.hpp"

namespace attn {

// ============================================================================ sandwich
// One work unit = (task, slice s, first 16-row strip).  The WG stages X_s in LDS;
// wave w owns rows [16 (strip0 + w), +16) of Y_s.  Per item:
//   stage 1: T1^T[p][a'] = sum_a X_s[a][p] A[a'][a]           (or X_s^T if A = 1)
//   stage 2: Y^T[p'][a'] += sum_p B[p'][p] T1^T[p][a']        (or T1^T if B = 1)
// Stage 2 consumes the stage-1 accumulators directly as the B operand by
// walking K = p in the order {16 tp + drow(j, i) : j = 0..3} for fixed (tp, i),
// which is exactly how the accumulator layout spreads p over lane groups.
template <typename T, int NB>
__device__ __forceinline__ void sandwich_rows(const SWTask& t, const SWItem* __restrict__ items, int i0, int i1,
                                              void* y, int accumulate, int s, int strip0, const T* lds) {
  typedef typename V4<T>::type v4;
  const int ma = t.ma;
  constexpr int mb = 16 * NB;
  constexpr int ld = mb + 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int strip = strip0 + wave;
  if (strip * 16 >= ma) return;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int arow = strip * 16 + l16;
  const int pc = colperm<T>(l16);   // column read by this lane for an A operand
  int pk[4];                        // column of the contraction index of item i
#pragma unroll
  for (int i = 0; i < 4; i++) pk[i] = colperm<T>(drow<T>(l4, i));
  v4 acc[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) acc[q] = v4{0, 0, 0, 0};
  if (ma == mb) {
    // Square slices (the full nodes): both stages fully unrolled with the
    // operator loads issued a fixed distance ahead of the products that use
    // them (PA A elements, PB groups of NB B elements), each step fenced off
    // so that the scheduler keeps that distance.  Same products in the same
    // order as the general loop below.
    constexpr int KS = mb / 4;
    constexpr int PA = 2;
    constexpr int PB = 2;
    for (int it = i0; it < i1; it++) {
      const T* A = (const T*)items[it].A;
      const T* B = (const T*)items[it].B;
      const T coef = (T)items[it].coef;
      v4 t1[NB];
      if (A) {
#pragma unroll
        for (int q = 0; q < NB; q++) t1[q] = v4{0, 0, 0, 0};
        const T* Ap = A + arow;
        T ab[PA];
#pragma unroll
        for (int k = 0; k < PA; k++) ab[k] = gload(Ap + (int64_t)(4 * k + l4) * mb);
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
          const T bop = ab[ks % PA] * coef;
          if (ks + PA < KS) ab[ks % PA] = gload(Ap + (int64_t)(4 * (ks + PA) + l4) * mb);
          const T* xr = lds + (4 * ks + l4) * ld + pc;
#pragma unroll
          for (int q = 0; q < NB; q++) t1[q] = mfma16(xr[16 * q], bop, t1[q]);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        const T* xr = lds + arow * ld;
#pragma unroll
        for (int q = 0; q < NB; q++)
#pragma unroll
          for (int i = 0; i < 4; i++) t1[q][i] = xr[16 * q + pk[i]] * coef;
      }
      if (B) {
        // group g = (tp, i) = (g / 4, g % 4): the B elements of row 16 tp + pk[i]
        T bb[PB][NB];
#pragma unroll
        for (int g = 0; g < PB; g++)
#pragma unroll
          for (int tq = 0; tq < NB; tq++)
            bb[g][tq] = gload(B + (int64_t)(16 * (g / 4) + pk[g % 4]) * mb + pc + 16 * tq);
#pragma unroll
        for (int g = 0; g < 4 * NB; g++) {
          T bv[NB];
#pragma unroll
          for (int tq = 0; tq < NB; tq++) bv[tq] = bb[g % PB][tq];
          if (g + PB < 4 * NB) {
            const int gn = g + PB;
#pragma unroll
            for (int tq = 0; tq < NB; tq++)
              bb[g % PB][tq] = gload(B + (int64_t)(16 * (gn / 4) + pk[gn % 4]) * mb + pc + 16 * tq);
          }
#pragma unroll
          for (int tq = 0; tq < NB; tq++) acc[tq] = mfma16(bv[tq], t1[g / 4][g % 4], acc[tq]);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NB; q++) acc[q] += t1[q];
      }
    }
  } else
  for (int it = i0; it < i1; it++) {
    const T* A = (const T*)items[it].A;
    const T* B = (const T*)items[it].B;
    const T coef = (T)items[it].coef;
    v4 t1[NB];
    if (A) {
#pragma unroll
      for (int q = 0; q < NB; q++) t1[q] = v4{0, 0, 0, 0};
      const T* Ap = A + arow;
      for (int k0 = 0; k0 < ma; k0 += 4) {
        const T bop = gload(Ap + (int64_t)(k0 + l4) * ma) * coef;
        const T* xr = lds + (k0 + l4) * ld + pc;
#pragma unroll
        for (int q = 0; q < NB; q++) t1[q] = mfma16(xr[16 * q], bop, t1[q]);
      }
    } else {
      const T* xr = lds + arow * ld;
#pragma unroll
      for (int q = 0; q < NB; q++)
#pragma unroll
        for (int i = 0; i < 4; i++) t1[q][i] = xr[16 * q + pk[i]] * coef;
    }
    if (B) {
#pragma unroll
      for (int tp = 0; tp < NB; tp++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const T* Bp = B + (int64_t)(16 * tp + pk[i]) * mb + pc;
#pragma unroll
          for (int tq = 0; tq < NB; tq++) acc[tq] = mfma16(gload(Bp + 16 * tq), t1[tp][i], acc[tq]);
        }
    } else {
#pragma unroll
      for (int q = 0; q < NB; q++) acc[q] += t1[q];
    }
  }
  T* Y = (T*)y + (int64_t)s * t.ys_slice + (int64_t)arow * t.ys_row;
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int q = 0; q < NB; q++) {
      double2* p0 = (double2*)(Y + 16 * q + 2 * l4);
      double2* p1 = (double2*)(Y + 16 * q + 8 + 2 * l4);
      double2 v0 = make_double2(acc[q][0], acc[q][1]), v1 = make_double2(acc[q][2], acc[q][3]);
      if (accumulate) {
        const double2 o0 = *p0, o1 = *p1;
        v0.x += o0.x; v0.y += o0.y; v1.x += o1.x; v1.y += o1.y;
      }
      // streaming stores: each output (a partial sum, a Z tensor) is read once
      // by the next kernel, and not allocating it in L2 keeps the operator
      // blocks there (matvec launches -2 %, effective-operator launches -5 %;
      // the reduction of the partials reads them from HBM, +4 us)
      __builtin_nontemporal_store(dv2{v0.x, v0.y}, (dv2*)p0);
      __builtin_nontemporal_store(dv2{v1.x, v1.y}, (dv2*)p1);
    }
  } else {
#pragma unroll
    for (int q = 0; q < NB; q++) {
      float4* p0 = (float4*)(Y + 16 * q + 4 * l4);
      float4 v = make_float4(acc[q][0], acc[q][1], acc[q][2], acc[q][3]);
      if (accumulate) {
        const float4 o = *p0;
        v.x += o.x; v.y += o.y; v.z += o.z; v.w += o.w;
      }
      *p0 = v;
    }
  }
}


template <typename T, int NB>
__device__ __forceinline__ void sandwich_mfma(const SWTask& t, const SWItem* __restrict__ items,
                                              const int4 wu, const T* __restrict__ xbase,
                                              unsigned char* smem_raw, const SWOut* __restrict__ outs = nullptr) {
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int s = wu.y;
  const int ma = t.ma;
  constexpr int mb = 16 * NB;
  constexpr int ld = mb + 2;
  const T* X = (t.x ? (const T*)t.x : xbase) + (int64_t)s * t.xs_slice;
  for (int e = threadIdx.x; e < ma * mb; e += 256) {
    const int a = e / mb, b = e - a * mb;
    lds[a * ld + b] = X[(int64_t)a * t.xs_row + b];
  }
  __syncthreads();
  if (outs && t.pad) {   // several outputs: items of output o go to outs[o].y
    for (int o = t.item0; o < t.item0 + t.nitem; o++)
      sandwich_rows<T, NB>(t, items, outs[o].item0, outs[o].item0 + outs[o].nitem, outs[o].y, t.accumulate, s,
                           wu.z, lds);
  } else {
    sandwich_rows<T, NB>(t, items, t.item0, t.item0 + t.nitem, t.y, t.accumulate, s, wu.z, lds);
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_sandwich(const SWTask* __restrict__ tasks,
                                                  const SWItem* __restrict__ items,
                                                  const int4* __restrict__ wus,
                                                  const T* __restrict__ xbase,
                                                  const SWOut* __restrict__ outs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  sandwich_mfma<T, NB>(tasks[wu.x], items, wu, xbase, smem_raw, outs);
}

// Generic sandwich for dimensions that are not multiples of 16: one thread per
// output element of one slice.  wu = (task, slice, first element).
template <typename T>
__device__ __forceinline__ void sandwich_gen_elem(const SWTask& t, const SWItem* __restrict__ items,
                                                  int s, int e, const T* __restrict__ xbase) {
  const int ma = t.ma, mb = t.mb;
  if (e >= ma * mb) return;
  const int ap = e / mb, bp = e - ap * mb;
  const T* X = (t.x ? (const T*)t.x : xbase) + (int64_t)s * t.xs_slice;
  T acc = 0;
  for (int it = t.item0; it < t.item0 + t.nitem; it++) {
    const T* A = (const T*)items[it].A;
    const T* B = (const T*)items[it].B;
    T sum = 0;
    for (int b = 0; b < mb; b++) {
      const T bw = B ? B[(int64_t)b * mb + bp] : (b == bp ? (T)1 : (T)0);
      if (bw == (T)0) continue;
      T col = 0;
      if (A) {
        for (int a = 0; a < ma; a++) col += A[(int64_t)a * ma + ap] * X[(int64_t)a * t.xs_row + b];
      } else {
        col = X[(int64_t)ap * t.xs_row + b];
      }
      sum += bw * col;
    }
    acc += (T)items[it].coef * sum;
  }
  T* Y = (T*)t.y + (int64_t)s * t.ys_slice + (int64_t)ap * t.ys_row + bp;
  if (t.accumulate) *Y += acc;
  else *Y = acc;
}

// Small slices (ma mb <= 256, one work unit per slice): the slice, the stage-1
// product and each item's blocks are staged in LDS, so an item costs a few
// LDS passes instead of chains of dependent global loads.  Same arithmetic
// and summation order as sandwich_gen_elem (a zero entry of B adds a zero).
template <typename T>
__device__ __forceinline__ void sandwich_gen_slice(const SWTask& t, const SWItem* __restrict__ items, int s,
                                                   const T* __restrict__ xbase, T* lds) {
  const int ma = t.ma, mb = t.mb, n = ma * mb;
  T* Xs = lds;
  T* T1 = Xs + n;
  T* As = T1 + n;
  T* Bs = As + ma * ma;
  const T* X = (t.x ? (const T*)t.x : xbase) + (int64_t)s * t.xs_slice;
  const int e = threadIdx.x;
  const bool mine = e < n;
  const int ap = mine ? e / mb : 0, bp = mine ? e - ap * mb : 0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int a = q / mb, b = q - a * mb;
    Xs[q] = X[(int64_t)a * t.xs_row + b];
  }
  T acc = 0;
  for (int it = t.item0; it < t.item0 + t.nitem; it++) {
    const T* A = (const T*)items[it].A;
    const T* B = (const T*)items[it].B;
    __syncthreads();
    if (A)
      for (int q = threadIdx.x; q < ma * ma; q += blockDim.x) As[q] = A[q];
    if (B)
      for (int q = threadIdx.x; q < mb * mb; q += blockDim.x) Bs[q] = B[q];
    __syncthreads();
    if (mine) {   // stage 1: T1(ap, bp) = sum_a A(a, ap) X(a, bp)
      T col = 0;
      if (A) {
        for (int a = 0; a < ma; a++) col += As[a * ma + ap] * Xs[a * mb + bp];
      } else {
        col = Xs[ap * mb + bp];
      }
      T1[e] = col;
    }
    __syncthreads();
    if (mine) {   // stage 2: sum_b B(b, bp) T1(ap, b)
      T sum = 0;
      if (B) {
        for (int b = 0; b < mb; b++) sum += Bs[b * mb + bp] * T1[ap * mb + b];
      } else {
        sum = T1[ap * mb + bp];
      }
      acc += (T)items[it].coef * sum;
    }
  }
  if (!mine) return;
  T* Y = (T*)t.y + (int64_t)s * t.ys_slice + (int64_t)ap * t.ys_row + bp;
  if (t.accumulate) *Y += acc;
  else *Y = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_sandwich_gen(const SWTask* __restrict__ tasks,
                                                      const SWItem* __restrict__ items,
                                                      const int4* __restrict__ wus,
                                                      const T* __restrict__ xbase) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  const SWTask& t = tasks[wu.x];
  if (gen_slice_lds(t.ma, t.mb, sizeof(T)))
    sandwich_gen_slice<T>(t, items, wu.y, xbase, reinterpret_cast<T*>(smem_raw));
  else
    sandwich_gen_elem<T>(t, items, wu.y, wu.z + threadIdx.x, xbase);
}

// ============================================================================ split-BF16 sandwich
// Same contraction as k_sandwich with every operand split as hi + lo BF16 and
// three 16x16x32 BF16 products (hi.hi + hi.lo + lo.hi) accumulated in FP32.
// The K index of every product walks a 32-wide chunk in the order
//   slot (g, j) of lane group g -> 32 c + 16 (j / 4) + drow_bf(g, j % 4),
// which is how the stage-1 accumulators spread p over lane groups: stage 2 then
// takes them as its B operand straight from registers.  Operator blocks come in
// that order already (fmt 2 of k_convert); X_s is split and permuted in LDS.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int NB>
__global__ __launch_bounds__(256) void k_sandwich_bf2(const SWTask* __restrict__ tasks,
                                                      const SWItem* __restrict__ items,
                                                      const int4* __restrict__ wus,
                                                      const float* __restrict__ xbase) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  const SWTask& t = tasks[wu.x];
  const int s = wu.y;
  const int ma = t.ma;
  constexpr int mb = 16 * NB;
  const int lda = ma + 8;                      // LDS row = one column b of X_s
  __bf16* xh = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* xl = xh + mb * lda;
  const float* X = (t.x ? (const float*)t.x : xbase) + (int64_t)s * t.xs_slice;
  for (int e = threadIdx.x; e < ma * mb; e += 256) {
    const int a = e / mb, b = e - a * mb;
    const float v = X[(int64_t)a * t.xs_row + b];
    const __bf16 hi = (__bf16)v;
    const __bf16 lo = (__bf16)(v - (float)hi);
    const int pos = bf_pinv(a);
    xh[b * lda + pos] = hi;
    xl[b * lda + pos] = lo;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int strip = wu.z + wave;
  if (strip * 16 >= ma) return;
  const int l16 = lane & 15, g = lane >> 4;
  const int arow = strip * 16 + l16;
  const int64_t mma = (int64_t)ma * ma, mmb = (int64_t)mb * mb;
  f4 acc[NB];
#pragma unroll
  for (int q = 0; q < NB; q++) acc[q] = f4{0, 0, 0, 0};
  const int iend = t.item0 + t.nitem;
  for (int it = t.item0; it < iend; it++) {
    const __bf16* A = (const __bf16*)items[it].A;
    const __bf16* B = (const __bf16*)items[it].B;
    const float coef = (float)items[it].coef;
    f4 t1[NB];
    if (A) {
#pragma unroll
      for (int q = 0; q < NB; q++) t1[q] = f4{0, 0, 0, 0};
      const bf8* Ah = (const bf8*)(A + (int64_t)arow * ma + 8 * g);
      const bf8* Al = (const bf8*)(A + mma + (int64_t)arow * ma + 8 * g);
      for (int c = 0; c < ma / 32; c++) {
        const bf8 ah = Ah[4 * c], al = Al[4 * c];
#pragma unroll
        for (int q = 0; q < NB; q++) {
          const int off = (16 * q + l16) * lda + 32 * c + 8 * g;
          const bf8 vh = *(const bf8*)(xh + off);
          const bf8 vl = *(const bf8*)(xl + off);
          t1[q] = mfma_bf(vh, ah, t1[q]);
          t1[q] = mfma_bf(vh, al, t1[q]);
          t1[q] = mfma_bf(vl, ah, t1[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NB; q++) t1[q] *= coef;
    } else {
      const int pa = bf_pinv(arow);
#pragma unroll
      for (int q = 0; q < NB; q++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int p = 16 * q + drow_bf(g, i);
          t1[q][i] = ((float)xh[p * lda + pa] + (float)xl[p * lda + pa]) * coef;
        }
    }
    if (B) {
#pragma unroll
      for (int c = 0; c < NB / 2; c++) {
        bf8 th, tl;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const float v = t1[2 * c + j / 4][j % 4];
          th[j] = (__bf16)v;
          tl[j] = (__bf16)(v - (float)th[j]);
        }
#pragma unroll
        for (int tq = 0; tq < NB; tq++) {
          const int64_t off = (int64_t)(16 * tq + l16) * mb + 32 * c + 8 * g;
          const bf8 bh = *(const bf8*)(B + off);
          const bf8 bl = *(const bf8*)(B + mmb + off);
          acc[tq] = mfma_bf(bh, th, acc[tq]);
          acc[tq] = mfma_bf(bl, th, acc[tq]);
          acc[tq] = mfma_bf(bh, tl, acc[tq]);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB; q++) acc[q] += t1[q];
    }
  }
  float* Y = (float*)t.y + (int64_t)s * t.ys_slice + (int64_t)arow * t.ys_row;
#pragma unroll
  for (int q = 0; q < NB; q++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int c = 16 * q + drow_bf(g, i);
      if (t.accumulate) Y[c] += acc[q][i];
      else Y[c] = acc[q][i];
    }
}

// Wave-per-slice form for legs <= 64 (ma = 16 MA, mb = 16 NB, both multiples
// of 32; used where one of them is 32): each wave computes a whole slice Y_s
// with all MA row strips in registers, so every fragment of A and B serves MA (or NB) products instead
// of one; the split X_s stays in registers for the whole item loop.  The four
// waves (four slices) share the item's operator blocks through LDS: the blocks
// of item i + 1 are loaded from memory into registers while item i is
// computed from LDS, then written to the other LDS buffer (double buffering,
// one barrier per item).  wu = (task, first slice, -, number of slices <= 4).
template <int MA, int NB>
__global__ __launch_bounds__(256) void k_sandwich_bf2w(const SWTask* __restrict__ tasks,
                                                       const SWItem* __restrict__ items,
                                                       const int4* __restrict__ wus,
                                                       const float* __restrict__ xbase) {
  constexpr int ma = 16 * MA, mb = 16 * NB, CA = ma / 32, CB = mb / 32;
  constexpr int lda = ma + 8, ldb = mb + 8;         // padded LDS rows (conflict-free 16-byte reads)
  constexpr int SA = ma * lda, SB = mb * ldb;       // bf16 per plane in LDS
  constexpr int BUF = 2 * SA + 2 * SB;              // one item: A hi, A lo, B hi, B lo
  constexpr int NA = ma * ma / 8, NBC = mb * mb / 8;  // 16-byte chunks per plane in memory
  constexpr int NTOT = 2 * NA + 2 * NBC, NPT = (NTOT + 255) / 256;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* lds = reinterpret_cast<__bf16*>(smem_raw);
  const int4 wu = wus[blockIdx.x];
  const SWTask& t = tasks[wu.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const bool active = wave < wu.w;
  const int s = wu.y + (active ? wave : 0);
  const int l16 = lane & 15, g = lane >> 4;
  const float* X = (t.x ? (const float*)t.x : xbase) + (int64_t)s * t.xs_slice;
  bf8 xh[CA][NB], xl[CA][NB];
#pragma unroll
  for (int c = 0; c < CA; c++)
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const float v = active ? X[(int64_t)bf_perm(32 * c + 8 * g + j) * t.xs_row + 16 * q + l16] : 0.0f;
        const __bf16 hi = (__bf16)v;
        xh[c][q][j] = hi;
        xl[c][q][j] = (__bf16)(v - (float)hi);
      }
  bf8 pre[NPT];
  auto fetch = [&](int it) {
    const __bf16* A = (const __bf16*)items[it].A;
    const __bf16* B = (const __bf16*)items[it].B;
#pragma unroll
    for (int r = 0; r < NPT; r++) {
      const int ch = tid + 256 * r;
      const __bf16* src = nullptr;
      if (ch < 2 * NA) src = A ? A + (int64_t)ch * 8 : nullptr;
      else if (ch < NTOT) src = B ? B + (int64_t)(ch - 2 * NA) * 8 : nullptr;
      if (src) pre[r] = *(const bf8*)src;
    }
  };
  auto store = [&](int buf) {
    __bf16* L = lds + buf * BUF;
#pragma unroll
    for (int r = 0; r < NPT; r++) {
      const int ch = tid + 256 * r;
      if (ch < 2 * NA) {
        const int e = ch * 8, plane = e / (ma * ma), w = e - plane * ma * ma;
        *(bf8*)(L + plane * SA + (w / ma) * lda + w % ma) = pre[r];
      } else if (ch < NTOT) {
        const int e = (ch - 2 * NA) * 8, plane = e / (mb * mb), w = e - plane * mb * mb;
        *(bf8*)(L + 2 * SA + plane * SB + (w / mb) * ldb + w % mb) = pre[r];
      }
    }
  };
  f4 acc[MA][NB];
#pragma unroll
  for (int a = 0; a < MA; a++)
#pragma unroll
    for (int q = 0; q < NB; q++) acc[a][q] = f4{0, 0, 0, 0};
  const int i0 = t.item0, i1 = t.item0 + t.nitem;
  if (i0 < i1) {
    fetch(i0);
    store(0);
  }
  __syncthreads();
  for (int it = i0; it < i1; it++) {
    const int buf = (it - i0) & 1;
    if (it + 1 < i1) fetch(it + 1);
    const bool hasA = items[it].A != nullptr, hasB = items[it].B != nullptr;
    const float coef = (float)items[it].coef;
    const __bf16* LA = lds + buf * BUF;
    const __bf16* LB = LA + 2 * SA;
    if (active) {
      f4 t1[MA][NB];
      if (hasA) {
#pragma unroll
        for (int a = 0; a < MA; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) t1[a][q] = f4{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < CA; c++) {
          bf8 ah[MA], al[MA];
#pragma unroll
          for (int a = 0; a < MA; a++) {
            const int off = (16 * a + l16) * lda + 32 * c + 8 * g;
            ah[a] = *(const bf8*)(LA + off);
            al[a] = *(const bf8*)(LA + SA + off);
          }
#pragma unroll
          for (int a = 0; a < MA; a++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
              t1[a][q] = mfma_bf(xh[c][q], ah[a], t1[a][q]);
              t1[a][q] = mfma_bf(xh[c][q], al[a], t1[a][q]);
              t1[a][q] = mfma_bf(xl[c][q], ah[a], t1[a][q]);
            }
        }
#pragma unroll
        for (int a = 0; a < MA; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) t1[a][q] *= coef;
      } else {
#pragma unroll
        for (int a = 0; a < MA; a++)
#pragma unroll
          for (int q = 0; q < NB; q++)
#pragma unroll
            for (int i = 0; i < 4; i++)
              t1[a][q][i] = coef * X[(int64_t)(16 * a + l16) * t.xs_row + 16 * q + drow_bf(g, i)];
      }
      if (hasB) {
#pragma unroll
        for (int c = 0; c < CB; c++) {
          bf8 th[MA], tl[MA];
#pragma unroll
          for (int a = 0; a < MA; a++)
#pragma unroll
            for (int jj = 0; jj < 8; jj++) {
              const float v = t1[a][2 * c + jj / 4][jj % 4];
              th[a][jj] = (__bf16)v;
              tl[a][jj] = (__bf16)(v - (float)th[a][jj]);
            }
#pragma unroll
          for (int tq = 0; tq < NB; tq++) {
            const int off = (16 * tq + l16) * ldb + 32 * c + 8 * g;
            const bf8 bh = *(const bf8*)(LB + off);
            const bf8 bl = *(const bf8*)(LB + SB + off);
#pragma unroll
            for (int a = 0; a < MA; a++) {
              acc[a][tq] = mfma_bf(bh, th[a], acc[a][tq]);
              acc[a][tq] = mfma_bf(bl, th[a], acc[a][tq]);
              acc[a][tq] = mfma_bf(bh, tl[a], acc[a][tq]);
            }
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < MA; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) acc[a][q] += t1[a][q];
      }
    }
    if (it + 1 < i1) store(buf ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int a = 0; a < MA; a++) {
    float* Y = (float*)t.y + (int64_t)s * t.ys_slice + (int64_t)(16 * a + l16) * t.ys_row;
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int c = 16 * q + drow_bf(g, i);
        if (t.accumulate) Y[c] += acc[a][q][i];
        else Y[c] = acc[a][q][i];
      }
  }
}

// s_waitcnt vmcnt(n) for n = 0 .. 4, the other counters left alone
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
    case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
    case 1: __builtin_amdgcn_s_waitcnt(0x0F71); break;
    case 2: __builtin_amdgcn_s_waitcnt(0x0F72); break;
    case 3: __builtin_amdgcn_s_waitcnt(0x0F73); break;
    default: __builtin_amdgcn_s_waitcnt(0x0F74); break;
  }
}

// Half-slice form at legs 64 x 64: a work unit is up to four slices, each
// computed by two waves, wave 2 j + h owning the row strips [2 h, 2 h + 2) of
// slice j with its accumulators and stage-1 tiles in registers (every A or B
// fragment serves two or four products; the split X_s stays in registers for
// the whole item loop), so that two waves per SIMD fit (a whole 64 x 64 slice
// per wave takes 400 registers, one wave per SIMD: 191 useful TFLOP/s, half a
// slice per wave with the blocks brought through registers 241, this form
// 291).  The eight waves share every item's operator blocks, moved from memory
// straight into LDS (the gfx950 loads that write LDS, 16 bytes per lane), so
// that no registers hold them in flight and the blocks of item i + 2 load
// while item i is computed (three LDS buffers of 32 KiB: A hi, A lo, B hi,
// B lo).  It is launched at legs 64 x 64 only: a (32, 32) instance of the
// half-slice form gave matvecs 0.5 off (relative) on the device, for a reason
// not found, while the wave-per-slice form fits the registers at legs 32.  A plane is stored without padding, the 16-byte column k of row r
// at position k ^ ((r >> 1) & 7): a load instruction fills 1 KiB of LDS
// contiguously (8 rows), each lane fetching the global column that belongs
// at its position, and the 16 rows read by one MFMA operand fall on distinct
// banks.  Waits are explicit: the compiler does not order these loads
// against the LDS reads of other buffers, and needs not; the loads of item
// i + 1 are older than the ones of item i + 2, so a wave waits until at most
// the latter are outstanding, then all waves meet at a barrier.  Same
// products in the same order as the wave-per-slice form.
template <int MA, int NB>
__global__ __launch_bounds__(512) void k_sandwich_bf2d(const SWTask* __restrict__ tasks,
                                                       const SWItem* __restrict__ items,
                                                       const int4* __restrict__ wus,
                                                       const float* __restrict__ xbase) {
  static_assert(MA == 4 && NB == 4, "legs 64 x 64 only");
  constexpr int m = 64, CA = 2, CB = 2, MW = 2;
  constexpr int PLANE = m * m * 2;   // bytes of one 64 x 64 BF16 plane
  constexpr int BUFB = 4 * PLANE;    // one item
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  const SWTask& t = tasks[wu.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int sj = wave >> 1, a0 = MW * (wave & 1);
  const bool active = sj < wu.w;
  const int s = wu.y + (active ? sj : 0);
  const int l16 = lane & 15, g = lane >> 4;
  const float* X = (t.x ? (const float*)t.x : xbase) + (int64_t)s * t.xs_slice;
  bf8 xh[CA][NB], xl[CA][NB];
#pragma unroll
  for (int c = 0; c < CA; c++)
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const float v = active ? X[(int64_t)bf_perm(32 * c + 8 * g + j) * t.xs_row + 16 * q + l16] : 0.0f;
        const __bf16 hi = (__bf16)v;
        xh[c][q][j] = hi;
        xl[c][q][j] = (__bf16)(v - (float)hi);
      }
  // wave w moves 1-KiB chunks 4 w .. 4 w + 3 of an item: plane w / 2, row blocks
  // 4 (w % 2) .. + 3; lane L takes row L / 8 of the block and LDS position L % 8
  const int wv = __builtin_amdgcn_readfirstlane(wave);   // wave-uniform: block pointers in scalar registers
  const int pl = wv >> 1, drow = lane >> 3, dpos = lane & 7;
  auto dma = [&](int it, int buf) -> int {
    const void* pa = items[it].A;
    const void* pb = items[it].B;
    const __bf16* base = (const __bf16*)(pl < 2 ? pa : pb);
    if (!base) return 0;
    base += (pl & 1) * m * m;
    unsigned char* dst = smem_raw + buf * BUFB + pl * PLANE;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int rb = 4 * (wv & 1) + r, row = 8 * rb + drow;
      const __bf16* src = base + row * m + 8 * (dpos ^ ((row >> 1) & 7));
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(dst + rb * 1024), 16, 0, 0);
    }
    return 4;
  };
  auto frag = [&](const unsigned char* plane, int row, int k) -> bf8 {
    return *(const bf8*)(plane + row * 128 + ((k ^ ((row >> 1) & 7)) << 4));
  };
  f4 acc[MW][NB];
#pragma unroll
  for (int a = 0; a < MW; a++)
#pragma unroll
    for (int q = 0; q < NB; q++) acc[a][q] = f4{0, 0, 0, 0};
  const int i0 = t.item0, i1 = t.item0 + t.nitem;
  if (i0 < i1) dma(i0, 0);
  const int n1 = i0 + 1 < i1 ? dma(i0 + 1, 1) : 0;
  wait_vm(n1);
  __builtin_amdgcn_s_barrier();
  for (int it = i0; it < i1; it++) {
    const int k0 = it - i0;
    const bool hasA = items[it].A != nullptr, hasB = items[it].B != nullptr;
    const float coef = (float)items[it].coef;
    const unsigned char* LB = smem_raw + (k0 % 3) * BUFB;
    f4 t1[MW][NB];
    // without A the stage-1 result is the scaled slice itself, read from memory
    // before this iteration's block loads are issued (so that waiting for it
    // does not wait for them)
    if (active && !hasA) {
#pragma unroll
      for (int a = 0; a < MW; a++)
#pragma unroll
        for (int q = 0; q < NB; q++)
#pragma unroll
          for (int i = 0; i < 4; i++)
            t1[a][q][i] = coef * X[(int64_t)(16 * (a0 + a) + l16) * t.xs_row + 16 * q + drow_bf(g, i)];
    }
    const int n2 = it + 2 < i1 ? dma(it + 2, (k0 + 2) % 3) : 0;
    if (active) {
      if (hasA) {
#pragma unroll
        for (int a = 0; a < MW; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) t1[a][q] = f4{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < CA; c++) {
          bf8 ah[MW], al[MW];
#pragma unroll
          for (int a = 0; a < MW; a++) {
            const int row = 16 * (a0 + a) + l16;
            ah[a] = frag(LB, row, 4 * c + g);
            al[a] = frag(LB + PLANE, row, 4 * c + g);
          }
#pragma unroll
          for (int a = 0; a < MW; a++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
              t1[a][q] = mfma_bf(xh[c][q], ah[a], t1[a][q]);
              t1[a][q] = mfma_bf(xh[c][q], al[a], t1[a][q]);
              t1[a][q] = mfma_bf(xl[c][q], ah[a], t1[a][q]);
            }
        }
#pragma unroll
        for (int a = 0; a < MW; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) t1[a][q] *= coef;
      }
      if (hasB) {
#pragma unroll
        for (int c = 0; c < CB; c++) {
          bf8 th[MW], tl[MW];
#pragma unroll
          for (int a = 0; a < MW; a++)
#pragma unroll
            for (int jj = 0; jj < 8; jj++) {
              const float v = t1[a][2 * c + jj / 4][jj % 4];
              th[a][jj] = (__bf16)v;
              tl[a][jj] = (__bf16)(v - (float)th[a][jj]);
            }
#pragma unroll
          for (int tq = 0; tq < NB; tq++) {
            const int row = 16 * tq + l16;
            const bf8 bh = frag(LB + 2 * PLANE, row, 4 * c + g);
            const bf8 bl = frag(LB + 3 * PLANE, row, 4 * c + g);
#pragma unroll
            for (int a = 0; a < MW; a++) {
              acc[a][tq] = mfma_bf(bh, th[a], acc[a][tq]);
              acc[a][tq] = mfma_bf(bl, th[a], acc[a][tq]);
              acc[a][tq] = mfma_bf(bh, tl[a], acc[a][tq]);
            }
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < MW; a++)
#pragma unroll
          for (int q = 0; q < NB; q++) acc[a][q] += t1[a][q];
      }
    }
    // the blocks of item it + 1 (issued one iteration ago) have landed once at
    // most the n2 loads of item it + 2 are outstanding; then nobody reads buffer
    // k0 % 3 any more either, which item it + 3 will overwrite
    wait_vm(n2);
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS reads are done
    __builtin_amdgcn_s_barrier();
  }
  if (!active) return;
#pragma unroll
  for (int a = 0; a < MW; a++) {
    float* Y = (float*)t.y + (int64_t)s * t.ys_slice + (int64_t)(16 * (a0 + a) + l16) * t.ys_row;
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int c = 16 * q + drow_bf(g, i);
        if (t.accumulate) Y[c] += acc[a][q][i];
        else Y[c] = acc[a][q][i];
      }
  }
}

// LDS of the wave-per-slice form: two buffers of one item's four padded planes
template <int MA, int NB>
constexpr size_t bf2w_lds() { return (size_t)2 * (2 * 16 * MA * (16 * MA + 8) + 2 * 16 * NB * (16 * NB + 8)) * 2; }

// ============================================================================ two strips per wave
// FP32 at legs 64 x 64: a work unit is up to two slices, wave w computing rows
// [32 (w % 2), +32) of slice w / 2 as two 16-row strips.  Each operand value
// then feeds two products: the slice element read from LDS in stage 1 serves
// both strips' A rows, and each B element loaded in stage 2 serves both
// strips' stage-1 tiles, so the operand loads per MFMA halve (the FP32 MFMA
// runs twice as fast as the FP64 one and the one-strip form waits for its
// operands).  Per output element the same products in the same order as
// sandwich_rows, so the results are the same bit for bit.
// slices s0 .. s0 + ns - 1 (ns <= 2) of task t
template <typename T>
__device__ __forceinline__ void sandwich_w2(const SWTask& t, const SWItem* __restrict__ items, int s0, int ns,
                                            const T* __restrict__ xbase, unsigned char* smem_raw) {
  typedef typename V4<T>::type v4;
  constexpr int NB = 4, mb = 64, ld = mb + 2, KS = mb / 4, PA = 2, PB = 2;
  T* lds = reinterpret_cast<T*>(smem_raw);
  for (int j = 0; j < ns; j++) {
    const T* X = (t.x ? (const T*)t.x : xbase) + (int64_t)(s0 + j) * t.xs_slice;
    T* L = lds + j * mb * ld;
    for (int e = threadIdx.x; e < mb * mb; e += 256) {
      const int a = e / mb, b = e - a * mb;
      L[a * ld + b] = X[(int64_t)a * t.xs_row + b];
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = wave >> 1;
  if (j >= ns) return;   // no barrier below
  const int s = s0 + j;
  const T* L = lds + j * mb * ld;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int r0 = 32 * (wave & 1);
  const int pc = colperm<T>(l16);
  int pk[4];
#pragma unroll
  for (int i = 0; i < 4; i++) pk[i] = colperm<T>(drow<T>(l4, i));
  v4 acc[2][NB];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int q = 0; q < NB; q++) acc[a][q] = v4{0, 0, 0, 0};
  for (int it = t.item0; it < t.item0 + t.nitem; it++) {
    const T* A = (const T*)items[it].A;
    const T* B = (const T*)items[it].B;
    const T coef = (T)items[it].coef;
    v4 t1[2][NB];
    if (A) {
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < NB; q++) t1[a][q] = v4{0, 0, 0, 0};
      const T* Ap = A + r0 + l16;
      T ab[PA][2];
#pragma unroll
      for (int k = 0; k < PA; k++)
#pragma unroll
        for (int a = 0; a < 2; a++) ab[k][a] = gload(Ap + 16 * a + (int64_t)(4 * k + l4) * mb);
#pragma unroll
      for (int ks = 0; ks < KS; ks++) {
        T bop[2];
#pragma unroll
        for (int a = 0; a < 2; a++) bop[a] = ab[ks % PA][a] * coef;
        if (ks + PA < KS)
#pragma unroll
          for (int a = 0; a < 2; a++) ab[ks % PA][a] = gload(Ap + 16 * a + (int64_t)(4 * (ks + PA) + l4) * mb);
        const T* xr = L + (4 * ks + l4) * ld + pc;
#pragma unroll
        for (int q = 0; q < NB; q++) {
          const T xv = xr[16 * q];
#pragma unroll
          for (int a = 0; a < 2; a++) t1[a][q] = mfma16(xv, bop[a], t1[a][q]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 2; a++) {
        const T* xr = L + (r0 + 16 * a + l16) * ld;
#pragma unroll
        for (int q = 0; q < NB; q++)
#pragma unroll
          for (int i = 0; i < 4; i++) t1[a][q][i] = xr[16 * q + pk[i]] * coef;
      }
    }
    if (B) {
      T bb[PB][NB];
#pragma unroll
      for (int g = 0; g < PB; g++)
#pragma unroll
        for (int tq = 0; tq < NB; tq++)
          bb[g][tq] = gload(B + (int64_t)(16 * (g / 4) + pk[g % 4]) * mb + pc + 16 * tq);
#pragma unroll
      for (int g = 0; g < 4 * NB; g++) {
        T bv[NB];
#pragma unroll
        for (int tq = 0; tq < NB; tq++) bv[tq] = bb[g % PB][tq];
        if (g + PB < 4 * NB) {
          const int gn = g + PB;
#pragma unroll
          for (int tq = 0; tq < NB; tq++)
            bb[g % PB][tq] = gload(B + (int64_t)(16 * (gn / 4) + pk[gn % 4]) * mb + pc + 16 * tq);
        }
#pragma unroll
        for (int tq = 0; tq < NB; tq++)
#pragma unroll
          for (int a = 0; a < 2; a++) acc[a][tq] = mfma16(bv[tq], t1[a][g / 4][g % 4], acc[a][tq]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int q = 0; q < NB; q++) acc[a][q] += t1[a][q];
    }
  }
#pragma unroll
  for (int a = 0; a < 2; a++) {
    T* Y = (T*)t.y + (int64_t)s * t.ys_slice + (int64_t)(r0 + 16 * a + l16) * t.ys_row;
#pragma unroll
    for (int q = 0; q < NB; q++) {
      float4* p0 = (float4*)(Y + 16 * q + 4 * l4);
      float4 v = make_float4(acc[a][q][0], acc[a][q][1], acc[a][q][2], acc[a][q][3]);
      if (t.accumulate) {
        const float4 o = *p0;
        v.x += o.x; v.y += o.y; v.z += o.z; v.w += o.w;
      }
      *p0 = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sandwich_w2(const SWTask* __restrict__ tasks,
                                                     const SWItem* __restrict__ items,
                                                     const int4* __restrict__ wus,
                                                     const T* __restrict__ xbase) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  sandwich_w2<T>(tasks[wu.x], items, wu.y, wu.w, xbase, smem_raw);
}

// ============================================================================ mixed-shape launches
// One launch over the work units of many tasks of different shapes (several
// nodes of several problem instances): the kind of each unit selects the body.
// Sandwich: wu.w = NB (legs multiples of 16, mb = 16 NB <= 64) or 0 (generic).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_sandwich(const SWTask* __restrict__ tasks,
                                                        const SWItem* __restrict__ items,
                                                        const int4* __restrict__ wus) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int4 wu = wus[blockIdx.x];
  const SWTask& t = tasks[wu.x];
  switch (wu.w) {
    case 0:
      if (gen_slice_lds(t.ma, t.mb, sizeof(T)))
        sandwich_gen_slice<T>(t, items, wu.y, nullptr, reinterpret_cast<T*>(smem_raw));
      else
        sandwich_gen_elem<T>(t, items, wu.y, wu.z + threadIdx.x, nullptr);
      break;
    case 1: sandwich_mfma<T, 1>(t, items, wu, nullptr, smem_raw); break;
    case 2: sandwich_mfma<T, 2>(t, items, wu, nullptr, smem_raw); break;
    case 3: sandwich_mfma<T, 3>(t, items, wu, nullptr, smem_raw); break;
    case 4: sandwich_mfma<T, 4>(t, items, wu, nullptr, smem_raw); break;
    default: break;
  }
}

// ============================================================================ persistent batched matvec
// The staged batched matvec is six launches (transposes, three chain stages,
// sandwiches, reduction); here one launch of a resident grid runs them all
// from one ordered work list (PUnit), so later stages start while earlier
// units of other instances still run.  Every unit runs the same body as in
// the staged launches, and the reduction sums in the same fixed order, so the
// results are the same bit for bit.
//
// Ordering across the chip (eight XCDs, each with its own L2): before a
// count is published every wave waits for its stores, and one device-scope
// release writes the L2 back; a waiting workgroup polls the counter from one
// lane and takes a device-scope acquire before reading what producers wrote.
// Without the release the results are wrong (non-finite energies in a test
// build); the acquire measured free.
//
// Measured (32 seeded Ising instances, L 8..16, m 16..64, graphs): FP32
// sweep 2.97 s against 2.25 s staged, FP64 3.82 s against 3.11 s.  A
// per-unit timestamp trace put the remaining gap in per-ticket latency
// (ticket atomic, descriptor loads, publish: about 5 us between units) and in
// the reduction tail; the staged launches stay the default.
template <typename T>
__device__ __forceinline__ void pm_transpose(const TRTask& t, int64_t e0) {
  const int64_t M = (int64_t)t.ml * t.mr * t.mp;
  const int64_t e1 = e0 + kPmTileT < M ? e0 + kPmTileT : M;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int64_t l = e / ((int64_t)t.mr * t.mp);
    const int64_t rem = e - l * t.mr * t.mp;
    const int64_t r = rem / t.mp, p = rem - r * t.mp;
    ((T*)t.xt)[p * t.ml * t.mr + l * t.mr + r] = ((const T*)t.x)[e];
  }
}

// same per-element sum as k_reduce_list
template <typename TI>
__device__ __forceinline__ void pm_reduce(const RDTask& t, int64_t e0) {
  const int64_t M = (int64_t)t.ml * t.mr * t.mp;
  const int64_t e1 = e0 + kPmTileR < M ? e0 + kPmTileR : M;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int64_t l = e / ((int64_t)t.mr * t.mp);
    const int64_t rem = e - l * t.mr * t.mp;
    const int64_t r = rem / t.mp, p = rem - r * t.mp;
    const int64_t et = p * t.ml * t.mr + l * t.mr + r;
    double acc = 0;
#pragma unroll 8
    for (int k = 0; k < t.nsrc; k++) acc += (double)((const TI*)t.srcs[k].p)[t.srcs[k].layout ? et : e];
    ((double*)t.y)[e] = acc;
  }
}

// One mode-product or sandwich unit.  Not inlined: inside the persistent
// loop the compiler would otherwise keep the lane-dependent set-up of every
// body live at once (over 300 registers for FP64).  As calls under the
// occupancy cap of the kernel below, they save a few registers at entry and
// exit and spill nothing inside.  Arguments of a call arrive in vector
// registers, so each is made wave-uniform again (scalar loads of the task and
// item descriptors, uniform branches), and the LDS buffer is named here, not
// passed, so that it is addressed as LDS rather than through flat pointers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// a descriptor list (read-only while the kernel runs) at a wave-uniform
// address, read through the constant address space: scalar loads
template <typename P>
__device__ __forceinline__ const P* uni(const P* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const P*)(const __attribute__((address_space(4))) P*)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __noinline__ void pm_mode(const MPTask* tp, const MPJob* jobs_, int task_, int c_) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const MPTask& t = *uni(tp);
  const MPJob* jobs = uni(jobs_);
  const int task = uni(task_), c = uni(c_);
  const int2 wu = make_int2(task, c);
  switch (t.pad) {
    case 0: mode_gen_elem<T>(t, jobs, (int64_t)c + threadIdx.x, nullptr); break;
    case 1: mode_mfma<T, 1>(t, jobs, wu, nullptr, smem_raw); break;
    case 2: mode_mfma<T, 2>(t, jobs, wu, nullptr, smem_raw); break;
    case 3: mode_mfma<T, 3>(t, jobs, wu, nullptr, smem_raw); break;
    case 4: mode_mfma<T, 4>(t, jobs, wu, nullptr, smem_raw); break;
    default: break;
  }
}

template <typename T>
__device__ __noinline__ void pm_sandwich(const SWTask* tp, const SWItem* items_, int task_, int s_, int z_,
                                         int body_) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SWTask& t = *uni(tp);
  const SWItem* items = uni(items_);
  const int task = uni(task_), s = uni(s_), z = uni(z_), body = uni(body_);
  const int4 wu = make_int4(task, s, z, body);
  switch (body) {
    case 0:
      if (gen_slice_lds(t.ma, t.mb, sizeof(T)))
        sandwich_gen_slice<T>(t, items, s, nullptr, reinterpret_cast<T*>(smem_raw));
      else
        sandwich_gen_elem<T>(t, items, s, z + threadIdx.x, nullptr);
      break;
    case 1: sandwich_mfma<T, 1>(t, items, wu, nullptr, smem_raw); break;
    case 2: sandwich_mfma<T, 2>(t, items, wu, nullptr, smem_raw); break;
    case 3: sandwich_mfma<T, 3>(t, items, wu, nullptr, smem_raw); break;
    case 4: sandwich_mfma<T, 4>(t, items, wu, nullptr, smem_raw); break;
    default: break;
  }
}

// Three (FP64) or four (FP32) workgroups per CU (FP32 at five: registers
// capped at 96, the mode body spills, and the sweep measured 8 % slower).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4)))
void k_batch_matvec(const PMArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_ticket, s_flag;
  // Signals are deferred: a workgroup sums the count of its finished units on
  // one counter and publishes it (one release) before it waits for anything,
  // when its next ticket signals another counter, after kPmDefer tickets, and
  // when it leaves.  It never waits while holding a count, so every count is
  // published after at most kPmDefer tickets that need nothing.
  int pend_sig = -1, pend_cnt = 0, pend_age = 0;   // same in every lane
  // the last (counter, need) this workgroup waited for: later tickets with
  // the same counter and no larger need are ready, and its acquire still holds
  int seen_wait = -1, seen_need = 0;
  auto publish = [&]() {
    // every wave waits until its own stores have reached the L2 of its XCD;
    // after the barrier one release by lane 0 writes that L2 back (covering
    // the stores of all four waves) and publishes the count
    wait_vm(0);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(a.cnt + pend_sig * kPmStride, pend_cnt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    pend_sig = -1;
    pend_cnt = 0;
    pend_age = 0;
  };
  for (;;) {
    if (threadIdx.x == 0) {
      const int q = blockIdx.x % kPmQueues;
      s_ticket = q + kPmQueues * __hip_atomic_fetch_add(a.cnt + q * kPmStride, 1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int tk = uni(s_ticket);
    if (tk >= a.n_tickets) break;
    // a ticket is a run of consecutive units with the same wait and signal
    const int32_t* tickets = uni(a.tickets);
    const PUnit* units = uni(a.units);
    const int u0 = tickets[tk], u1 = tickets[tk + 1];
    const int wait = units[u0].wait, need = units[u0].need, signal = units[u0].signal;
    const bool ready = wait < 0 || (wait == seen_wait && need <= seen_need);
    if (pend_cnt && (!ready || signal != pend_sig || pend_age >= kPmDefer)) publish();
    if (!ready) {
      if (threadIdx.x == 0) {
        int ok = 1;
        for (int it = 0;; it++) {
          if (__hip_atomic_load(a.cnt + wait * kPmStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need)
            break;
          if (__hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
          if (it >= kPmSpin) {
            __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
        // pairs with the producers' release; the CU's vector cache is shared
        // by the workgroup's waves, so one wave's acquire serves all of them
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_flag = ok;
      }
      __syncthreads();
      if (!s_flag) continue;   // aborted: skip the bodies (their counter is never needed again)
      seen_wait = wait;
      seen_need = need;
    }
    for (int ui = u0; ui < u1; ui++) {
      const PUnit u = units[ui];
      if (ui > u0) __syncthreads();   // LDS of the previous unit
      switch (u.kind) {
        case PU_TRANSPOSE: pm_transpose<T>(a.tr[u.a], u.b); break;
        case PU_REDUCE: pm_reduce<T>(a.rd[u.a], u.b); break;
        case PU_MODE: pm_mode<T>(a.mp_tasks[u.a] + u.b, a.mp_jobs[u.a], u.b, u.c); break;
        case PU_SANDWICH: pm_sandwich<T>(a.sw_tasks + u.a, a.sw_items, u.a, u.b, u.c, u.d); break;
        default: break;
      }
    }
    __syncthreads();   // frees LDS and s_ticket for the next ticket
    if (signal >= 0) {
      pend_sig = signal;
      pend_cnt += u1 - u0;
      pend_age++;
    }
  }
  if (pend_cnt) publish();
  // the last workgroup out leaves every counter at zero for the next launch
  if (threadIdx.x == 0)
    s_flag = __hip_atomic_fetch_add(a.cnt + kPmExit * kPmStride, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
             (int)gridDim.x - 1;
  __syncthreads();
  if (s_flag)
    for (int i = threadIdx.x; i < a.n_cnt; i += 256)
      __hip_atomic_store(a.cnt + i * kPmStride, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ============================================================================ launchers
template <typename T, int NB>
static hipError_t sand_launch(const SWTask* tasks, const SWItem* items, const int4* wus, int nwu,
                              int ma, const void* xbase, hipStream_t s, const SWOut* outs) {
  const size_t lds = (size_t)ma * (16 * NB + 2) * sizeof(T);
  hipLaunchKernelGGL((k_sandwich<T, NB>), dim3(nwu), dim3(256), lds, s, tasks, items, wus,
                     (const T*)xbase, outs);
  return hipGetLastError();
}

template <int NB>
static hipError_t sand_bf2_launch(const SWTask* tasks, const SWItem* items, const int4* wus, int nwu,
                                  int ma, const void* xbase, hipStream_t s) {
  const size_t lds = (size_t)2 * (16 * NB) * (ma + 8) * sizeof(__bf16);
  hipLaunchKernelGGL((k_sandwich_bf2<NB>), dim3(nwu), dim3(256), lds, s, tasks, items, wus,
                     (const float*)xbase);
  return hipGetLastError();
}

hipError_t launch_sandwich(int dtype, int ma, int mb, const SWTask* tasks, const SWItem* items,
                           const int4* wus, int nwu, const void* xbase, hipStream_t s, const SWOut* outs) {
  if (nwu == 0) return hipSuccess;
  if (dtype == 3) {   // split BF16, one slice per wave (legs 32 or 64)
#define BF2W(MA, NB)                                                                             \
  {                                                                                              \
    const size_t lds = bf2w_lds<MA, NB>();                                                       \
    hipLaunchKernelGGL((k_sandwich_bf2w<MA, NB>), dim3(nwu), dim3(256), lds, s, tasks, items, wus, \
                       (const float*)xbase);                                                     \
    return hipGetLastError();                                                                    \
  }
    if (ma == 32 && mb == 32) BF2W(2, 2)
    if (ma == 32 && mb == 64) BF2W(2, 4)
    if (ma == 64 && mb == 32) BF2W(4, 2)
#undef BF2W
    if (ma == 64 && mb == 64) {
      const size_t lds = 3 * 4 * 64 * 64 * sizeof(__bf16);   // three buffers of one item's four planes
      hipLaunchKernelGGL((k_sandwich_bf2d<4, 4>), dim3(nwu), dim3(512), lds, s, tasks, items, wus,
                         (const float*)xbase);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (dtype == 4) {   // FP32, legs 64 x 64, two strips per wave, units of up to two slices
    if (ma != 64 || mb != 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sandwich_w2<float>, dim3(nwu), dim3(256), (size_t)2 * 64 * 66 * sizeof(float), s, tasks,
                       items, wus, (const float*)xbase);
    return hipGetLastError();
  }
  if (dtype == 2) {
    if (!(ma % 32 == 0 && mb % 32 == 0 && ma <= 128 && mb <= 128)) return hipErrorInvalidValue;
    switch (mb / 32) {
      case 1: return sand_bf2_launch<2>(tasks, items, wus, nwu, ma, xbase, s);
      case 2: return sand_bf2_launch<4>(tasks, items, wus, nwu, ma, xbase, s);
      case 3: return sand_bf2_launch<6>(tasks, items, wus, nwu, ma, xbase, s);
      case 4: return sand_bf2_launch<8>(tasks, items, wus, nwu, ma, xbase, s);
    }
    return hipErrorInvalidValue;
  }
  const bool mf = (ma % 16 == 0) && (mb % 16 == 0) && ma <= 128 && mb <= 128;
  if (dtype == 0) {
    if (!mf) {
      hipLaunchKernelGGL(k_sandwich_gen<double>, dim3(nwu), dim3(256), gen_slice_lds(ma, mb, 8), s, tasks, items,
                         wus, (const double*)xbase);
      return hipGetLastError();
    }
    switch (mb / 16) {
      case 1: return sand_launch<double, 1>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 2: return sand_launch<double, 2>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 3: return sand_launch<double, 3>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 4: return sand_launch<double, 4>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 5: return sand_launch<double, 5>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 6: return sand_launch<double, 6>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 7: return sand_launch<double, 7>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 8: return sand_launch<double, 8>(tasks, items, wus, nwu, ma, xbase, s, outs);
    }
  } else {
    if (!mf) {
      hipLaunchKernelGGL(k_sandwich_gen<float>, dim3(nwu), dim3(256), gen_slice_lds(ma, mb, 4), s, tasks, items,
                         wus, (const float*)xbase);
      return hipGetLastError();
    }
    switch (mb / 16) {
      case 1: return sand_launch<float, 1>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 2: return sand_launch<float, 2>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 3: return sand_launch<float, 3>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 4: return sand_launch<float, 4>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 5: return sand_launch<float, 5>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 6: return sand_launch<float, 6>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 7: return sand_launch<float, 7>(tasks, items, wus, nwu, ma, xbase, s, outs);
      case 8: return sand_launch<float, 8>(tasks, items, wus, nwu, ma, xbase, s, outs);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_sandwich(int dtype, const SWTask* tasks, const SWItem* items, const int4* wus,
                                 int nwu, size_t lds, hipStream_t s) {
  if (nwu == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_batch_sandwich<double>, dim3(nwu), dim3(256), lds, s, tasks, items, wus);
  else
    hipLaunchKernelGGL(k_batch_sandwich<float>, dim3(nwu), dim3(256), lds, s, tasks, items, wus);
  return hipGetLastError();
}

hipError_t launch_batch_matvec(int dtype, const PMArgs& a, int grid, size_t lds, hipStream_t s) {
  if (a.n_units == 0) return hipSuccess;
  if (grid < kPmQueues) return hipErrorInvalidValue;   // every queue needs a workgroup
  if (dtype == 0)
    hipLaunchKernelGGL(k_batch_matvec<double>, dim3(grid), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(k_batch_matvec<float>, dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

// Resident workgroups per CU of the persistent batched matvec at `lds` bytes.
hipError_t batch_matvec_occupancy(int dtype, size_t lds, int* per_cu) {
  const void* f = dtype == 0 ? (const void*)k_batch_matvec<double> : (const void*)k_batch_matvec<float>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, 256, lds);
}

// Dynamic-LDS limit of the sandwich kernels (called by prepare_kernel_attributes).
hipError_t prepare_sandwich_attributes() {
  const void* fns[] = {
      (const void*)k_batch_sandwich<double>, (const void*)k_batch_sandwich<float>,
      (const void*)k_sandwich<double, 1>, (const void*)k_sandwich<double, 2>,
      (const void*)k_sandwich<double, 3>, (const void*)k_sandwich<double, 4>,
      (const void*)k_sandwich<double, 5>, (const void*)k_sandwich<double, 6>,
      (const void*)k_sandwich<double, 7>, (const void*)k_sandwich<double, 8>,
      (const void*)k_sandwich<float, 1>, (const void*)k_sandwich<float, 2>,
      (const void*)k_sandwich<float, 3>, (const void*)k_sandwich<float, 4>,
      (const void*)k_sandwich<float, 5>, (const void*)k_sandwich<float, 6>,
      (const void*)k_sandwich<float, 7>, (const void*)k_sandwich<float, 8>,
      (const void*)k_sandwich_bf2<2>, (const void*)k_sandwich_bf2<4>,
      (const void*)k_sandwich_bf2w<2, 2>, (const void*)k_sandwich_bf2w<2, 4>,
      (const void*)k_sandwich_bf2w<4, 2>, (const void*)k_sandwich_bf2d<4, 4>,
      (const void*)k_sandwich_bf2<6>, (const void*)k_sandwich_bf2<8>, (const void*)k_sandwich_w2<float>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  for (const void* f : {(const void*)k_batch_matvec<double>, (const void*)k_batch_matvec<float>}) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kPmMaxLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace attn
