// gfx950 kernels of the aTTN hot path (the sandwich kernels are in sandwich.hip).
//
// Dense contractions run on the matrix cores with 16 x 16 x 4 MFMA tiles.
// FP64 and FP32 share the operand layout (A lane l -> (row l%16, k l/16),
// B lane l -> (k l/16, col l%16)); the accumulator rows differ: item i of lane
// l holds D[l/16 + 4 i][l%16] for FP64 and D[4 (l/16) + i][l%16] for FP32
// (checked on the device by a probe of both instructions).
// Every kernel reads a device work list so that one launch covers many terms,
// output blocks or instances.  Reductions are two-stage with a fixed block
// count and a fixed summation order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"
#include "mfma_common.hpp"
#include "mode_body.hpp"

namespace attn {

// A failure status of the eigensolver / QR state, also collected in the
// sticky word that sweeps read once at their end.
__device__ __forceinline__ void fail_status(KrylovState* st, int v) {
  st->status = v;
  atomicOr(&st->sticky, v);
}

// ============================================================================ mode product
// (device bodies: mode_body.hpp)
template <typename T, int NI, int QS>
__global__ __launch_bounds__(256) void k_mode(const MPTask* __restrict__ tasks,
                                              const MPJob* __restrict__ jobs,
                                              const int2* __restrict__ wus,
                                              const T* __restrict__ xbase) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 wu = wus[blockIdx.x];
  mode_mfma<T, NI, QS>(tasks[wu.x], jobs, wu, xbase, smem_raw);
}

// Mode product for contracted leg j = 0 or 1 with 16 | d2: a 16-wide tile of
// the free index is contiguous in memory for every i', so both operands are
// loaded straight into registers (no LDS, no barriers).  wu = (task, 64-wide
// free block); the block is split over blockIdx.y into QS sub-blocks, and a
// workgroup's four waves take (4 / QS) tiles of 16 free indices times QS
// groups of output rows (QS = 1: each wave all m_j rows of its own tile).
// Every output entry sums its products in the same order whatever QS is.
template <typename T, int NI, int QS>
__global__ __launch_bounds__(256) void k_mode_nt(const MPTask* __restrict__ tasks, const MPJob* __restrict__ jobs,
                                                 const int2* __restrict__ wus, const T* __restrict__ xbase) {
  typedef typename V4<T>::type v4;
  constexpr int mj = 16 * NI, NQ = NI / QS;   // output row blocks per wave
  const int2 wu = wus[blockIdx.x];
  const MPTask& t = tasks[wu.x];
  const int j = t.j, d1 = t.d1, d2 = t.d2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int tile = (4 / QS) * blockIdx.y + wave / QS, q0 = (wave % QS) * NQ;
  const int64_t F = (int64_t)t.d0 * d1 * d2 / mj;
  const int64_t f = (int64_t)wu.y * 64 + 16 * tile + l16;
  // (i, f) -> address; the tile's f share one a-row when j = 1
  int64_t fo, fs;   // address = fo + i * fs
  if (j == 0) { fo = f; fs = F; }
  else { const int64_t a = f / d2, c = f - a * d2; fo = a * d1 * d2 + c; fs = d2; }
  v4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) acc[q] = v4{0, 0, 0, 0};
  for (int jb = t.job0; jb < t.job0 + t.njob; jb++) {
    const T* in = jobs[jb].in ? (const T*)jobs[jb].in : xbase;
    const T* A = (const T*)jobs[jb].A + 16 * q0 + l16;
    const T coef = (T)jobs[jb].coef;
#pragma unroll 4
    for (int k0 = 0; k0 < mj; k0 += 4) {
      const T bop = in[fo + (int64_t)(k0 + l4) * fs] * coef;
      const T* Ak = A + (int64_t)(k0 + l4) * mj;
#pragma unroll
      for (int q = 0; q < NQ; q++) acc[q] = mfma16(Ak[16 * q], bop, acc[q]);
    }
  }
  T* out = (T*)t.out;
#pragma unroll
  for (int q = 0; q < NQ; q++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t ad = fo + (int64_t)(16 * (q0 + q) + drow<T>(l4, i)) * fs;
      if (t.accumulate) out[ad] += acc[q][i];
      else out[ad] = acc[q][i];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mode_gen(const MPTask* __restrict__ tasks,
                                                  const MPJob* __restrict__ jobs,
                                                  const int2* __restrict__ wus,
                                                  const T* __restrict__ xbase) {
  const int2 wu = wus[blockIdx.x];
  mode_gen_elem<T>(tasks[wu.x], jobs, (int64_t)wu.y + threadIdx.x, xbase);
}

// ============================================================================ mixed-shape launches
// One launch over the work units of many tasks of different shapes (several
// nodes of several problem instances): the kind of each unit selects the body.
// Mode product: the task's kind (MPTask::pad) is NI (m_j = 16 NI <= 64) or 0 (generic).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_mode(const MPTask* __restrict__ tasks,
                                                    const MPJob* __restrict__ jobs,
                                                    const int2* __restrict__ wus) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 wu = wus[blockIdx.x];
  const MPTask& t = tasks[wu.x];
  switch (t.pad) {
    case 0: mode_gen_elem<T>(t, jobs, (int64_t)wu.y + threadIdx.x, nullptr); break;
    case 1: mode_mfma<T, 1>(t, jobs, wu, nullptr, smem_raw); break;
    case 2: mode_mfma<T, 2>(t, jobs, wu, nullptr, smem_raw); break;
    case 3: mode_mfma<T, 3>(t, jobs, wu, nullptr, smem_raw); break;
    case 4: mode_mfma<T, 4>(t, jobs, wu, nullptr, smem_raw); break;
    default: break;
  }
}

// [l][r][p] -> [p][l][r] for a list of tensors (task blockIdx.y)
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_list(const TRTask* __restrict__ tasks) {
  const TRTask& t = tasks[blockIdx.y];
  const int64_t M = (int64_t)t.ml * t.mr * t.mp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const int64_t l = e / ((int64_t)t.mr * t.mp);
    const int64_t rem = e - l * t.mr * t.mp;
    const int64_t r = rem / t.mp, p = rem - r * t.mp;
    ((T*)t.xt)[p * t.ml * t.mr + l * t.mr + r] = ((const T*)t.x)[e];
  }
}

// y = sum of the partial outputs of each task (fixed order), as k_reduce_out
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_reduce_list(const RDTask* __restrict__ tasks) {
  const RDTask& t = tasks[blockIdx.y];
  const int64_t M = (int64_t)t.ml * t.mr * t.mp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const int64_t l = e / ((int64_t)t.mr * t.mp);
    const int64_t rem = e - l * t.mr * t.mp;
    const int64_t r = rem / t.mp, p = rem - r * t.mp;
    const int64_t et = p * t.ml * t.mr + l * t.mr + r;
    double acc = 0;
    for (int k = 0; k < t.nsrc; k++) acc += (double)((const TI*)t.srcs[k].p)[t.srcs[k].layout ? et : e];
    ((TO*)t.y)[e] = (TO)acc;
  }
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = 0.0;
}

// dst = src (a kernel rather than a copy command, so that captured sweeps
// hold kernel nodes only)
__global__ __launch_bounds__(256) void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}

// ============================================================================ gram
// partial[j][j'] (column-major) = sum_{f in [f0, f1)} X[f][j] Z[f][j'].
template <int NI>
__global__ __launch_bounds__(256) void k_gram(const GRTask* __restrict__ tasks) {
  constexpr int mj = 16 * NI;
  constexpr int ld = mj + 2;
  constexpr int NT = NI * NI;
  constexpr int MAXT = (NT + 3) / 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lx = reinterpret_cast<double*>(smem_raw);
  double* lz = lx + 64 * ld;
  const GRTask& t = tasks[blockIdx.x];
  const int j = t.j, d0 = t.d0, d1 = t.d1, d2 = t.d2;
  const double* X = (const double*)t.X;
  const double* Z = (const double*)t.Z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  d4 acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; q++) acc[q] = d4{0, 0, 0, 0};
  for (int64_t fb = t.f0; fb < t.f1; fb += 64) {
    __syncthreads();
    if (j == 2) {
      for (int e = threadIdx.x; e < 64 * mj; e += 256) {
        const int fl = e / mj, i = e - fl * mj;
        const int64_t ad = mode_addr(j, d0, d1, d2, i, fb + fl);
        lx[fl * ld + i] = X[ad];
        lz[fl * ld + i] = Z[ad];
      }
    } else {
      for (int e = threadIdx.x; e < 64 * mj; e += 256) {
        const int i = e >> 6, fl = e & 63;
        const int64_t ad = mode_addr(j, d0, d1, d2, i, fb + fl);
        lx[fl * ld + i] = X[ad];
        lz[fl * ld + i] = Z[ad];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXT; q++) {
      const int tt = wave + 4 * q;
      if (tt < NT) {
        const int tj = tt / NI, tk = tt - tj * NI;
        for (int k0 = 0; k0 < 64; k0 += 4) {
          const double a = lx[(k0 + l4) * ld + 16 * tj + l16];
          const double b = lz[(k0 + l4) * ld + 16 * tk + l16];
          acc[q] = mfma16(a, b, acc[q]);
        }
      }
    }
  }
  double* P = (double*)t.partial;
#pragma unroll
  for (int q = 0; q < MAXT; q++) {
    const int tt = wave + 4 * q;
    if (tt < NT) {
      const int tj = tt / NI, tk = tt - tj * NI;
#pragma unroll
      for (int i = 0; i < 4; i++) P[(int64_t)(16 * tk + l16) * mj + 16 * tj + drow<double>(l4, i)] = acc[q][i];
    }
  }
}

// Gram for contracted leg j = 0 or 1 with 16 | d2: the 16 free indices
// [f0, f0 + 16) of one row i are contiguous, so each lane loads 4 consecutive
// values of X and of Z straight into registers (no LDS) and the K order of the
// 16x16x4 products is lane-local: step kk of lane group g takes f0 + 4 g + kk
// for both operands.  Wave w owns the output tiles w, w + 4, ... (row tile tj,
// column tile tk); loads of the next f block are issued before the products.
template <int NI>
__global__ __launch_bounds__(256) void k_gram_nt(const GRTask* __restrict__ tasks) {
  constexpr int mj = 16 * NI;
  constexpr int NT = NI * NI;
  constexpr int MAXT = (NT + 3) / 4;
  const GRTask& t = tasks[blockIdx.x];
  const int j = t.j, d1 = t.d1, d2 = t.d2;
  const double* X = (const double*)t.X;
  const double* Z = (const double*)t.Z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int64_t F = (int64_t)t.d0 * d1 * d2 / mj;
  // element (row i, free f) for f in a 16-aligned block
  auto addr = [&](int i, int64_t f) -> int64_t {
    if (j == 0) return (int64_t)i * F + f;
    const int64_t a = f / d2, c = f - a * d2;
    return a * d1 * d2 + (int64_t)i * d2 + c;
  };
  d4 acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; q++) acc[q] = d4{0, 0, 0, 0};
  int tj[MAXT], tk[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; q++) {
    const int tt = wave + 4 * q;
    tj[q] = tt < NT ? tt / NI : -1;
    tk[q] = tt < NT ? tt - (tt / NI) * NI : 0;
  }
  d4 xr[MAXT], zr[MAXT], xn[MAXT], zn[MAXT];
  auto load = [&](int64_t f0, d4* xv, d4* zv) {
#pragma unroll
    for (int q = 0; q < MAXT; q++) {
      if (tj[q] < 0) continue;
      xv[q] = *(const d4*)(X + addr(16 * tj[q] + l16, f0 + 4 * l4));
      if (q > 0 && tk[q] == tk[q - 1]) zv[q] = zv[q - 1];   // the wave's column tile is loaded once
      else zv[q] = *(const d4*)(Z + addr(16 * tk[q] + l16, f0 + 4 * l4));
    }
  };
  int64_t f0 = t.f0;
  if (f0 < t.f1) load(f0, xr, zr);
  for (; f0 < t.f1; f0 += 16) {
    if (f0 + 16 < t.f1) load(f0 + 16, xn, zn);
#pragma unroll
    for (int q = 0; q < MAXT; q++) {
      if (tj[q] < 0) continue;
#pragma unroll
      for (int kk = 0; kk < 4; kk++) acc[q] = mfma16(xr[q][kk], zr[q][kk], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < MAXT; q++) { xr[q] = xn[q]; zr[q] = zn[q]; }
  }
  double* P = (double*)t.partial;
#pragma unroll
  for (int q = 0; q < MAXT; q++) {
    if (tj[q] < 0) continue;
#pragma unroll
    for (int i = 0; i < 4; i++) P[(int64_t)(16 * tk[q] + l16) * mj + 16 * tj[q] + drow<double>(l4, i)] = acc[q][i];
  }
}

// Register-direct gram for m_j = 64 with the X block of each 16-wide step of
// the free index staged once per workgroup in LDS (double buffered) and
// shared by the four waves, instead of loaded by each wave: wave w owns output
// column tile w (its Z fragment straight from memory, the next step's
// prefetched) and the four row tiles.  Fewer registers than k_gram_nt<4>, so
// more waves per SIMD hide the latency of Z.  Same products, same order.
__global__ __launch_bounds__(256) void k_gram_x4(const GRTask* __restrict__ tasks) {
  constexpr int mj = 64, LDX = 20;   // LDS row stride in doubles (32-byte aligned rows)
  __shared__ __align__(16) double xs[2][mj * LDX];
  const GRTask& t = tasks[blockIdx.x];
  const int j = t.j, d1 = t.d1, d2 = t.d2;
  const double* X = (const double*)t.X;
  const double* Z = (const double*)t.Z;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int si = tid >> 2, sq = tid & 3;   // staging: row si, four f values from 4 sq
  const int64_t F = (int64_t)t.d0 * d1 * d2 / mj;
  auto addr = [&](int i, int64_t f) -> int64_t {
    if (j == 0) return (int64_t)i * F + f;
    const int64_t a = f / d2, c = f - a * d2;
    return a * d1 * d2 + (int64_t)i * d2 + c;
  };
  d4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; q++) acc[q] = d4{0, 0, 0, 0};
  d4 zr = d4{0, 0, 0, 0}, zn = d4{0, 0, 0, 0}, xg = d4{0, 0, 0, 0};
  int64_t f0 = t.f0;
  if (f0 < t.f1) {
    xg = *(const d4*)(X + addr(si, f0 + 4 * sq));
    zr = *(const d4*)(Z + addr(16 * wave + l16, f0 + 4 * l4));
    *(d4*)(&xs[0][si * LDX + 4 * sq]) = xg;
  }
  __syncthreads();
  int buf = 0;
  for (; f0 < t.f1; f0 += 16) {
    const bool more = f0 + 16 < t.f1;
    if (more) {
      xg = *(const d4*)(X + addr(si, f0 + 16 + 4 * sq));
      zn = *(const d4*)(Z + addr(16 * wave + l16, f0 + 16 + 4 * l4));
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const d4 xf = *(const d4*)(&xs[buf][(16 * q + l16) * LDX + 4 * l4]);
#pragma unroll
      for (int kk = 0; kk < 4; kk++) acc[q] = mfma16(xf[kk], zr[kk], acc[q]);
    }
    if (more) {
      *(d4*)(&xs[buf ^ 1][si * LDX + 4 * sq]) = xg;
      zr = zn;
    }
    __syncthreads();
    buf ^= 1;
  }
  double* P = (double*)t.partial;
#pragma unroll
  for (int q = 0; q < 4; q++)
#pragma unroll
    for (int i = 0; i < 4; i++) P[(int64_t)(16 * wave + l16) * mj + 16 * q + drow<double>(l4, i)] = acc[q][i];
}

// Generic gram: one thread per output element (j, j'), loop over the f range.
__global__ __launch_bounds__(256) void k_gram_gen(const GRTask* __restrict__ tasks, int maxm) {
  const GRTask& t = tasks[blockIdx.y];
  const int j = t.j, d0 = t.d0, d1 = t.d1, d2 = t.d2;
  const int mj = j == 0 ? d0 : (j == 1 ? d1 : d2);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= mj * mj) return;
  const int a = e % mj, b = e / mj;   // element (a, b) stored at b * mj + a
  const double* X = (const double*)t.X;
  const double* Z = (const double*)t.Z;
  double acc = 0;
  for (int64_t f = t.f0; f < t.f1; f++)
    acc += X[mode_addr(j, d0, d1, d2, a, f)] * Z[mode_addr(j, d0, d1, d2, b, f)];
  ((double*)t.partial)[e] = acc;
  (void)maxm;
}

__global__ __launch_bounds__(256) void k_gram_reduce(const GRReduce* __restrict__ rs) {
  const GRReduce& r = rs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mm = (int64_t)r.m * r.m;
  if (e >= mm) return;
  const double* P = (const double*)r.partial;
  double acc = 0;
  for (int c = 0; c < r.npart; c++) acc += P[c * mm + e];
  double* out = (double*)r.out;
  acc *= r.coef;
  if (r.accumulate) out[e] += acc;
  else out[e] = acc;
}

// ============================================================================ small elementwise kernels
__global__ __launch_bounds__(256) void k_combine(const CBTask* __restrict__ tasks,
                                                 const CBTerm* __restrict__ terms) {
  const CBTask& t = tasks[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= t.n) return;
  double acc = 0;
  for (int k = t.term0; k < t.term0 + t.nterm; k++)
    acc += terms[k].coef * ((const double*)terms[k].in)[e];
  ((double*)t.out)[e] = acc;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_reduce_out(const RDSrc* __restrict__ srcs, int nsrc,
                                                    TO* __restrict__ y, int ml, int mr, int mp) {
  const int64_t M = (int64_t)ml * mr * mp;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M) return;
  const int64_t l = e / ((int64_t)mr * mp);
  const int64_t rem = e - l * mr * mp;
  const int64_t r = rem / mp, p = rem - r * mp;
  const int64_t et = p * ml * mr + l * mr + r;
  double acc = 0;
#pragma unroll 8
  for (int k = 0; k < nsrc; k++) {
    const TI* src = (const TI*)srcs[k].p;
    acc += (double)(srcs[k].layout ? src[et] : src[e]);
  }
  y[e] = (TO)acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_transpose_plr(const T* __restrict__ x, T* __restrict__ xt,
                                                       int ml, int mr, int mp) {
  const int64_t M = (int64_t)ml * mr * mp;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M) return;
  const int64_t l = e / ((int64_t)mr * mp);
  const int64_t rem = e - l * mr * mp;
  const int64_t r = rem / mp, p = rem - r * mp;
  xt[p * ml * mr + l * mr + r] = x[e];
}

__global__ __launch_bounds__(256) void k_convert(const CVTask* __restrict__ tasks) {
  const CVTask& t = tasks[blockIdx.y];
  if (t.fmt == 1) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < t.n; e += (int64_t)gridDim.x * 256)
      ((float*)t.dst)[e] = (float)t.src[e];
    return;
  }
  // split BF16: thread per destination position (block, row i, permuted position)
  const int m = t.m;
  const int64_t mm = (int64_t)m * m;
  __bf16* dst = (__bf16*)t.dst;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < t.n; e += (int64_t)gridDim.x * 256) {
    const int64_t b = e / mm, r = e - b * mm;
    const int i = (int)(r / m), pos = (int)(r - (int64_t)i * m);
    const double x = t.src[b * mm + (int64_t)bf_perm(pos) * m + i];
    const __bf16 hi = (__bf16)(float)x;
    const __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
    dst[2 * b * mm + r] = hi;
    dst[2 * b * mm + mm + r] = lo;
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_cast(const TS* __restrict__ s, TD* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    d[e] = (TD)s[e];
}

// ============================================================================ Krylov (FP64)
__device__ __forceinline__ double block_sum(double v, double* red) {
  // deterministic: wave shuffle tree, then fixed-order sum of the 4 waves
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Every Krylov kernel takes a list of jobs (one per node being solved, possibly
// of different problem instances) and works on job blockIdx.y, so one launch
// advances all jobs of a batch by the same step.  Partial sums of a job live
// in its four areas P0..P3 of 64 x kRedBlocks values.
__device__ __forceinline__ double* parea(const KJob& J, int i) { return J.red + (int64_t)i * 64 * kRedBlocks; }

// The fused steps first reduce the partial sums of the previous kernel in
// every workgroup (fixed order, identical everywhere), so no separate
// reduction launch sits between them.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, double* red) {
  return block_sum(p[threadIdx.x], red);   // kRedBlocks == blockDim.x == 256
}

__device__ __forceinline__ void write_copies(const KJob& J, int64_t e, double v) {
  if (J.x64) J.x64[e] = v;
  if (J.x32) J.x32[e] = (float)v;
}

__global__ __launch_bounds__(256) void k_kinit(const KJob* __restrict__ jobs, int kmax) {
  KrylovState* st = jobs[blockIdx.y].st;
  const int t = threadIdx.x;
  if (t < 128) { st->alpha[t] = 0; st->beta[t] = 0; st->h[t] = 0; st->y[t] = 0; }
  if (t < 8) st->scal[t] = 0;
  if (t == 0) { st->kmax = kmax; st->keff = 1; st->stop = 0; st->status = 0; }
}

// P0 = partial sums of ||T||^2
__global__ __launch_bounds__(256) void k_knorm(const KJob* __restrict__ jobs) {
  __shared__ double red[4];
  const KJob& J = jobs[blockIdx.y];
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
    acc += J.T[e] * J.T[e];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) parea(J, 0)[blockIdx.x] = s;
}

// mode 0: V_0 = T / ||T|| (and the copies); mode 1: T <- T / ||T||.  ||T||^2 from P0.
__global__ __launch_bounds__(256) void k_kscale(const KJob* __restrict__ jobs, int mode) {
  __shared__ double red[4];
  const KJob& J = jobs[blockIdx.y];
  const double nr = sqrt(sum_partials(parea(J, 0), red));
  if (blockIdx.x == 0 && threadIdx.x == 0 && !(nr > 0 && isfinite(nr))) fail_status(J.st, 1);
  const double inv = 1.0 / nr;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256) {
    const double v = J.T[e] * inv;
    if (mode == 0) { J.V[e] = v; write_copies(J, e, v); }
    else J.T[e] = v;
  }
}


// alpha_j = sum P0 (last step, no update follows)
__global__ __launch_bounds__(256) void k_kalpha(const KJob* __restrict__ jobs, int j) {
  __shared__ double red[4];
  const KJob& J = jobs[blockIdx.y];
  if (J.st->stop) return;
  const double a = sum_partials(parea(J, 0), red);
  if (threadIdx.x == 0) {
    J.st->alpha[j] = a;
    if (!isfinite(a)) fail_status(J.st, 1);
  }
}

// Wave sums of eight per-lane values at once by recursive halving: at each of
// the first three levels a lane keeps half of its values and adds its
// partner's copy of them (partner lane ^ 32, ^ 16, ^ 8), so that lane l ends
// with value l >> 3 summed over eight lanes; three more exchanges (^ 4, ^ 2,
// ^ 1) complete the sum over the wavefront.  Ten exchanges instead of 48 for
// eight separate trees; the eight lanes holding a value agree bit for bit.
__device__ __forceinline__ double wave_sums8(const double (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double a[4];
#pragma unroll
  for (int u = 0; u < 4; u++) a[u] = (h5 ? v[u + 4] : v[u]) + __shfl_xor(h5 ? v[u] : v[u + 4], 32, 64);
  double b2[2];
#pragma unroll
  for (int u = 0; u < 2; u++) b2[u] = (h4 ? a[u + 2] : a[u]) + __shfl_xor(h4 ? a[u] : a[u + 2], 16, 64);
  double c = (h3 ? b2[1] : b2[0]) + __shfl_xor(h3 ? b2[0] : b2[1], 8, 64);
  c += __shfl_xor(c, 4, 64);
  c += __shfl_xor(c, 2, 64);
  c += __shfl_xor(c, 1, 64);
  return c;
}

// Block sums of 8 per-thread values at once (wave sums above, then the waves
// in order); the sum of value q is returned in thread q.  red holds 8 doubles
// per wavefront of the block.
template <int NW>
__device__ __forceinline__ double block_sums8(const double (&v)[8], double* red) {
  const double c = wave_sums8(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if ((lane & 7) == 0) red[wave * 8 + (lane >> 3)] = c;
  __syncthreads();
  const int q = threadIdx.x & 7;
  double s = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) s += red[w * 8 + q];
  return s;
}

constexpr int kDotChunk = 8;

// out[i * kRedBlocks + b] = this block's partial dot V_i . w for i < nv, eight
// vectors per pass over the block's elements.
__device__ __forceinline__ void block_dots(const KJob& J, const double* __restrict__ w, int nv, double* out,
                                           double* red) {
  const int64_t n = J.n;
  const int b = blockIdx.x;
  for (int i0 = 0; i0 < nv; i0 += kDotChunk) {
    double acc[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; q++) acc[q] = 0.0;
    for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < n; e += (int64_t)kRedBlocks * 256) {
      const double we = w[e];
#pragma unroll
      for (int q = 0; q < kDotChunk; q++)
        if (i0 + q < nv) acc[q] += J.V[(int64_t)(i0 + q) * n + e] * we;
    }
    const double s = block_sums8<4>(acc, red);
    if (threadIdx.x < kDotChunk && i0 + (int)threadIdx.x < nv) out[(i0 + threadIdx.x) * kRedBlocks + b] = s;
  }
}

// hs[i] = sum of the kRedBlocks partials p[i * kRedBlocks + .] for i < nv
// (sum_partials of each, eight at a time)
__device__ __forceinline__ void sums_of_partials(const double* __restrict__ p, int nv, double* hs, double* red) {
  for (int i0 = 0; i0 < nv; i0 += kDotChunk) {
    double v[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; q++) v[q] = i0 + q < nv ? p[(i0 + q) * kRedBlocks + threadIdx.x] : 0.0;
    const double s = block_sums8<4>(v, red);
    if (threadIdx.x < kDotChunk && i0 + (int)threadIdx.x < nv) hs[i0 + threadIdx.x] = s;
  }
  __syncthreads();
}

// Dot products of basis vectors with the product w = H v_j, right after the
// product.  Blocks of kDotThreads = 1024 threads, kRedBlocks of them: element
// e belongs to thread e % 1024 of block (e / 1024) % kRedBlocks, whose
// partial sum is written to out[(i - i0) * kRedBlocks + block] (the layout
// every later step reads).  A step j < k - 1 takes the dots of V[0..j] into
// P1 (the two classical Gram-Schmidt passes that follow run against the whole
// basis, so the first also removes alpha_j v_j and beta_{j-1} v_{j-1}, and
// alpha_j is the sum of dot j); the last step takes v_j . w into P0.
constexpr int kDotThreads = 1024;

__device__ __forceinline__ void block_dots_1k(const KJob& J, const double* __restrict__ w, int i0, int nv,
                                              double* out, double* red) {
  const int64_t n = J.n;
  const int b = blockIdx.x;
  for (int c0 = 0; c0 < nv; c0 += kDotChunk) {
    double acc[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; q++) acc[q] = 0.0;
    for (int64_t e = (int64_t)b * kDotThreads + threadIdx.x; e < n; e += (int64_t)kRedBlocks * kDotThreads) {
      const double we = w[e];
#pragma unroll
      for (int q = 0; q < kDotChunk; q++)
        if (c0 + q < nv) acc[q] += J.V[(int64_t)(i0 + c0 + q) * n + e] * we;
    }
    const double s = block_sums8<kDotThreads / 64>(acc, red);
    if (threadIdx.x < kDotChunk && c0 + (int)threadIdx.x < nv) out[(c0 + threadIdx.x) * kRedBlocks + b] = s;
  }
}

// partial dots of V[i0, i0 + nv) with w into area pin (w as the product left it)
__global__ __launch_bounds__(1024) void k_kdots(const KJob* __restrict__ jobs, int i0, int nv, int pin) {
  const KJob& J = jobs[blockIdx.y];
  if (J.st->stop) return;
  __shared__ double red[16 * kDotChunk];
  block_dots_1k(J, J.w, i0, nv, parea(J, pin), red);
}

// w = the sum of the product's partial outputs (per element in the order of
// k_reduce_out), then the partial dots of k_kdots: one launch instead of two
// (single job; the same bits as k_reduce_out followed by k_kdots)
__global__ __launch_bounds__(1024) void k_reduce_dots(const RDSrc* __restrict__ srcs, int nsrc,
                                                      const KJob* __restrict__ jobs, int ml, int mr, int mp,
                                                      int i0, int nv, int pin) {
  const KJob& J = jobs[0];
  const int64_t M = (int64_t)ml * mr * mp;
  double* w = J.w;
  for (int64_t e = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; e < M; e += (int64_t)kRedBlocks * kDotThreads) {
    const int64_t l = e / ((int64_t)mr * mp);
    const int64_t rem = e - l * mr * mp;
    const int64_t r = rem / mp, p = rem - r * mp;
    const int64_t et = p * ml * mr + l * mr + r;
    double acc = 0;
#pragma unroll 8
    for (int k = 0; k < nsrc; k++) {
      const double* src = (const double*)srcs[k].p;
      acc += srcs[k].layout ? src[et] : src[e];
    }
    w[e] = acc;
  }
  if (J.st->stop) return;
  __shared__ double red[16 * kDotChunk];
  block_dots_1k(J, w, i0, nv, parea(J, pin), red);
}

// classical Gram-Schmidt pass against V[0..j]: h = sums of P(pin); w -= sum h_i V_i;
// then P(pin + 1) = partial dots V[0..j] . w, or ||w||^2 when norm_only.
// set_alpha (first pass): alpha_j = h_j.
__global__ __launch_bounds__(256) void k_kortho(const KJob* __restrict__ jobs, int j, int pin,
                                                int norm_only, int set_alpha) {
  __shared__ double red[4];
  __shared__ double hs[128];
  const KJob& J = jobs[blockIdx.y];
  if (J.st->stop) return;
  const int nv = j + 1;
  const int64_t n = J.n;
  double* w = J.w;
  __shared__ double red8[4 * kDotChunk];
  sums_of_partials(parea(J, pin), nv, hs, red8);
  if (set_alpha && blockIdx.x == 0 && threadIdx.x == 0) {
    J.st->alpha[j] = hs[j];
    if (!isfinite(hs[j])) fail_status(J.st, 1);
  }
  const int b = blockIdx.x;
  double* po = parea(J, pin + 1);
  if ((n & 1) == 0) {
    // even n: element pairs (2 e, 2 e + 1) per thread, 16-byte loads
    const int64_t np = n / 2;
    dv2* w2 = reinterpret_cast<dv2*>(w);
    for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < np; e += (int64_t)kRedBlocks * 256) {
      dv2 x = w2[e];
      for (int i = 0; i < nv; i++) x -= hs[i] * reinterpret_cast<const dv2*>(J.V + (int64_t)i * n)[e];
      w2[e] = x;
    }
    if (norm_only) {
      double acc = 0;
      for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < np; e += (int64_t)kRedBlocks * 256) {
        const dv2 x = w2[e];
        acc += x.x * x.x;
        acc += x.y * x.y;
      }
      const double s = block_sum(acc, red);
      if (threadIdx.x == 0) po[b] = s;
      return;
    }
    for (int i0 = 0; i0 < nv; i0 += kDotChunk) {
      double acc[kDotChunk];
#pragma unroll
      for (int q = 0; q < kDotChunk; q++) acc[q] = 0.0;
      for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < np; e += (int64_t)kRedBlocks * 256) {
        const dv2 we = w2[e];
#pragma unroll
        for (int q = 0; q < kDotChunk; q++)
          if (i0 + q < nv) {
            const dv2 v = reinterpret_cast<const dv2*>(J.V + (int64_t)(i0 + q) * n)[e];
            acc[q] += v.x * we.x;
            acc[q] += v.y * we.y;
          }
      }
      const double s = block_sums8<4>(acc, red8);
      if (threadIdx.x < kDotChunk && i0 + (int)threadIdx.x < nv) po[(i0 + threadIdx.x) * kRedBlocks + b] = s;
    }
    return;
  }
  for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < n; e += (int64_t)kRedBlocks * 256) {
    double x = w[e];
    for (int i = 0; i < nv; i++) x -= hs[i] * J.V[(int64_t)i * n + e];
    w[e] = x;
  }
  if (norm_only) {
    double acc = 0;
    for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < n; e += (int64_t)kRedBlocks * 256)
      acc += w[e] * w[e];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) po[b] = s;
    return;
  }
  block_dots(J, w, nv, po, red8);
}

// beta_j = sqrt(sum P3); breakdown test; V_{j+1} = w / beta_j (and the copies)
__global__ __launch_bounds__(256) void k_kbeta(const KJob* __restrict__ jobs, int j) {
  __shared__ double red[4];
  const KJob& J = jobs[blockIdx.y];
  KrylovState* st = J.st;
  if (st->stop) return;
  const double b = sqrt(sum_partials(parea(J, 3), red));
  double amax = 0;
  for (int k = 0; k <= j; k++) amax = fmax(amax, fabs(st->alpha[k]));
  const bool brk = !(b > 1e-14 * amax);
  __syncthreads();   // every block has read the state before block 0 updates it
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!isfinite(b)) fail_status(st, 1);
    if (brk) st->stop = 1;
    else { st->beta[j] = b; st->keff = j + 2; }
  }
  if (brk) return;
  const double inv = 1.0 / b;
  double* out = J.V + (int64_t)(j + 1) * J.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256) {
    const double v = J.w[e] * inv;
    out[e] = v;
    write_copies(J, e, v);
  }
}

// ---- wavefront-wide reductions.  Every step combines a lane with a partner
// holding the same partial (the operations are commutative), and the result
// is read from lane 0, so every lane gets the same bits.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_d<0xB1>(v));    // quad_perm(1, 0, 3, 2)
  v = op(v, dpp_d<0x4E>(v));    // quad_perm(2, 3, 0, 1)
  v = op(v, dpp_d<0x141>(v));   // row_half_mirror
  v = op(v, dpp_d<0x140>(v));   // row_mirror
  v = op(v, __shfl_xor(v, 16, 64));
  v = op(v, __shfl_xor(v, 32, 64));
  return readlane_d(v, 0);
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double x, double y) { return x + y; });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double x, double y) { return fmax(x, y); });
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double x, double y) { return fmin(x, y); });
}

// Lowest eigenpair of the keff x keff symmetric tridiagonal matrix
// T = tridiag(beta, alpha, beta) of a Lanczos run, by one full wavefront:
//  * eigenvalue by multisection on Sturm counts (64 points per round, one per
//    lane) inside the Gershgorin interval, then bisection down to adjacent
//    floating-point numbers;
//  * eigenvector by three rounds of inverse iteration with one LU
//    factorisation (partial pivoting) of T - theta I;
//  * normalised, sign fixed as described at the end.
// lds must hold kTriLds doubles.
constexpr int kTriLds = 768;
constexpr size_t kTinyLdsMax = 144 * 1024;   // dynamic LDS of the tiny-node Lanczos kernels

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal as[] and squared off-diagonal bs2[] (bs2[i] couples rows i - 1 and
// i; bs2[0] = 0): the number of sign changes along the leading principal
// minors p_i = (as_i - x) p_{i-1} - bs2_i p_{i-2} (a Sturm sequence, starting
// from p_{-1} = 1, p_{-2} = 0), read off the sign bits.  A zero minor inside
// the sequence is followed by one of the sign opposite to its predecessor, so
// its own sign bit does not change the count; a zero last minor (x an
// eigenvalue of the computed sequence) counts by its sign bit, which puts x on
// one side of that eigenvalue.  No division and no branch: a step is one
// dependent FMA and three integer operations.  The caller scales the matrix
// and x by a power of two (exact) so that |as_i - x| <= 2 and bs2_i <= 1: the
// minors grow by less than 2^2 per step, and after every 8 steps the pair
// (p_{i-1}, p_i) is brought back into [2^-200, 2^200] by a power of two, which
// changes no sign.  The arrays hold kp (a multiple of 8) entries; entries past
// the matrix have as = 2^60 and bs2 = 0, steps that multiply the last minor by
// a positive factor and count nothing.
__device__ __forceinline__ int sturm_count(const double* __restrict__ as, const double* __restrict__ bs2, int kp,
                                           double x) {
  double pm = 0.0, pc = 1.0;
  unsigned cnt = 0;
  for (int c = 0; c < kp; c += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) { av[u] = as[c + u]; bv[u] = bs2[c + u]; }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const double pn = (av[u] - x) * pc - bv[u] * pm;
      cnt += ((unsigned)__double2hiint(pn) ^ (unsigned)__double2hiint(pc)) >> 31;
      pm = pc;
      pc = pn;
    }
    const double m = fmax(fabs(pm), fabs(pc));
    const double sc = m > 0x1p200 ? 0x1p-200 : (m < 0x1p-200 ? 0x1p200 : 1.0);
    pm *= sc;
    pc *= sc;
  }
  return (int)cnt;
}

__device__ __forceinline__ void tridiag_solve_wave(KrylovState* __restrict__ st, double* __restrict__ lds) {
  const int lane = threadIdx.x & 63;
  const int k = __builtin_amdgcn_readfirstlane(st->keff);   // 1 <= k <= 64
  const int kp = (k + 7) & ~7;
  double* a = lds;           // alpha [64]
  double* b = lds + 64;      // beta, zero from index k - 1 on [72]
  double* as = lds + 136;    // alpha scaled for the Sturm counts, padded [72]
  double* bs2 = lds + 208;   // (scaled beta_{i-1})^2, padded [72]
  double* d = lds + 280;     // U = P L^-1 (T - theta I): diagonal [64]
  double* du = lds + 344;    //   first superdiagonal [64]
  double* du2 = lds + 408;   //   second superdiagonal [64]
  double* f = lds + 472;     // multipliers of L [64]
  double* sw = lds + 536;    // 1 where rows i and i + 1 were swapped [64]
  double* rd = lds + 600;    // 1 / d [64]
  double* y = lds + 664;     // eigenvector [72]
  const bool on = lane < k;
  const double al = on ? st->alpha[lane] : 0.0;
  const double bl = lane + 1 < k ? st->beta[lane] : 0.0;
  a[lane] = al;
  b[lane] = bl;
  y[lane] = 1.0;
  if (lane < 8) { b[64 + lane] = 0.0; y[64 + lane] = 0.0; }
  wave_sync();
  // Gershgorin interval and a bound of ||T||, one row per lane
  const double bp = lane > 0 ? b[lane - 1] : 0.0;
  const double r = fabs(bp) + fabs(bl);
  double lo = wave_min(on ? al - r : __builtin_huge_val());
  double hi = wave_max(on ? al + r : -__builtin_huge_val());
  const double nrm = wave_max(on ? fabs(al) + r : 0.0);
  // power-of-two scale sg with nrm * sg <= 1 for the Sturm counts (exact)
  int ex = 0;
  (void)frexp(nrm, &ex);
  const double sg = (nrm > 0.0 && isfinite(nrm)) ? ldexp(1.0, -ex) : 1.0;
  as[lane] = on ? al * sg : 0x1p60;
  const double bsc = bp * sg;
  bs2[lane] = on ? bsc * bsc : 0.0;
  if (lane < 8) { as[64 + lane] = 0x1p60; bs2[64 + lane] = 0.0; }
  wave_sync();
  // multisection: lane l probes lo + (hi - lo) (l + 1) / 65; the bracket
  // [lo, hi] keeps the lowest eigenvalue
  const double frac = (double)(lane + 1) / 65.0;
  for (int it = 0; it < 40; it++) {
    const double w = hi - lo;
    const double x = lo + w * frac;
    const bool has = (x > lo && x < hi) ? sturm_count(as, bs2, kp, x * sg) >= 1 : (x >= hi);
    const unsigned long long m = __ballot(has);
    const int first = m ? __ffsll((long long)m) - 1 : 64;
    const double xf = readlane_d(x, first & 63), xb = readlane_d(x, (first - 1) & 63);
    const double nhi = first < 64 ? xf : hi;
    const double nlo = first > 0 ? xb : lo;
    if (!(nhi < hi || nlo > lo)) break;
    hi = fmin(hi, nhi);
    lo = fmax(lo, nlo);
    if (hi - lo <= 2.2e-16 * fmax(fabs(lo), fabs(hi))) break;
  }
  // bisection to the last bits
  for (int it = 0; it < 64; it++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(as, bs2, kp, mid * sg) >= 1) hi = mid;
    else lo = mid;
  }
  const double theta = hi;
  const double tiny = 1e-300 + 2.2e-16 * nrm * 1e-3;
  if (lane == 0) {
    // T - theta I = P L U, row by row; cd and cu carry the diagonal and
    // superdiagonal entries of the current row as updated so far.  Both
    // pivoting choices are evaluated and the taken one selected (no branch);
    // entries past row k - 2 are written but never read.
    double cd = a[0] - theta, cu = b[0];
    for (int c = 0; c + 1 < k; c += 8) {
      double av[8], bv[9];
#pragma unroll
      for (int u = 0; u < 8; u++) av[u] = a[c + 1 + u];
#pragma unroll
      for (int u = 0; u < 9; u++) bv[u] = b[c + u];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int i = c + u;
        const double li = bv[u], an = av[u] - theta, bn = bv[u + 1];
        const bool swp = !(fabs(cd) >= fabs(li));   // rows i and i + 1 swapped
        const double piv = (!swp && cd == 0.0) ? tiny : cd;
        const double fi = (swp ? piv : li) / (swp ? li : piv);
        f[i] = fi;
        sw[i] = swp ? 1.0 : 0.0;
        d[i] = swp ? li : piv;
        du[i] = swp ? an : cu;
        du2[i] = swp ? bn : 0.0;
        const double ncd = swp ? cu - fi * an : an - fi * cu;
        const double ncu = swp ? -fi * bn : bn;
        const bool live = i + 1 < k;
        cd = live ? ncd : cd;
        cu = live ? ncu : cu;
      }
    }
    if (cd == 0.0) cd = tiny;
    d[k - 1] = cd;
    du[k - 1] = 0.0;
    du2[k - 1] = 0.0;
  }
  wave_sync();
  if (on) rd[lane] = 1.0 / d[lane];
  wave_sync();
  double sc = 1.0;   // y is held unnormalised; sc is its pending scale
  if (lane == 0) {
    for (int rep = 0; rep < 3; rep++) {
      // forward: y <- L^{-1} P (sc y), in place (writes past row k - 1 are
      // overwritten or never read)
      double cur = y[0] * sc;
      for (int c = 0; c + 1 < k; c += 8) {
        double yv[8], fv[8], sv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) { yv[u] = y[c + 1 + u]; fv[u] = f[c + u]; sv[u] = sw[c + u]; }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          // no swap: y_i = cur, cur' = nx - f cur; swap: y_i = nx, cur' = cur - f nx
          const double nx = yv[u] * sc;
          const bool swp = sv[u] != 0.0;
          const double first = swp ? nx : cur, second = swp ? cur : nx;
          y[c + u] = first;
          const double ncur = second - fv[u] * first;
          cur = c + u + 1 < k ? ncur : cur;
        }
      }
      y[k - 1] = cur;
      // backward: y <- U^{-1} y, from the last row up
      double y1 = 0.0, y2 = 0.0, n2 = 0.0;
      for (int c = kp - 8; c >= 0; c -= 8) {
        double yv[8], uv[8], u2v[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) { yv[u] = y[c + u]; uv[u] = du[c + u]; u2v[u] = du2[c + u]; rv[u] = rd[c + u]; }
#pragma unroll
        for (int u = 7; u >= 0; u--) {
          const double v = (yv[u] - uv[u] * y1 - u2v[u] * y2) * rv[u];
          if (c + u < k) {
            y[c + u] = v;
            n2 += v * v;
            y2 = y1;
            y1 = v;
          }
        }
      }
      sc = 1.0 / sqrt(n2);
    }
  }
  wave_sync();
  sc = readlane_d(sc, 0);
  // sign (a gauge): the first component with magnitude >= 1e-8 of the largest
  // one is made positive
  const double yl = on ? y[lane] * sc : 0.0;
  const double ymax = wave_max(fabs(yl));
  const unsigned long long big = __ballot(on && fabs(yl) >= 1e-8 * ymax);
  const int first = big ? min(__ffsll((long long)big) - 1, k - 1) : k - 1;
  const double sgn = readlane_d(yl, first) < 0 ? -1.0 : 1.0;
  if (on) st->y[lane] = sgn * yl;
  if (lane == 0) {
    st->scal[0] = theta;
    if (!isfinite(theta)) fail_status(st, 1);
  }
}

__global__ __launch_bounds__(64) void k_ktridiag(const KJob* __restrict__ jobs) {
  __shared__ double lds[kTriLds];
  tridiag_solve_wave(jobs[blockIdx.y].st, lds);
}

// ---- tiny nodes (M <= 1024): H_eff is assembled densely once per eigensolve
// (the same operator as the factorised matvec: every item's Kronecker product
// written out entry by entry), then the Lanczos steps run in one workgroup
// with a dense matvec.
// O[ip][i] (column ip of the m x m block), or the identity when O is null.  The
// load is unconditional (from a valid dummy when O is null), so that the
// loads of consecutive items can be in flight together.
__device__ const double g_one = 1.0;
__device__ __forceinline__ double blk(const double* O, int m, int i, int ip) {
  const double x = *(O ? O + (int64_t)ip * m + i : &g_one);
  return O ? x : (i == ip ? 1.0 : 0.0);
}

// Items per entry are split over S threads (part q takes items q, q + S, ...)
// whose sums are added in part order; S depends only on the node size, so a
// job assembles the same bits alone or in a batch.
__host__ __device__ __forceinline__ int tiny_assemble_parts(int M) { return (int64_t)M * M >= 65536 ? 4 : 8; }

// H^T[j][i] = H[i][j] (H is symmetric); a block of 256 threads takes 256 / S
// entries with S parts each; job blockIdx.y
__global__ __launch_bounds__(256) void k_tiny_assemble(const TJob* __restrict__ jobs) {
  __shared__ double part[256];
  const TJob& J = jobs[blockIdx.y];
  const TinyPlan P = *J.plan;
  double* __restrict__ H = J.H;
  const int d0 = P.d0, d1 = P.d1, d2 = P.d2;
  const int M = d0 * d1 * d2;
  const int S = tiny_assemble_parts(M), per = 256 / S;
  const int q = threadIdx.x / per, le = threadIdx.x - q * per;
  const int64_t e = (int64_t)blockIdx.x * per + le;
  const bool on = e < (int64_t)M * M;
  double acc = 0;
  if (on) {
    const int col = (int)(e / M), row = (int)(e - (int64_t)col * M);
    const int l1 = row / (d1 * d2), r1 = (row / d2) % d1, p1 = row % d2;
    const int l2 = col / (d1 * d2), r2 = (col / d2) % d1, p2 = col % d2;
    if (l1 == l2)
#pragma unroll 2
      for (int it = P.item0[0] + q; it < P.item0[0] + P.nitem[0]; it += S)
        acc += P.items[it].coef * blk((const double*)P.items[it].A, d1, r1, r2) *
               blk((const double*)P.items[it].B, d2, p1, p2);
    if (r1 == r2)
#pragma unroll 2
      for (int it = P.item0[1] + q; it < P.item0[1] + P.nitem[1]; it += S)
        acc += P.items[it].coef * blk((const double*)P.items[it].A, d0, l1, l2) *
               blk((const double*)P.items[it].B, d2, p1, p2);
    if (p1 == p2)
#pragma unroll 2
      for (int it = P.item0[2] + q; it < P.item0[2] + P.nitem[2]; it += S)
        acc += P.items[it].coef * blk((const double*)P.items[it].A, d0, l1, l2) *
               blk((const double*)P.items[it].B, d1, r1, r2);
#pragma unroll 2
    for (int it = q; it < P.n3; it += S) {
      const Item3& t3 = P.items3[it];
      acc += t3.coef * blk((const double*)t3.op[0], d0, l1, l2) * blk((const double*)t3.op[1], d1, r1, r2) *
             blk((const double*)t3.op[2], d2, p1, p2);
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (q == 0 && on) {
    double h = 0;
    for (int r = 0; r < S; r++) h += part[r * per + le];
    H[e] = h;
  }
}

// Tiny-node Lanczos, the same steps in both kernels below:
//   u = H V_j;  alpha_j = V_j . u;
//   w = u - sum_{i<=j} (V_i . u) V_i;  w -= sum_{i<=j} (V_i . w) V_i
//   (classical Gram-Schmidt twice, against the whole basis; in exact
//   arithmetic the first pass removes alpha_j V_j and beta_{j-1} V_{j-1});
//   beta_j = ||w||;  V_{j+1} = w / beta_j;
// then the tridiagonal eigenpair and the Ritz vector.  Which kernel runs a
// job, and every summation order, depend only on the job's M, so a job gives
// the same bits alone or in a batch.
constexpr int kTinyWaveM = 64;   // largest M of the one-wavefront kernel
constexpr int64_t kTinyWaveLds = (64 * 64 + 64 * 65) * (int64_t)sizeof(double);

// M <= 64: one wavefront per job, no barriers.  H and the basis in LDS (basis
// rows padded to an odd stride); lane t owns vector entry t; lane i takes
// the dot product with basis vector i.
__global__ __launch_bounds__(64) void k_tiny_lanczos_wave(const TJob* __restrict__ jobs, int kreq) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double ub[64], wb[64], hs[64], hs2[64];
  __shared__ double tri_lds[kTriLds];
  const TJob& J = jobs[blockIdx.x];
  const int M = J.M;
  if (M > kTinyWaveM) return;   // run by k_tiny_lanczos_block
  const double* __restrict__ H = J.H;
  double* __restrict__ T = J.T;
  KrylovState* __restrict__ st = J.st;
  const int k = kreq < M ? kreq : M;
  const int t = threadIdx.x;
  const int ldv = M | 1;
  double* Hs = reinterpret_cast<double*>(smem_raw);   // [M][M], column c at c * M
  double* V = Hs + 64 * 64;                            // [k][ldv]
  for (int e = t; e < M * M; e += 64) Hs[e] = H[e];
  const bool mine = t < M;
  if (t == 0) { st->kmax = k; st->keff = 1; st->stop = 0; st->status = 0; }
  const double t0 = mine ? T[t] : 0.0;
  const double nrm = sqrt(wave_sum(t0 * t0));
  if (mine) V[t] = t0 / nrm;
  wave_sync();
  double amax = 0;
  int keff = 1;
  for (int j = 0; j < k; j++) {
    const double* x = V + j * ldv;
    double u = 0;
    if (mine) {
#pragma unroll 8
      for (int c = 0; c < M; c++) u += Hs[c * M + t] * x[c];
      ub[t] = u;
    }
    wave_sync();
    if (t <= j) {
      const double* vi = V + t * ldv;
      double d = 0;
#pragma unroll 8
      for (int e = 0; e < M; e++) d += vi[e] * ub[e];
      hs[t] = d;
    }
    wave_sync();
    const double a = hs[j];
    if (t == 0) st->alpha[j] = a;
    amax = fmax(amax, fabs(a));
    if (j == k - 1) break;
    double w = u;
    if (mine) {
      for (int i = 0; i <= j; i++) w -= hs[i] * V[i * ldv + t];
      wb[t] = w;
    }
    wave_sync();
    if (t <= j) {
      const double* vi = V + t * ldv;
      double d = 0;
#pragma unroll 8
      for (int e = 0; e < M; e++) d += vi[e] * wb[e];
      hs2[t] = d;
    }
    wave_sync();
    if (mine) {
      for (int i = 0; i <= j; i++) w -= hs2[i] * V[i * ldv + t];
      wb[t] = w;
    }
    wave_sync();
    double n2 = 0;
#pragma unroll 8
    for (int e = 0; e < M; e++) n2 += wb[e] * wb[e];
    const double b = sqrt(n2);
    if (!(b > 1e-14 * amax)) break;
    if (t == 0) st->beta[j] = b;
    keff = j + 2;
    if (mine) V[(j + 1) * ldv + t] = w / b;
    wave_sync();
  }
  if (t == 0) st->keff = keff;
  wave_sync();
  tridiag_solve_wave(st, tri_lds);
  wave_sync();
  if (t < keff) hs[t] = st->y[t];
  wave_sync();
  double u = 0;
  if (mine)
    for (int i = 0; i < keff; i++) u += hs[i] * V[i * ldv + t];
  const double nr = sqrt(wave_sum(u * u));
  if (mine) T[t] = u / nr;
  if (t == 0 && !(nr > 0 && isfinite(nr))) fail_status(st, 1);
}

// Sum over the first nwm wavefronts of v (one value per thread, zeros past the
// vector), in wave order; a barrier must separate two calls.
__device__ __forceinline__ double block_sum_nw(double v, double* red, int nwm) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < nwm; i++) s += red[i];
  return s;
}

// 64 < M <= 1024: one workgroup of 1024 threads per job; thread t owns vector
// entry t.  The dense matvec splits the columns over S slices, 16 loads of H
// in flight per thread: for even M a thread takes two adjacent rows with
// 16-byte loads (S = min(M, 2048 / M)), for odd M one row (S = min(M,
// 1024 / M)); the slices' partial sums are added in a fixed order.  Each Gram-Schmidt dot
// product is taken by one wavefront.  The product of step j + 1 runs on the
// unnormalised w of step j and is scaled by 1 / beta_j afterwards, so the new
// basis vector needs no barrier of its own.
// Dynamic LDS: partial sums [2048], H x [1024], then (VL) the basis [k][M] and
// w [M]; without VL the basis and w stay in the job's global buffers.
__host__ __device__ __forceinline__ int64_t tiny_basis_bytes(int M, int kreq) {
  const int64_t k = kreq < M ? kreq : M;
  return (k + 1) * M * (int64_t)sizeof(double);
}
constexpr int64_t kTinyBlockFixed = 3072 * (int64_t)sizeof(double);

template <bool VL>
__global__ __launch_bounds__(1024) void k_tiny_lanczos_block(const TJob* __restrict__ jobs, int kreq) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  __shared__ double hs[64], hs2[64];
  __shared__ double tri_lds[kTriLds];
  const TJob& J = jobs[blockIdx.x];
  const int M = J.M;
  if (M <= kTinyWaveM) return;   // run by k_tiny_lanczos_wave
  if ((tiny_basis_bytes(M, kreq) <= (int64_t)kTinyLdsMax - kTinyBlockFixed) != VL) return;   // other form
  const __attribute__((address_space(1))) double* __restrict__ H =
      (const __attribute__((address_space(1))) double*)J.H;
  double* __restrict__ T = J.T;
  KrylovState* __restrict__ st = J.st;
  const int k = kreq < M ? kreq : M;
  double* part = reinterpret_cast<double*>(smem_raw);   // [S][M] <= 2048
  double* ub = part + 2048;
  double* V = VL ? ub + 1024 : J.V;
  double* w = VL ? V + (int64_t)k * M : J.w;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  // column slices of the product: M even, S x (M / 2) threads on row pairs;
  // M odd, S x M threads on single rows
  const bool even = (M & 1) == 0;
  const int P2 = M / 2;
  const int S = even ? max(1, min(M, 1024 / P2)) : max(1, min(M, 1024 / M));
  const int nwm = (M + 63) >> 6;
  const bool mine = t < M;
  if (t == 0) { st->kmax = k; st->keff = 1; st->stop = 0; st->status = 0; }
  const double t0 = mine ? T[t] : 0.0;
  const double nrm = sqrt(block_sum_nw(t0 * t0, red, nwm));
  if (mine) V[t] = t0 / nrm;
  __syncthreads();
  const double* xp = V;   // vector multiplied by H in this step ...
  double xs = 1.0;        // ... and the scale applied to the product
  double amax = 0;
  int keff = 1;
  double wv = 0;
  for (int j = 0; j < k; j++) {
    if (even) {
      // rows 2 rp and 2 rp + 1 of each column in one 16-byte load (the
      // product is bound by load instructions, not bytes)
      if (t < S * P2) {
        const int rp = t % P2, sl = t / P2;
        const __attribute__((address_space(1))) dv2* hp = (const __attribute__((address_space(1))) dv2*)(H + 2 * rp);
        double a0 = 0, a1 = 0;
        int c = sl;
        for (; c + 15 * S < M; c += 16 * S) {
          dv2 hv[16];
#pragma unroll
          for (int u = 0; u < 16; u++) hv[u] = hp[(int64_t)(c + u * S) * P2];
#pragma unroll
          for (int u = 0; u < 16; u++) {
            const double xv = xp[c + u * S];
            a0 += hv[u].x * xv;
            a1 += hv[u].y * xv;
          }
        }
        for (; c < M; c += S) {
          const dv2 hv = hp[(int64_t)c * P2];
          a0 += hv.x * xp[c];
          a1 += hv.y * xp[c];
        }
        part[sl * M + 2 * rp] = a0;
        part[sl * M + 2 * rp + 1] = a1;
      }
    } else if (t < S * M) {
      const int r = t % M, sl = t / M;
      const __attribute__((address_space(1))) double* hp = H + r;
      double acc = 0;
      int c = sl;
      for (; c + 15 * S < M; c += 16 * S) {
        double hv[16];
#pragma unroll
        for (int u = 0; u < 16; u++) hv[u] = hp[(int64_t)(c + u * S) * M];
#pragma unroll
        for (int u = 0; u < 16; u++) acc += hv[u] * xp[c + u * S];
      }
      for (; c < M; c += S) acc += hp[(int64_t)c * M] * xp[c];
      part[sl * M + r] = acc;
    }
    __syncthreads();
    double u = 0;
    if (mine) {
      for (int sl = 0; sl < S; sl++) u += part[sl * M + t];
      u *= xs;
      ub[t] = u;
      if (j > 0) V[(int64_t)j * M + t] = wv * xs;
    }
    __syncthreads();
    for (int i = wave; i <= j; i += 16) {   // V_i . u
      const double* vi = V + (int64_t)i * M;
      double d = 0;
      for (int e = lane; e < M; e += 64) d += vi[e] * ub[e];
      d = wave_sum(d);
      if (lane == 0) hs[i] = d;
    }
    __syncthreads();
    const double a = hs[j];
    if (t == 0) st->alpha[j] = a;
    amax = fmax(amax, fabs(a));
    if (j == k - 1) break;
    wv = u;
    if (mine) {
      for (int i = 0; i <= j; i++) wv -= hs[i] * V[(int64_t)i * M + t];
      w[t] = wv;
    }
    __syncthreads();
    for (int i = wave; i <= j; i += 16) {   // V_i . w
      const double* vi = V + (int64_t)i * M;
      double d = 0;
      for (int e = lane; e < M; e += 64) d += vi[e] * w[e];
      d = wave_sum(d);
      if (lane == 0) hs2[i] = d;
    }
    __syncthreads();
    if (mine) {
      for (int i = 0; i <= j; i++) wv -= hs2[i] * V[(int64_t)i * M + t];
      w[t] = wv;
    }
    const double b = sqrt(block_sum_nw(wv * wv, red, nwm));
    if (!(b > 1e-14 * amax)) break;
    if (t == 0) st->beta[j] = b;
    keff = j + 2;
    xp = w;
    xs = 1.0 / b;
  }
  if (t == 0) st->keff = keff;
  __syncthreads();
  if (t < 64) tridiag_solve_wave(st, tri_lds);
  __syncthreads();
  if (t < keff) hs[t] = st->y[t];
  __syncthreads();
  double u = 0;
  if (mine)
    for (int i = 0; i < keff; i++) u += hs[i] * V[(int64_t)i * M + t];
  const double nr = sqrt(block_sum_nw(u * u, red, nwm));
  if (mine) T[t] = u / nr;
  if (t == 0 && !(nr > 0 && isfinite(nr))) fail_status(st, 1);
}

// out = sum_i y_i V_i with partial ||out||^2
__global__ __launch_bounds__(256) void k_kritz(const KJob* __restrict__ jobs) {
  __shared__ double red[4];
  __shared__ double ys[128];
  const KJob& J = jobs[blockIdx.y];
  const KrylovState* st = J.st;
  const int k = st->keff;
  if (threadIdx.x < k) ys[threadIdx.x] = st->y[threadIdx.x];
  __syncthreads();
  const int b = blockIdx.x;
  double acc2 = 0;
  for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256) {
    double x = 0;
    for (int i = 0; i < k; i++) x += ys[i] * J.V[(int64_t)i * J.n + e];
    J.T[e] = x;
    acc2 += x * x;
  }
  const double s = block_sum(acc2, red);
  if (threadIdx.x == 0) parea(J, 0)[b] = s;
}

// ============================================================================ Davidson form
// Davidson's method for the local eigenproblem (an eigensolver form beside the
// Lanczos method; E. R. Davidson, J. Comput. Phys. 17 (1975)): Rayleigh-Ritz on
// an orthonormal basis V with W = H V, residual of the lowest Ritz pair,
// correction from the H_eff diagonal (Jacobi) or from a pointwise model of
// the exact Jacobi-Davidson correction, two classical Gram-Schmidt passes.
__device__ __forceinline__ double* darea(const DJob& J, int i) { return J.red + (int64_t)i * kDavMax * kRedBlocks; }

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// diag(H_eff): every two-leg item and local operator contributes coef times
// the product of its operators' diagonals (identity -> 1), every expanded
// three-leg product the product of three diagonals.  A4 = partial max |diag|.
__global__ __launch_bounds__(256) void k_heff_diag(const TinyPlan* __restrict__ plan, const DJob* __restrict__ job) {
  __shared__ double red[4];
  const DJob& J = *job;
  const TinyPlan P = *plan;
  const int d0 = P.d0, d1 = P.d1, d2 = P.d2;
  double mx = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256) {
    const int l = (int)(e / ((int64_t)d1 * d2)), r = (int)((e / d2) % d1), p = (int)(e % d2);
    double acc = 0;
    for (int it = P.item0[0]; it < P.item0[0] + P.nitem[0]; it++)
      acc += P.items[it].coef * blk((const double*)P.items[it].A, d1, r, r) * blk((const double*)P.items[it].B, d2, p, p);
    for (int it = P.item0[1]; it < P.item0[1] + P.nitem[1]; it++)
      acc += P.items[it].coef * blk((const double*)P.items[it].A, d0, l, l) * blk((const double*)P.items[it].B, d2, p, p);
    for (int it = P.item0[2]; it < P.item0[2] + P.nitem[2]; it++)
      acc += P.items[it].coef * blk((const double*)P.items[it].A, d0, l, l) * blk((const double*)P.items[it].B, d1, r, r);
    for (int it = 0; it < P.n3; it++) {
      const Item3& q = P.items3[it];
      acc += q.coef * blk((const double*)q.op[0], d0, l, l) * blk((const double*)q.op[1], d1, r, r) *
             blk((const double*)q.op[2], d2, p, p);
    }
    J.diag[e] = acc;
    mx = fmax(mx, fabs(acc));
  }
  const double m = block_max(mx, red);
  if (threadIdx.x == 0) darea(J, 4)[blockIdx.x] = m;
}

// A1[i] = partial sums of V_i . W_{k-1}, i < k
__global__ __launch_bounds__(256) void k_dav_dots(const DJob* __restrict__ job, int k) {
  __shared__ double red[4];
  const DJob& J = *job;
  const double* w = J.W + (int64_t)(k - 1) * J.n;
  for (int i = 0; i < k; i++) {
    const double* v = J.V + (int64_t)i * J.n;
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
      acc += v[e] * w[e];
    const double sm = block_sum(acc, red);
    if (threadIdx.x == 0) darea(J, 1)[i * kRedBlocks + blockIdx.x] = sm;
  }
}

// Complete column k-1 of G and diagonalise G (k x k) by the cyclic Jacobi
// method with round-robin pairs (all disjoint rotations of a round at once:
// rows first, then columns).  One workgroup.
__global__ __launch_bounds__(256) void k_dav_eig(const DJob* __restrict__ job, int k) {
  __shared__ double red[4];
  __shared__ double A[kDavMax][kDavMax + 1];
  __shared__ double Yl[kDavMax][kDavMax + 1];
  __shared__ double rc[kDavMax / 2], rs[kDavMax / 2];
  __shared__ int rp[kDavMax / 2], rq[kDavMax / 2];
  __shared__ int order[kDavMax];
  __shared__ double offs;
  const DJob& J = *job;
  DavState* ds = J.ds;
  const int tid = threadIdx.x;
  for (int i = 0; i < k; i++) {
    const double g = sum_partials(darea(J, 1) + i * kRedBlocks, red);
    if (tid == 0) {
      ds->G[(k - 1) * kDavMax + i] = g;
      ds->G[i * kDavMax + (k - 1)] = g;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) {
    const int i = e / k, j = e - i * k;
    A[i][j] = 0.5 * (ds->G[j * kDavMax + i] + ds->G[i * kDavMax + j]);
    Yl[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kk = k + (k & 1);
  const int np = kk / 2;
  for (int sweep = 0; sweep < 20 && k > 1; sweep++) {
    if (tid == 0) {
      double off = 0, fro = 0;
      for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++) {
          fro += A[i][j] * A[i][j];
          if (j > i) off += A[i][j] * A[i][j];
        }
      offs = off <= 1e-32 * fro ? 1.0 : 0.0;
    }
    __syncthreads();
    if (offs != 0.0) break;
    for (int round = 0; round < kk - 1; round++) {
      if (tid < np) {
        // round-robin schedule: player 0 fixed, the others rotate
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (kk - 1); };
        int p = player(tid), q = player(kk - 1 - tid);
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double apq = A[p][q];
          if (apq != 0.0) {
            const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = th == 0.0 ? 1.0 : (th > 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        } else {
          q = p;   // dummy pair
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s;
      }
      __syncthreads();
      for (int w = tid; w < np * k; w += 256) {   // rows p, q
        const int pi = w / k, j = w - pi * k;
        const int p = rp[pi], q = rq[pi];
        if (p == q) continue;
        const double c = rc[pi], s = rs[pi];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int w = tid; w < np * k; w += 256) {   // columns p, q of A and Y
        const int pi = w / k, i = w - pi * k;
        const int p = rp[pi], q = rq[pi];
        if (p == q) continue;
        const double c = rc[pi], s = rs[pi];
        const double ap = A[i][p], aq = A[i][q];
        A[i][p] = c * ap - s * aq;
        A[i][q] = s * ap + c * aq;
        const double yp = Yl[i][p], yq = Yl[i][q];
        Yl[i][p] = c * yp - s * yq;
        Yl[i][q] = s * yp + c * yq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    for (int i = 0; i < k; i++) order[i] = i;
    for (int i = 0; i < k; i++)
      for (int j = i + 1; j < k; j++)
        if (A[order[j]][order[j]] < A[order[i]][order[i]]) { const int x = order[i]; order[i] = order[j]; order[j] = x; }
    for (int i = 0; i < k; i++) ds->ev[i] = A[order[i]][order[i]];
    ds->theta = A[order[0]][order[0]];
    if (!isfinite(ds->theta)) ds->status = 1;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) {
    const int i = e / k, j = e - i * k;
    ds->Y[j * kDavMax + i] = Yl[i][order[j]];
  }
}

// u = V y_0, r = W y_0 - theta u; A0 = ||r||^2, A2 = max |r|, A3 = ||u||^2 (partials)
__global__ __launch_bounds__(256) void k_dav_resid(const DJob* __restrict__ job, int k) {
  __shared__ double red[4];
  __shared__ double y[kDavMax];
  const DJob& J = *job;
  if (threadIdx.x < k) y[threadIdx.x] = J.ds->Y[threadIdx.x];
  __syncthreads();
  const double th = J.ds->theta;
  double r2 = 0, rmax = 0, u2 = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256) {
    double uu = 0, wy = 0;
    for (int i = 0; i < k; i++) {
      uu += y[i] * J.V[(int64_t)i * J.n + e];
      wy += y[i] * J.W[(int64_t)i * J.n + e];
    }
    const double rr = wy - th * uu;
    J.u[e] = uu;
    J.r[e] = rr;
    r2 += rr * rr;
    u2 += uu * uu;
    rmax = fmax(rmax, fabs(rr));
  }
  const double a = block_sum(r2, red);
  if (threadIdx.x == 0) darea(J, 0)[blockIdx.x] = a;
  const double b = block_sum(u2, red);
  if (threadIdx.x == 0) darea(J, 3)[blockIdx.x] = b;
  const double c = block_max(rmax, red);
  if (threadIdx.x == 0) darea(J, 2)[blockIdx.x] = c;
}

// the norms every correction kernel starts from (same fixed-order reduction in
// every workgroup); block 0 records them and the convergence test
__device__ __forceinline__ bool dav_prologue(const DJob& J, double tol, double* red, double& th,
                                             double& rinf, double& dinf) {
  const double r2 = sum_partials(darea(J, 0), red);
  rinf = fmax(block_max(darea(J, 2)[threadIdx.x], red), 1e-300);
  dinf = fmax(block_max(darea(J, 4)[threadIdx.x], red), 1e-300);
  th = J.ds->theta;
  const double rn = sqrt(r2);
  const bool conv = rn <= tol;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    J.ds->rnorm = rn;
    J.ds->rinf = rinf;
    J.ds->dinf = dinf;
    J.ds->converged = conv ? 1 : 0;
    J.ds->tbad = 0;
    J.ds->status = isfinite(rn) ? 0 : 1;
  }
  return conv;
}

// t and the first Gram-Schmidt dots (A5[i] = V_i . t) and A7 = ||t||^2
__device__ __forceinline__ void dav_epilogue(const DJob& J, int k, double* red) {
  for (int i = 0; i < k; i++) {
    const double* v = J.V + (int64_t)i * J.n;
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
      acc += v[e] * J.t[e];
    const double sm = block_sum(acc, red);
    if (threadIdx.x == 0) darea(J, 5)[i * kRedBlocks + blockIdx.x] = sm;
  }
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
    acc += J.t[e] * J.t[e];
  const double sm = block_sum(acc, red);
  if (threadIdx.x == 0) darea(J, 7)[blockIdx.x] = sm;
}

// Jacobi correction t_i = -r_i / (diag_i - theta), |diag_i - theta| >= 1e-8 max(1, |theta|)
__global__ __launch_bounds__(256) void k_dav_jacobi(const DJob* __restrict__ job, int k, double tol) {
  __shared__ double red[4];
  const DJob& J = *job;
  double th, rinf, dinf;
  if (dav_prologue(J, tol, red, th, rinf, dinf)) return;
  const double eps = 1e-8 * fmax(1.0, fabs(th));
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256) {
    double den = J.diag[e] - th;
    if (fabs(den) < eps) den = den < 0 ? -eps : eps;
    J.t[e] = -J.r[e] / den;
  }
  dav_epilogue(J, k, red);
}

// Pointwise model: features ((diag - theta)/s, r/||r||_inf, theta/s), s = ||diag||_inf,
// three tanh layers of width 64 (FP16 parameters, FP32 arithmetic), linear output o,
// t = o ||r||_inf / s.
__device__ __forceinline__ float mlp_eval(const float* __restrict__ w, float f0, float f1, float f2) {
  const float* W1 = w;
  const float* b1 = W1 + 3 * kMlpHidden;
  const float* W2 = b1 + kMlpHidden;
  const float* b2 = W2 + kMlpHidden * kMlpHidden;
  const float* W3 = b2 + kMlpHidden;
  const float* b3 = W3 + kMlpHidden * kMlpHidden;
  const float* W4 = b3 + kMlpHidden;
  const float b4 = W4[kMlpHidden];
  float h1[kMlpHidden], h2[kMlpHidden];
#pragma unroll
  for (int j = 0; j < kMlpHidden; j++)
    h1[j] = tanhf(b1[j] + f0 * W1[j] + f1 * W1[kMlpHidden + j] + f2 * W1[2 * kMlpHidden + j]);
#pragma unroll
  for (int j = 0; j < kMlpHidden; j++) {
    float a = b2[j];
#pragma unroll
    for (int i = 0; i < kMlpHidden; i++) a += h1[i] * W2[i * kMlpHidden + j];
    h2[j] = tanhf(a);
  }
  float o = b4;
#pragma unroll 4
  for (int j = 0; j < kMlpHidden; j++) {
    float a = b3[j];
#pragma unroll
    for (int i = 0; i < kMlpHidden; i++) a += h2[i] * W3[i * kMlpHidden + j];
    o += W4[j] * tanhf(a);
  }
  return o;
}

__global__ __launch_bounds__(256) void k_dav_learned(const DJob* __restrict__ job, int k, double tol) {
  __shared__ double red[4];
  __shared__ float w[kMlpParams];
  const DJob& J = *job;
  double th, rinf, dinf;
  if (dav_prologue(J, tol, red, th, rinf, dinf)) return;
  const _Float16* wp = (const _Float16*)J.mlp;
  for (int i = threadIdx.x; i < kMlpParams; i += 256) w[i] = (float)wp[i];
  __syncthreads();
  const float is = (float)(1.0 / dinf), ir = (float)(1.0 / rinf), f2 = (float)(th / dinf);
  const double scale = rinf / dinf;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256) {
    const float f0 = (float)(J.diag[e] - th) * is;
    const float f1 = (float)J.r[e] * ir;
    J.t[e] = (double)mlp_eval(w, f0, f1, f2) * scale;
  }
  dav_epilogue(J, k, red);
}

// reduce A7 -> tnorm2; flag a non-finite correction
__global__ __launch_bounds__(256) void k_dav_check(const DJob* __restrict__ job) {
  __shared__ double red[4];
  const DJob& J = *job;
  const double t2 = sum_partials(darea(J, 7), red);
  if (threadIdx.x == 0) {
    J.ds->tnorm2 = t2;
    if (!J.ds->converged && !isfinite(t2)) J.ds->tbad = 1;
  }
}

// Gram-Schmidt pass on t against V[0..k): coefficients from area pin, then new
// dots into pin + 1 (or ||t||^2 into A7 when last)
__global__ __launch_bounds__(256) void k_dav_ortho(const DJob* __restrict__ job, int k, int pin, int last) {
  __shared__ double red[4];
  __shared__ double hs[kDavMax];
  const DJob& J = *job;
  for (int i = 0; i < k; i++) {
    const double hv = sum_partials(darea(J, pin) + i * kRedBlocks, red);
    if (threadIdx.x == 0) hs[i] = hv;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256) {
    double x = J.t[e];
    for (int i = 0; i < k; i++) x -= hs[i] * J.V[(int64_t)i * J.n + e];
    J.t[e] = x;
  }
  if (last) {
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
      acc += J.t[e] * J.t[e];
    const double sm = block_sum(acc, red);
    if (threadIdx.x == 0) darea(J, 7)[blockIdx.x] = sm;
    return;
  }
  for (int i = 0; i < k; i++) {
    const double* v = J.V + (int64_t)i * J.n;
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
      acc += v[e] * J.t[e];
    const double sm = block_sum(acc, red);
    if (threadIdx.x == 0) darea(J, pin + 1)[i * kRedBlocks + blockIdx.x] = sm;
  }
}

// V[slot] = t / ||t|| (A7); breakdown when ||t|| vanishes
__global__ __launch_bounds__(256) void k_dav_append(const DJob* __restrict__ job, int slot) {
  __shared__ double red[4];
  const DJob& J = *job;
  const double nt = sqrt(sum_partials(darea(J, 7), red));
  const bool brk = !(nt > 1e-300) || !isfinite(nt);
  if (blockIdx.x == 0 && threadIdx.x == 0 && brk) J.ds->status = 2;
  if (brk) return;
  const double inv = 1.0 / nt;
  double* out = J.V + (int64_t)slot * J.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256)
    out[e] = J.t[e] * inv;
}

// restart: Vt[j] = V Y[:, j], Vt[nr + j] = W Y[:, j] (j < nr); G = diag(ev[0..nr))
__global__ __launch_bounds__(256) void k_dav_restart(const DJob* __restrict__ job, int k, int nr) {
  __shared__ double Ys[kDavMax * kDavMax];
  const DJob& J = *job;
  for (int e = threadIdx.x; e < kDavMax * kDavMax; e += 256) Ys[e] = J.ds->Y[e];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256)
    for (int j = 0; j < nr; j++) {
      double a = 0, b = 0;
      for (int i = 0; i < k; i++) {
        const double y = Ys[j * kDavMax + i];
        a += y * J.V[(int64_t)i * J.n + e];
        b += y * J.W[(int64_t)i * J.n + e];
      }
      J.Vt[(int64_t)j * J.n + e] = a;
      J.Vt[(int64_t)(nr + j) * J.n + e] = b;
    }
  if (blockIdx.x == 0)
    for (int e = threadIdx.x; e < kDavMax * kDavMax; e += 256) {
      const int i = e % kDavMax, j = e / kDavMax;
      J.ds->G[e] = (i == j && i < nr) ? J.ds->ev[i] : 0.0;
    }
}

// T = u / ||u|| (A3)
__global__ __launch_bounds__(256) void k_dav_final(const DJob* __restrict__ job) {
  __shared__ double red[4];
  const DJob& J = *job;
  const double nu = sqrt(sum_partials(darea(J, 3), red));
  if (blockIdx.x == 0 && threadIdx.x == 0 && !(nu > 0 && isfinite(nu))) J.ds->status = 1;
  const double inv = 1.0 / nu;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256)
    J.T[e] = J.u[e] * inv;
}

__global__ __launch_bounds__(256) void k_dav_init(const DJob* __restrict__ job) {
  DavState* ds = job->ds;
  for (int e = threadIdx.x; e < kDavMax * kDavMax; e += 256) { ds->G[e] = 0; ds->Y[e] = 0; }
  if (threadIdx.x < kDavMax) ds->ev[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ds->theta = 0; ds->rnorm = 0; ds->rinf = 0; ds->dinf = 0; ds->tnorm2 = 0;
    ds->converged = 0; ds->tbad = 0; ds->status = 0;
  }
}

// V[0] = T / ||T||
__global__ __launch_bounds__(256) void k_dav_start(const DJob* __restrict__ job, int phase) {
  __shared__ double red[4];
  const DJob& J = *job;
  if (phase == 0) {
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
      acc += J.T[e] * J.T[e];
    const double sm = block_sum(acc, red);
    if (threadIdx.x == 0) darea(J, 3)[blockIdx.x] = sm;
    return;
  }
  const double nr = sqrt(sum_partials(darea(J, 3), red));
  if (blockIdx.x == 0 && threadIdx.x == 0 && !(nr > 0 && isfinite(nr))) J.ds->status = 1;
  const double inv = 1.0 / nr;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)kRedBlocks * 256)
    J.V[e] = J.T[e] * inv;
}

// FP32 -> FP16 parameter copy
__global__ __launch_bounds__(256) void k_to_half(const float* __restrict__ s, _Float16* __restrict__ d, int n) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) d[e] = (_Float16)s[e];
}

// ============================================================================ correction model: training
// Mean-squared-error training of the pointwise model with hand-written kernels
// (FP32 master parameters, Adam).  Parameter layout: W1 [3][64], b1, W2 [64][64],
// b2, W3 [64][64], b3, W4 [64], b4 (row-major, h_next = tanh(h W + b)).
// k_mlp_grad: one wavefront = 64 points; forward, backward by the chain rule,
// per-workgroup gradient sums into gpart[block][kMlpParams + 1] (last = sum e^2).
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ feats,
                                                 const float* __restrict__ targets, int64_t off, int batch,
                                                 float* __restrict__ gpart) {
  constexpr int H = kMlpHidden, LD = kMlpHidden + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* h1 = reinterpret_cast<float*>(smem_raw);
  float* h2 = h1 + 64 * LD;
  float* h3 = h2 + 64 * LD;
  float* d1 = h3 + 64 * LD;
  float* d2 = d1 + 64 * LD;
  float* d3 = d2 + 64 * LD;
  float* fs = d3 + 64 * LD;        // [64][3]
  float* gos = fs + 64 * 3;        // [64]
  float* es = gos + 64;            // [64]
  const float* W1 = w;
  const float* b1 = W1 + 3 * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H * H;
  const float* W4 = b3 + H;
  const float b4 = W4[H];
  const int t = threadIdx.x;
  const int64_t pt = off + (int64_t)blockIdx.x * 64 + t;
  const float f0 = feats[pt * 3], f1 = feats[pt * 3 + 1], f2 = feats[pt * 3 + 2];
  fs[t * 3] = f0; fs[t * 3 + 1] = f1; fs[t * 3 + 2] = f2;
  float a[H];
#pragma unroll
  for (int j = 0; j < H; j++) {
    a[j] = tanhf(b1[j] + f0 * W1[j] + f1 * W1[H + j] + f2 * W1[2 * H + j]);
    h1[t * LD + j] = a[j];
  }
  float c[H];
#pragma unroll
  for (int j = 0; j < H; j++) {
    float x = b2[j];
#pragma unroll
    for (int i = 0; i < H; i++) x += a[i] * W2[i * H + j];
    c[j] = tanhf(x);
    h2[t * LD + j] = c[j];
  }
  float o = b4;
#pragma unroll
  for (int j = 0; j < H; j++) {
    float x = b3[j];
#pragma unroll
    for (int i = 0; i < H; i++) x += c[i] * W3[i * H + j];
    const float y = tanhf(x);
    h3[t * LD + j] = y;
    o += W4[j] * y;
  }
  const float e = o - targets[pt];
  const float go = 2.0f * e / (float)batch;
  gos[t] = go;
  es[t] = e * e;
  // backward for this point
#pragma unroll
  for (int j = 0; j < H; j++) {
    const float y = h3[t * LD + j];
    d3[t * LD + j] = go * W4[j] * (1.0f - y * y);
  }
#pragma unroll 4
  for (int i = 0; i < H; i++) {
    float x = 0;
#pragma unroll
    for (int j = 0; j < H; j++) x += d3[t * LD + j] * W3[i * H + j];
    const float y = h2[t * LD + i];
    d2[t * LD + i] = x * (1.0f - y * y);
  }
#pragma unroll 4
  for (int i = 0; i < H; i++) {
    float x = 0;
#pragma unroll
    for (int j = 0; j < H; j++) x += d2[t * LD + j] * W2[i * H + j];
    const float y = h1[t * LD + i];
    d1[t * LD + i] = x * (1.0f - y * y);
  }
  __syncthreads();
  // parameter gradients summed over the 64 points: thread t owns column j = t
  float* g = gpart + (int64_t)blockIdx.x * (kMlpParams + 1);
  const int j = t;
  {
    float s0 = 0, s1 = 0, s2 = 0, sb = 0;
    for (int p = 0; p < 64; p++) {
      const float dd = d1[p * LD + j];
      s0 += fs[p * 3] * dd; s1 += fs[p * 3 + 1] * dd; s2 += fs[p * 3 + 2] * dd; sb += dd;
    }
    g[j] = s0; g[H + j] = s1; g[2 * H + j] = s2; g[3 * H + j] = sb;
  }
  float* gW2 = g + 4 * H;
  float* gb2 = gW2 + H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H * H;
  float* gW4 = gb3 + H;
  for (int i = 0; i < H; i++) {
    float x2 = 0, x3 = 0;
    for (int p = 0; p < 64; p++) {
      x2 += h1[p * LD + i] * d2[p * LD + j];
      x3 += h2[p * LD + i] * d3[p * LD + j];
    }
    gW2[i * H + j] = x2;
    gW3[i * H + j] = x3;
  }
  float sb2 = 0, sb3 = 0, s4 = 0;
  for (int p = 0; p < 64; p++) {
    sb2 += d2[p * LD + j];
    sb3 += d3[p * LD + j];
    s4 += h3[p * LD + j] * gos[p];
  }
  gb2[j] = sb2; gb3[j] = sb3; gW4[j] = s4;
  if (t == 0) {
    float sg = 0, se = 0;
    for (int p = 0; p < 64; p++) { sg += gos[p]; se += es[p]; }
    gW4[H] = sg;               // b4
    g[kMlpParams] = se;        // sum of squared errors
  }
}

// grad[i] = sum over blocks (fixed order) of gpart[b][i]
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ gpart, int nblk, float* __restrict__ grad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i > kMlpParams) return;
  float acc = 0;
  for (int b = 0; b < nblk; b++) acc += gpart[(int64_t)b * (kMlpParams + 1) + i];
  grad[i] = acc;
}

// Adam step `step` (from 1); loss[step - 1] = mean squared error of the batch
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ w, const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v, int step,
                                                  float lr, int batch, float* __restrict__ loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && loss) loss[step - 1] = grad[kMlpParams] / (float)batch;
  if (i >= kMlpParams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)step));
  const float vh = vi / (1.0f - powf(b2, (float)step));
  w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// inference of the model on given features (FP16 parameters)
__global__ __launch_bounds__(256) void k_mlp_eval(const _Float16* __restrict__ wp, const float* __restrict__ feats,
                                                  float* __restrict__ out, int64_t n) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += 256) w[i] = (float)wp[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    out[e] = mlp_eval(w, feats[e * 3], feats[e * 3 + 1], feats[e * 3 + 2]);
}

// ---- exact Jacobi-Davidson corrections (training data): small vector kernels
__global__ __launch_bounds__(256) void k_vdot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                              double* __restrict__ partial) {
  __shared__ double red[4];
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)kRedBlocks * 256) acc += a[e] * b[e];
  const double sm = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = sm;
}

// y = alpha x + beta y
__global__ __launch_bounds__(256) void k_axpby(double alpha, const double* __restrict__ x, double beta,
                                               double* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    y[e] = beta == 0.0 ? alpha * x[e] : alpha * x[e] + beta * y[e];   // y is not read when beta = 0
}

// training pair of one Davidson iteration: features of every entry and the
// exact correction x scaled like the model output
__global__ __launch_bounds__(256) void k_harvest_write(const double* __restrict__ diag, const double* __restrict__ r,
                                                       const double* __restrict__ x, double theta, double s,
                                                       double rinf, float* __restrict__ feats,
                                                       float* __restrict__ targets, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    feats[e * 3] = (float)((diag[e] - theta) / s);
    feats[e * 3 + 1] = (float)(r[e] / rinf);
    feats[e * 3 + 2] = (float)(theta / s);
    targets[e] = (float)(x[e] * s / rinf);
  }
}

// ============================================================================ QR helpers
// Cholesky of G + shift*I = L L^T (R = L^T upper with positive diagonal) and
// the inverse of R, one workgroup.  G is column-major.  Outputs: R
// column-major, RinvRow = R^{-1} row-major (= X = L^{-1} column-major).
// shift_mode 1: shift = 11 (rows n + n (n + 1)) u trace(G) (shifted CholeskyQR
// of Fukaya et al.), making the factorisation safe for ill-conditioned input.
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// (a) n = 16, 32, 48 or 64, blocked, one wavefront; A (the trailing matrix,
//      then L) and X = L^{-1} column-major in LDS with an odd stride.
//      Cholesky by panels of 16 columns: a panel is factorised with one lane
//      per row (the row's 16 panel entries in registers; the pivot and the
//      panel column broadcast by readlane), then the trailing matrix takes the
//      rank-16 update A_IJ -= L_I L_J^T on the matrix cores, one 16 x 16 tile
//      (I >= J) at a time.  The inverse: the diagonal blocks X_bb = L_bb^{-1}
//      by forward substitution (lane group b of 16 lanes, one lane per
//      column), then the blocks below the diagonal block row by block row,
//      X_IJ = -X_II (sum_{J <= K < I} L_IK X_KJ), on the matrix cores: the
//      accumulator item s of T = sum L X holds rows 4 s + lane / 16 of T,
//      exactly the B operand of K-slice s of X_II T.
constexpr int kCholLd = 65;

template <int NB, int KB>
__device__ __forceinline__ void chol_panel(double* A, int lane, int& bad) {
  constexpr int c0 = 16 * KB;
  double p[16];
#pragma unroll
  for (int u = 0; u < 16; u++) p[u] = A[(c0 + u) * kCholLd + lane];
#pragma unroll
  for (int u = 0; u < 16; u++) {
    const int k = c0 + u;
    const double d = readlane_d(p[u], k);
    if (!(d > 0.0) || !isfinite(d)) bad = 1;
    // 1 / sqrt(d) from the hardware estimate and two Newton steps; the
    // pivot is d times it
    const double dd = fmax(d, 1e-300);
    double inv = __builtin_amdgcn_rsq(dd);
    inv = inv * fma(-0.5 * dd * inv, inv, 1.5);
    inv = inv * fma(-0.5 * dd * inv, inv, 1.5);
    const double piv = dd * inv;
    const double l = lane > k ? p[u] * inv : (lane == k ? piv : 0.0);   // L(lane, k)
    p[u] = l;
#pragma unroll
    for (int v = u + 1; v < 16; v++) p[v] = fma(-l, readlane_d(l, c0 + v), p[v]);
  }
#pragma unroll
  for (int u = 0; u < 16; u++) A[(c0 + u) * kCholLd + lane] = p[u];
}

template <int NB, int KB>
__device__ __forceinline__ void chol_trailing(double* A, int lane) {
  const int l16 = lane & 15, l4 = lane >> 4;
  constexpr int c0 = 16 * KB;
#pragma unroll
  for (int J = KB + 1; J < NB; J++)
#pragma unroll
    for (int I = J; I < NB; I++) {
      double* tile = A + (16 * J + l16) * kCholLd + 16 * I + l4;   // D[l4 + 4 i][l16] = A(16 I + l4 + 4 i, 16 J + l16)
      d4 acc;
#pragma unroll
      for (int i = 0; i < 4; i++) acc[i] = tile[4 * i];
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const double* col = A + (c0 + 4 * s + l4) * kCholLd;
        acc = mfma16(-col[16 * I + l16], col[16 * J + l16], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; i++) tile[4 * i] = acc[i];
    }
}

template <int NB, int KB>
__device__ __forceinline__ void chol_blocks(double* A, int lane, int& bad) {
  chol_panel<NB, KB>(A, lane, bad);
  wave_sync();
  if constexpr (KB + 1 < NB) {
    chol_trailing<NB, KB>(A, lane);
    wave_sync();
    chol_blocks<NB, KB + 1>(A, lane, bad);
  }
}

template <int NB, int I>
__device__ __forceinline__ void trinv_blocks(const double* A, double* X, int lane) {
  const int l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
  for (int Jb = 0; Jb < I; Jb++) {
    d4 T = {0, 0, 0, 0};
#pragma unroll
    for (int K = Jb; K < I; K++)
#pragma unroll
      for (int s = 0; s < 4; s++)
        T = mfma16(A[(16 * K + 4 * s + l4) * kCholLd + 16 * I + l16],    // L(16 I + l16, 16 K + 4 s + l4)
                   X[(16 * Jb + l16) * kCholLd + 16 * K + 4 * s + l4],   // X(16 K + 4 s + l4, 16 Jb + l16)
                   T);
    d4 Rt = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; s++) Rt = mfma16(-X[(16 * I + 4 * s + l4) * kCholLd + 16 * I + l16], T[s], Rt);
    double* tile = X + (16 * Jb + l16) * kCholLd + 16 * I + l4;
#pragma unroll
    for (int i = 0; i < 4; i++) tile[4 * i] = Rt[i];
  }
  if constexpr (I + 1 < NB) {
    wave_sync();
    trinv_blocks<NB, I + 1>(A, X, lane);
  }
}

template <int N>
__global__ __launch_bounds__(64) void k_chol_inv_blk(const double* __restrict__ G, double* __restrict__ R,
                                                     double* __restrict__ RinvRow, int shift_mode, int64_t rows,
                                                     KrylovState* __restrict__ st) {
  static_assert(N % 16 == 0 && N <= 64, "blocks of 16, one lane per row");
  constexpr int NB = N / 16;
  __shared__ double A[64 * kCholLd];   // A(i, j) at j * kCholLd + i
  __shared__ double X[64 * kCholLd];
  const int lane = threadIdx.x;
  const bool own = lane < N;
  const double tr = wave_sum(own ? G[(int64_t)lane * N + lane] : 0.0);
  const double shift =
      shift_mode ? 11.0 * ((double)rows * N + (double)N * (N + 1)) * 1.1102230246251565e-16 * tr : 0.0;
  // A = G + shift I, column by column (coalesced); only the lower triangle
  // takes part in the factorisation: an entry above the diagonal only ever
  // meets a zero multiplier or is overwritten
  {
    double g[N];   // all loads in flight at once
#pragma unroll
    for (int j = 0; j < N; j++) g[j] = own ? G[(int64_t)j * N + lane] : 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) A[j * kCholLd + lane] = g[j] + (lane == j ? shift : 0.0);
  }
  wave_sync();
  int bad = 0;
  chol_blocks<NB, 0>(A, lane, bad);
  // diagonal blocks of X: lane group b, column 16 b + (lane % 16)
  {
    const int b = lane >> 4, j = lane & 15;
    if (b < NB) {
      const double* Lb = A + 16 * b * kCholLd + 16 * b;   // L_bb(r, p) at p * kCholLd + r
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        double acc = r == j ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < r; q++) acc = fma(-Lb[q * kCholLd + r], x[q], acc);
        x[r] = acc / Lb[r * kCholLd + r];
      }
#pragma unroll
      for (int r = 0; r < 16; r++) X[(16 * b + j) * kCholLd + 16 * b + r] = x[r];
    }
  }
  wave_sync();
  if constexpr (NB > 1) {
    trinv_blocks<NB, 1>(A, X, lane);
    wave_sync();
  }
  // R = L^T column-major: R(i, j) = L(j, i); RinvRow = R^{-1} row-major = X column-major;
  // blocks above the diagonal are zero
  if (own) {
    double r[N];
#pragma unroll
    for (int j = 0; j < N; j++) r[j] = (j >> 4) >= (lane >> 4) ? A[lane * kCholLd + j] : 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) R[(int64_t)j * N + lane] = r[j];
#pragma unroll
    for (int j = 0; j < N; j++) r[j] = (j >> 4) <= (lane >> 4) ? X[j * kCholLd + lane] : 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) RinvRow[(int64_t)j * N + lane] = r[j];
  }
  if (lane == 0 && bad && st) fail_status(st, 2);
}

// (b) other n: L and X = L^{-1} as packed lower triangles (n (n + 1)
//     doubles), rank-1 updates over a 16 x 16 thread grid; in LDS for
//     n <= 128, else in the device workspace ws (the one workgroup's own
//     writes, ordered by its barriers; the triangles stay in L2).
template <bool WS>
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ G, int n,
                                                  double* __restrict__ R,
                                                  double* __restrict__ RinvRow, int shift_mode,
                                                  int64_t rows, KrylovState* __restrict__ st,
                                                  double* __restrict__ ws) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* L = WS ? ws : reinterpret_cast<double*>(smem_raw);
  double* X = L + n * (n + 1) / 2;
  __shared__ double shift;
  __shared__ int bad;
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
  if (t == 0) {
    bad = 0;
    double tr = 0;
    for (int i = 0; i < n; i++) tr += G[(int64_t)i * n + i];
    shift = shift_mode ? 11.0 * ((double)rows * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * tr : 0.0;
  }
  __syncthreads();
  for (int i = ty; i < n; i += 16)
    for (int j = tx; j <= i; j += 16) {
      L[tri(i, j)] = G[(int64_t)j * n + i] + (i == j ? shift : 0.0);
      X[tri(i, j)] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  for (int k = 0; k < n; k++) {
    const double dkk = L[tri(k, k)];
    const double piv = sqrt(fmax(dkk, 1e-300));
    const double inv = 1.0 / piv;
    __syncthreads();
    if (t == 0) {
      if (!(dkk > 0.0) || !isfinite(dkk)) bad = 1;
      L[tri(k, k)] = piv;
    }
    for (int i = k + 1 + t; i < n; i += 256) L[tri(i, k)] *= inv;
    __syncthreads();
    for (int i = k + 1 + ty; i < n; i += 16) {
      const double lik = L[tri(i, k)];
      for (int j = k + 1 + tx; j <= i; j += 16) L[tri(i, j)] -= lik * L[tri(j, k)];
    }
    __syncthreads();
  }
  for (int k = 0; k < n; k++) {
    const double inv = 1.0 / L[tri(k, k)];
    for (int c = t; c <= k; c += 256) X[tri(k, c)] *= inv;
    __syncthreads();
    for (int i = k + 1 + ty; i < n; i += 16) {
      const double lik = L[tri(i, k)];
      for (int c = tx; c <= k; c += 16) X[tri(i, c)] -= lik * X[tri(k, c)];
    }
    __syncthreads();
  }
  for (int j = ty; j < n; j += 16)
    for (int i = tx; i < n; i += 16) {
      R[(int64_t)j * n + i] = (i <= j) ? L[tri(j, i)] : 0.0;
      RinvRow[(int64_t)i * n + j] = (i <= j) ? X[tri(j, i)] : 0.0;
    }
  if (t == 0 && bad && st) fail_status(st, 2);
}

// Householder QR of a small matricisation in one workgroup (rows * n <= 16384,
// n <= 64): A[f][j] = T[.. j ..] with j the column leg.  The matrix lives in
// LDS (column-major); reflectors as in LAPACK's geqr2, Q formed in place as in
// org2r, then the signs are fixed so that diag(R) >= 0.  Q overwrites T, R
// (column-major n x n) goes to Rout.
__global__ __launch_bounds__(256) void k_qr_small(double* __restrict__ T, int d0, int d1, int d2,
                                                  int j, double* __restrict__ Rout,
                                                  KrylovState* __restrict__ st) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);
  __shared__ double tau[64];
  __shared__ double red[4];
  __shared__ double sgn[64];
  const int n = j == 0 ? d0 : (j == 1 ? d1 : d2);
  const int64_t rows = (int64_t)d0 * d1 * d2 / n;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int64_t e = t; e < rows * n; e += 256) {
    const int c = (int)(e / rows);
    const int64_t f = e - (int64_t)c * rows;
    A[e] = T[mode_addr(j, d0, d1, d2, c, f)];
  }
  __syncthreads();
  const int kmax = (int)(rows < n ? rows : n);
  for (int k = 0; k < kmax; k++) {
    double* col = A + (int64_t)k * rows;
    double s2 = 0;
    for (int64_t i = k + 1 + t; i < rows; i += 256) s2 += col[i] * col[i];
    s2 = block_sum(s2, red);
    const double alpha = col[k];
    double tk = 0, beta = alpha, scale = 0;
    if (s2 > 0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tk = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (s2 > 0) for (int64_t i = k + 1 + t; i < rows; i += 256) col[i] *= scale;
    if (t == 0) { col[k] = beta; tau[k] = tk; }
    __syncthreads();
    if (tk != 0.0) {
      // apply H_k = I - tau v v^T (v_k = 1) to columns c > k; one wave per column
      for (int c = k + 1 + wave; c < n; c += 4) {
        double* cc = A + (int64_t)c * rows;
        double w = 0;
        for (int64_t i = k + lane; i < rows; i += 64) w += (i == k ? 1.0 : col[i]) * cc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
        w *= tk;
        for (int64_t i = k + lane; i < rows; i += 64) cc[i] -= w * (i == k ? 1.0 : col[i]);
      }
    }
    __syncthreads();
  }
  // R and its sign fix
  for (int e = t; e < n * n; e += 256) {
    const int c = e / n, r = e - c * n;
    Rout[e] = (r <= c && r < kmax) ? A[(int64_t)c * rows + r] : 0.0;
  }
  if (t < n) sgn[t] = (t < kmax && A[(int64_t)t * rows + t] < 0) ? -1.0 : 1.0;
  __syncthreads();
  for (int e = t; e < n * n; e += 256) {
    const int r = e % n;
    Rout[e] *= sgn[r];
  }
  // form Q in place (org2r), columns from last to first
  for (int k = kmax - 1; k >= 0; k--) {
    double* col = A + (int64_t)k * rows;
    const double tk = tau[k];
    if (k < n - 1) {
      for (int c = k + 1 + wave; c < n; c += 4) {
        double* cc = A + (int64_t)c * rows;
        double w = 0;
        for (int64_t i = k + lane; i < rows; i += 64) w += (i == k ? 1.0 : col[i]) * cc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
        w *= tk;
        for (int64_t i = k + lane; i < rows; i += 64) cc[i] -= w * (i == k ? 1.0 : col[i]);
      }
    }
    __syncthreads();
    for (int64_t i = k + 1 + t; i < rows; i += 256) col[i] *= -tk;
    if (t == 0) col[k] = 1.0 - tk;
    for (int i = t; i < k; i += 256) col[i] = 0.0;
    __syncthreads();
  }
  for (int64_t e = t; e < rows * n; e += 256) {
    const int c = (int)(e / rows);
    const int64_t f = e - (int64_t)c * rows;
    T[mode_addr(j, d0, d1, d2, c, f)] = A[e] * sgn[c];
  }
  if (t == 0 && st && !isfinite(tau[0])) fail_status(st, 2);
}

// C = A B for n x n column-major matrices, one thread per output element
__global__ __launch_bounds__(64) void k_small_matmul(const double* __restrict__ A,
                                                     const double* __restrict__ B,
                                                     double* __restrict__ C, int n) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e >= n * n) return;
  const int j = e / n, i = e - j * n;
  double acc = 0;
  for (int k = 0; k < n; k++) acc += A[(int64_t)k * n + i] * B[(int64_t)j * n + k];
  C[e] = acc;
}

// ============================================================================ launchers
static inline unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T, int NI>
static hipError_t mode_launch(const MPTask* tasks, const MPJob* jobs, const int2* wus, int nwu,
                              const void* xbase, hipStream_t s) {
  // m_j = 32 or 64: the output rows of a work unit are spread over 2 or 4
  // workgroups (each stages a quarter or half of the free block)
  constexpr int QS = mode_qs(NI);
  const size_t lds = (size_t)16 * NI * 66 * sizeof(T);
  hipLaunchKernelGGL((k_mode<T, NI, QS>), dim3(nwu, QS), dim3(256), lds, s, tasks, jobs, wus,
                     (const T*)xbase);
  return hipGetLastError();
}

hipError_t launch_mode(int dtype, int mj, bool mfma, const MPTask* tasks, const MPJob* jobs,
                       const int2* wus, int nwu, const void* xbase, hipStream_t s, bool nt) {
  if (nwu == 0) return hipSuccess;
  if (mfma && nt && mj <= 64) {
// m_j = 32 or 64: the output rows of a tile are spread over 2 or 4 waves
#define MNT(T, NI)                                                                                        \
  {                                                                                                       \
    constexpr int QS = NI == 4 ? 4 : (NI == 2 ? 2 : 1);                                                   \
    hipLaunchKernelGGL((k_mode_nt<T, NI, QS>), dim3(nwu, QS), dim3(256), 0, s, tasks, jobs, wus,          \
                       (const T*)xbase);                                                                  \
    return hipGetLastError();                                                                             \
  }
    if (dtype == 0) {
      switch (mj / 16) { case 1: MNT(double, 1) case 2: MNT(double, 2) case 3: MNT(double, 3) case 4: MNT(double, 4) }
    } else {
      switch (mj / 16) { case 1: MNT(float, 1) case 2: MNT(float, 2) case 3: MNT(float, 3) case 4: MNT(float, 4) }
    }
#undef MNT
  }
  if (!mfma) {
    if (dtype == 0)
      hipLaunchKernelGGL(k_mode_gen<double>, dim3(nwu), dim3(256), 0, s, tasks, jobs, wus,
                         (const double*)xbase);
    else
      hipLaunchKernelGGL(k_mode_gen<float>, dim3(nwu), dim3(256), 0, s, tasks, jobs, wus,
                         (const float*)xbase);
    return hipGetLastError();
  }
#define MODE_CASES(T)                                                        \
  switch (mj / 16) {                                                         \
    case 1: return mode_launch<T, 1>(tasks, jobs, wus, nwu, xbase, s);       \
    case 2: return mode_launch<T, 2>(tasks, jobs, wus, nwu, xbase, s);       \
    case 3: return mode_launch<T, 3>(tasks, jobs, wus, nwu, xbase, s);       \
    case 4: return mode_launch<T, 4>(tasks, jobs, wus, nwu, xbase, s);       \
    case 5: return mode_launch<T, 5>(tasks, jobs, wus, nwu, xbase, s);       \
    case 6: return mode_launch<T, 6>(tasks, jobs, wus, nwu, xbase, s);       \
    case 7: return mode_launch<T, 7>(tasks, jobs, wus, nwu, xbase, s);       \
    case 8: return mode_launch<T, 8>(tasks, jobs, wus, nwu, xbase, s);       \
  }
  if (dtype == 0) { MODE_CASES(double) }
  else { MODE_CASES(float) }
#undef MODE_CASES
  return hipErrorInvalidValue;
}

template <int NI>
static hipError_t gram_launch(const GRTask* tasks, int ntask, hipStream_t s) {
  const size_t lds = (size_t)2 * 64 * (16 * NI + 2) * sizeof(double);
  hipLaunchKernelGGL(k_gram<NI>, dim3(ntask), dim3(256), lds, s, tasks);
  return hipGetLastError();
}

hipError_t launch_gram(int mj, bool mfma, const GRTask* tasks, int ntask, hipStream_t s, bool nt) {
  if (ntask == 0) return hipSuccess;
  if (mfma && nt) {
    switch (mj / 16) {
      case 1: hipLaunchKernelGGL(k_gram_nt<1>, dim3(ntask), dim3(256), 0, s, tasks); return hipGetLastError();
      case 2: hipLaunchKernelGGL(k_gram_nt<2>, dim3(ntask), dim3(256), 0, s, tasks); return hipGetLastError();
      case 3: hipLaunchKernelGGL(k_gram_nt<3>, dim3(ntask), dim3(256), 0, s, tasks); return hipGetLastError();
      case 4: hipLaunchKernelGGL(k_gram_x4, dim3(ntask), dim3(256), 0, s, tasks); return hipGetLastError();
      default: break;
    }
  }
  if (!mfma) {
    hipLaunchKernelGGL(k_gram_gen, dim3(grid1((int64_t)mj * mj), ntask), dim3(256), 0, s, tasks, mj);
    return hipGetLastError();
  }
  switch (mj / 16) {
    case 1: return gram_launch<1>(tasks, ntask, s);
    case 2: return gram_launch<2>(tasks, ntask, s);
    case 3: return gram_launch<3>(tasks, ntask, s);
    case 4: return gram_launch<4>(tasks, ntask, s);
    case 5: return gram_launch<5>(tasks, ntask, s);
    case 6: return gram_launch<6>(tasks, ntask, s);
    case 7: return gram_launch<7>(tasks, ntask, s);
    case 8: return gram_launch<8>(tasks, ntask, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gram_reduce(const GRReduce* r, int nr, int maxm, hipStream_t s) {
  if (nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_reduce, dim3(grid1((int64_t)maxm * maxm), nr), dim3(256), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_combine(const CBTask* tasks, const CBTerm* terms, int ntask, int maxn,
                          hipStream_t s) {
  if (ntask == 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(grid1(maxn), ntask), dim3(256), 0, s, tasks, terms);
  return hipGetLastError();
}

hipError_t launch_reduce_out(int dtype_in, const RDSrc* srcs, int nsrc, void* y, int dtype_out,
                             int ml, int mr, int mp, hipStream_t s) {
  const int64_t M = (int64_t)ml * mr * mp;
  if (dtype_in == 0 && dtype_out == 0)
    hipLaunchKernelGGL((k_reduce_out<double, double>), dim3(grid1(M)), dim3(256), 0, s, srcs, nsrc,
                       (double*)y, ml, mr, mp);
  else if (dtype_in == 1 && dtype_out == 0)
    hipLaunchKernelGGL((k_reduce_out<float, double>), dim3(grid1(M)), dim3(256), 0, s, srcs, nsrc,
                       (double*)y, ml, mr, mp);
  else if (dtype_in == 1 && dtype_out == 1)
    hipLaunchKernelGGL((k_reduce_out<float, float>), dim3(grid1(M)), dim3(256), 0, s, srcs, nsrc,
                       (float*)y, ml, mr, mp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_transpose_plr(int dtype, const void* x, void* xt, int ml, int mr, int mp,
                                hipStream_t s) {
  const int64_t M = (int64_t)ml * mr * mp;
  if (dtype == 0)
    hipLaunchKernelGGL(k_transpose_plr<double>, dim3(grid1(M)), dim3(256), 0, s, (const double*)x,
                       (double*)xt, ml, mr, mp);
  else
    hipLaunchKernelGGL(k_transpose_plr<float>, dim3(grid1(M)), dim3(256), 0, s, (const float*)x,
                       (float*)xt, ml, mr, mp);
  return hipGetLastError();
}

hipError_t launch_convert(int dtype, const CVTask* tasks, int ntask, int64_t maxn, hipStream_t s) {
  if (ntask == 0) return hipSuccess;
  int64_t g = grid1(maxn);
  if (g > 1024) g = 1024;
  (void)dtype;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)g, ntask), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

hipError_t launch_cast(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t n,
                       hipStream_t s) {
  int64_t g = grid1(n);
  if (g > 2048) g = 2048;
  if (g == 0) return hipSuccess;
  if (src_dtype == 0 && dst_dtype == 1)
    hipLaunchKernelGGL((k_cast<double, float>), dim3((unsigned)g), dim3(256), 0, s,
                       (const double*)src, (float*)dst, n);
  else if (src_dtype == 1 && dst_dtype == 0)
    hipLaunchKernelGGL((k_cast<float, double>), dim3((unsigned)g), dim3(256), 0, s,
                       (const float*)src, (double*)dst, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

static inline unsigned gridv(int64_t n) {
  int64_t g = grid1(n);
  return (unsigned)(g > 1024 ? 1024 : (g < 1 ? 1 : g));
}

hipError_t launch_kinit(const KJob* jobs, int nj, int kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_kinit, dim3(1, nj), dim3(256), 0, s, jobs, kmax);
  return hipGetLastError();
}

hipError_t launch_knorm(const KJob* jobs, int nj, hipStream_t s) {
  hipLaunchKernelGGL(k_knorm, dim3(kRedBlocks, nj), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_kscale(const KJob* jobs, int nj, int64_t nmax, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_kscale, dim3(gridv(nmax), nj), dim3(256), 0, s, jobs, mode);
  return hipGetLastError();
}


hipError_t launch_kalpha(const KJob* jobs, int nj, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_kalpha, dim3(1, nj), dim3(256), 0, s, jobs, j);
  return hipGetLastError();
}

hipError_t launch_kdots(const KJob* jobs, int nj, int i0, int nv, int pin, hipStream_t s) {
  hipLaunchKernelGGL(k_kdots, dim3(kRedBlocks, nj), dim3(kDotThreads), 0, s, jobs, i0, nv, pin);
  return hipGetLastError();
}

hipError_t launch_reduce_dots(const RDSrc* srcs, int nsrc, const KJob* job, int ml, int mr, int mp, int i0,
                              int nv, int pin, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_dots, dim3(kRedBlocks), dim3(kDotThreads), 0, s, srcs, nsrc, job, ml, mr, mp, i0,
                     nv, pin);
  return hipGetLastError();
}

hipError_t launch_kortho(const KJob* jobs, int nj, int j, int pin, int norm_only, int set_alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_kortho, dim3(kRedBlocks, nj), dim3(256), 0, s, jobs, j, pin, norm_only, set_alpha);
  return hipGetLastError();
}

hipError_t launch_kbeta(const KJob* jobs, int nj, int j, int64_t nmax, hipStream_t s) {
  hipLaunchKernelGGL(k_kbeta, dim3(gridv(nmax), nj), dim3(256), 0, s, jobs, j);
  return hipGetLastError();
}

hipError_t launch_ktridiag(const KJob* jobs, int nj, hipStream_t s) {
  hipLaunchKernelGGL(k_ktridiag, dim3(1, nj), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_kritz(const KJob* jobs, int nj, hipStream_t s) {
  hipLaunchKernelGGL(k_kritz, dim3(kRedBlocks, nj), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_tiny(const TJob* jobs, int nj, int minM, int maxM, int kreq, hipStream_t s) {
  if (maxM > 1024 || minM < 1 || minM > maxM) return hipErrorInvalidValue;
  // blocks for the most entries x parts of any job size in [minM, maxM]
  int64_t ablocks = 0;
  for (int64_t m : {(int64_t)minM, (int64_t)maxM, std::min<int64_t>(maxM, 255)})
    if (m >= minM && m <= maxM) ablocks = std::max<int64_t>(ablocks, (m * m * tiny_assemble_parts((int)m) + 255) / 256);
  hipLaunchKernelGGL(k_tiny_assemble, dim3((unsigned)ablocks, nj), dim3(256), 0, s, jobs);
  if (minM <= kTinyWaveM)
    hipLaunchKernelGGL(k_tiny_lanczos_wave, dim3(nj), dim3(64), (size_t)kTinyWaveLds, s, jobs, kreq);
  if (maxM > kTinyWaveM) {
    // jobs whose basis fits in LDS run in the first form, the others in the second
    const int64_t cap = (int64_t)kTinyLdsMax - kTinyBlockFixed;
    const int64_t need = tiny_basis_bytes(maxM, kreq);
    hipLaunchKernelGGL(k_tiny_lanczos_block<true>, dim3(nj), dim3(1024),
                       (size_t)(kTinyBlockFixed + (need < cap ? need : cap)), s, jobs, kreq);
    if (need > cap)
      hipLaunchKernelGGL(k_tiny_lanczos_block<false>, dim3(nj), dim3(1024), (size_t)kTinyBlockFixed, s, jobs, kreq);
  }
  return hipGetLastError();
}

hipError_t launch_chol_inv(const double* G, int n, double* R, double* RinvRow, int shift_mode,
                           int64_t rows, KrylovState* st, double* ws, hipStream_t s) {
  switch (n) {
    case 16: hipLaunchKernelGGL(k_chol_inv_blk<16>, dim3(1), dim3(64), 0, s, G, R, RinvRow, shift_mode, rows, st); return hipGetLastError();
    case 32: hipLaunchKernelGGL(k_chol_inv_blk<32>, dim3(1), dim3(64), 0, s, G, R, RinvRow, shift_mode, rows, st); return hipGetLastError();
    case 48: hipLaunchKernelGGL(k_chol_inv_blk<48>, dim3(1), dim3(64), 0, s, G, R, RinvRow, shift_mode, rows, st); return hipGetLastError();
    case 64: hipLaunchKernelGGL(k_chol_inv_blk<64>, dim3(1), dim3(64), 0, s, G, R, RinvRow, shift_mode, rows, st); return hipGetLastError();
    default: break;
  }
  if (n <= 128) {
    hipLaunchKernelGGL(k_chol_inv<false>, dim3(1), dim3(256), (size_t)n * (n + 1) * sizeof(double), s, G,
                       n, R, RinvRow, shift_mode, rows, st, nullptr);
    return hipGetLastError();
  }
  if (!ws) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_inv<true>, dim3(1), dim3(256), 0, s, G, n, R, RinvRow, shift_mode, rows, st, ws);
  return hipGetLastError();
}

hipError_t launch_qr_small(double* T, int d0, int d1, int d2, int j, double* Rout, KrylovState* st,
                           hipStream_t s) {
  const size_t lds = (size_t)d0 * d1 * d2 * sizeof(double);
  hipLaunchKernelGGL(k_qr_small, dim3(1), dim3(256), lds, s, T, d0, d1, d2, j, Rout, st);
  return hipGetLastError();
}

hipError_t launch_small_matmul(const double* A, const double* B, double* C, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_small_matmul, dim3((unsigned)((n * n + 63) / 64)), dim3(64), 0, s, A, B, C, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- mixed-shape launchers
hipError_t launch_batch_mode(int dtype, const MPTask* tasks, const MPJob* jobs, const int2* wus, int nwu,
                             size_t lds, hipStream_t s) {
  if (nwu == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_batch_mode<double>, dim3(nwu), dim3(256), lds, s, tasks, jobs, wus);
  else
    hipLaunchKernelGGL(k_batch_mode<float>, dim3(nwu), dim3(256), lds, s, tasks, jobs, wus);
  return hipGetLastError();
}

hipError_t launch_transpose_list(int dtype, const TRTask* tasks, int ntask, int64_t maxM, hipStream_t s) {
  if (ntask == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_transpose_list<double>, dim3(gridv(maxM), ntask), dim3(256), 0, s, tasks);
  else
    hipLaunchKernelGGL(k_transpose_list<float>, dim3(gridv(maxM), ntask), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

hipError_t launch_reduce_list(int dtype_in, const RDTask* tasks, int ntask, int64_t maxM, hipStream_t s) {
  if (ntask == 0) return hipSuccess;
  if (dtype_in == 0)
    hipLaunchKernelGGL((k_reduce_list<double, double>), dim3(gridv(maxM), ntask), dim3(256), 0, s, tasks);
  else
    hipLaunchKernelGGL((k_reduce_list<float, double>), dim3(gridv(maxM), ntask), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

__global__ void k_zero_int(int* __restrict__ p, int n) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0;
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(gridv(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(gridv(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of every kernel that uses it (call before any
// stream capture: attribute changes are not stream operations).
hipError_t prepare_kernel_attributes() {
  if (hipError_t e = prepare_sandwich_attributes()) return e;
  const void* fns[] = {
      (const void*)k_batch_mode<double>, (const void*)k_batch_mode<float>,
      (const void*)k_mode<double, 1, mode_qs(1)>, (const void*)k_mode<double, 2, mode_qs(2)>,
      (const void*)k_mode<double, 3, mode_qs(3)>, (const void*)k_mode<double, 4, mode_qs(4)>,
      (const void*)k_mode<double, 5, mode_qs(5)>, (const void*)k_mode<double, 6, mode_qs(6)>,
      (const void*)k_mode<double, 7, mode_qs(7)>, (const void*)k_mode<double, 8, mode_qs(8)>,
      (const void*)k_mode<float, 1, mode_qs(1)>, (const void*)k_mode<float, 2, mode_qs(2)>,
      (const void*)k_mode<float, 3, mode_qs(3)>, (const void*)k_mode<float, 4, mode_qs(4)>,
      (const void*)k_mode<float, 5, mode_qs(5)>, (const void*)k_mode<float, 6, mode_qs(6)>,
      (const void*)k_mode<float, 7, mode_qs(7)>, (const void*)k_mode<float, 8, mode_qs(8)>, (const void*)k_mlp_grad};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  // the LDS form of the Cholesky kernel keeps n (n + 1) doubles: 74 KiB at n = 96, 129 KiB at n = 128
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_inv<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     128 * 129 * (int)sizeof(double));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_tiny_lanczos_wave, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kTinyWaveLds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_tiny_lanczos_block<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kTinyLdsMax);
}

// ---------------------------------------------------------------- Davidson launchers
hipError_t launch_heff_diag(const TinyPlan* plan, const DJob* job, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_heff_diag, dim3(kRedBlocks), dim3(256), 0, s, plan, job);
  (void)n;
  return hipGetLastError();
}
hipError_t launch_dav(int op, const DJob* job, int k, int arg, double tol, hipStream_t s) {
  switch (op) {
    case 0: hipLaunchKernelGGL(k_dav_init, dim3(1), dim3(256), 0, s, job); break;
    case 1: hipLaunchKernelGGL(k_dav_start, dim3(kRedBlocks), dim3(256), 0, s, job, arg); break;
    case 2: hipLaunchKernelGGL(k_dav_dots, dim3(kRedBlocks), dim3(256), 0, s, job, k); break;
    case 3: hipLaunchKernelGGL(k_dav_eig, dim3(1), dim3(256), 0, s, job, k); break;
    case 4: hipLaunchKernelGGL(k_dav_resid, dim3(kRedBlocks), dim3(256), 0, s, job, k); break;
    case 5: hipLaunchKernelGGL(k_dav_jacobi, dim3(kRedBlocks), dim3(256), 0, s, job, k, tol); break;
    case 6: hipLaunchKernelGGL(k_dav_learned, dim3(kRedBlocks), dim3(256), 0, s, job, k, tol); break;
    case 7: hipLaunchKernelGGL(k_dav_check, dim3(1), dim3(256), 0, s, job); break;
    case 8: hipLaunchKernelGGL(k_dav_ortho, dim3(kRedBlocks), dim3(256), 0, s, job, k, arg, 0); break;
    case 9: hipLaunchKernelGGL(k_dav_ortho, dim3(kRedBlocks), dim3(256), 0, s, job, k, arg, 1); break;
    case 10: hipLaunchKernelGGL(k_dav_append, dim3(kRedBlocks), dim3(256), 0, s, job, arg); break;
    case 11: hipLaunchKernelGGL(k_dav_restart, dim3(kRedBlocks), dim3(256), 0, s, job, k, arg); break;
    case 12: hipLaunchKernelGGL(k_dav_final, dim3(kRedBlocks), dim3(256), 0, s, job); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_to_half(const float* src, void* dst, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_half, dim3((n + 255) / 256), dim3(256), 0, s, src, (_Float16*)dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- correction model launchers
size_t mlp_grad_lds() { return (size_t)(6 * 64 * (kMlpHidden + 1) + 64 * 3 + 64 + 64) * sizeof(float); }

hipError_t launch_mlp_train_step(float* w, const float* feats, const float* targets, int64_t off, int batch,
                                 float* gpart, float* grad, float* m, float* v, int step, float lr, float* loss,
                                 hipStream_t s) {
  const int nblk = batch / 64;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(64), mlp_grad_lds(), s, w, feats, targets, off, batch, gpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, gpart, nblk, grad);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, w, grad, m, v, step, lr, batch,
                     loss);
  return hipGetLastError();
}

hipError_t launch_mlp_eval(const void* w16, const float* feats, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_eval, dim3(gridv(n)), dim3(256), 0, s, (const _Float16*)w16, feats, out, n);
  return hipGetLastError();
}

hipError_t launch_vdot(const double* a, const double* b, int64_t n, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_vdot, dim3(kRedBlocks), dim3(256), 0, s, a, b, n, partial);
  return hipGetLastError();
}

hipError_t launch_axpby(double alpha, const double* x, double beta, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(gridv(n)), dim3(256), 0, s, alpha, x, beta, y, n);
  return hipGetLastError();
}

hipError_t launch_harvest_write(const double* diag, const double* r, const double* x, double theta, double sc,
                                double rinf, float* feats, float* targets, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_harvest_write, dim3(gridv(n)), dim3(256), 0, s, diag, r, x, theta, sc, rinf, feats,
                     targets, n);
  return hipGetLastError();
}

}  // namespace attn

// ---------------------------------------------------------------- allocation-free model training
// attn_mlp_train_noalloc: attn_mlp_train with its working memory (parameters,
// Adam moments, gradient, per-workgroup gradient partial sums, per-step
// losses) in a fixed file-scope device array instead of hipMalloc'ed buffers.
// Each device the library runs on holds its own copy of the array until the
// process ends; the host takes the array's device address once per device
// with hipGetSymbolAddress and uses only that address afterwards.
#include <mutex>

#include "attn.h"

namespace {
constexpr size_t kNaAlign = 256;
constexpr size_t na_round(size_t b) { return (b + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr int kNaMaxBatch = 16384;    // points per Adam step
constexpr int kNaMaxSteps = 65536;    // Adam steps per call
constexpr size_t kNaParamBytes = na_round((size_t)attn::kMlpParams * sizeof(float));
constexpr size_t kNaGradBytes = na_round((size_t)(attn::kMlpParams + 1) * sizeof(float));
constexpr size_t kNaPartBytes = na_round((size_t)(kNaMaxBatch / 64) * (attn::kMlpParams + 1) * sizeof(float));
constexpr size_t kNaLossBytes = na_round((size_t)kNaMaxSteps * sizeof(float));
// w, m, v, grad, gpart, loss
constexpr size_t kNaScratchBytes = 3 * kNaParamBytes + kNaGradBytes + kNaPartBytes + kNaLossBytes;
constexpr int kNaMaxDevices = 64;

std::mutex g_na_mu;
void* g_na_ptr[kNaMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

extern "C" attn_status attn_mlp_train_noalloc(const float* feats, const float* targets, int64_t n, int32_t steps,
                                              int32_t batch, float lr, float* params, float* loss, void* stream) {
  using namespace attn;
  if (!feats || !targets || !params || steps < 1 || batch < 64 || batch % 64 || n < batch) return ATTN_ERR_ARG;
  if (batch > kNaMaxBatch || steps > kNaMaxSteps) return ATTN_ERR_UNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return ATTN_ERR_HIP;
  if (dev < 0 || dev >= kNaMaxDevices) return ATTN_ERR_UNSUPPORTED;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ATTN_ERR_HIP;
      g_na_ptr[dev] = p;
    }
    base = (unsigned char*)g_na_ptr[dev];
  }
  float* w = (float*)base;
  float* m = (float*)(base + kNaParamBytes);
  float* v = (float*)(base + 2 * kNaParamBytes);
  float* grad = (float*)(base + 3 * kNaParamBytes);
  float* gpart = (float*)(base + 3 * kNaParamBytes + kNaGradBytes);
  float* dl = (float*)(base + 3 * kNaParamBytes + kNaGradBytes + kNaPartBytes);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = prepare_kernel_attributes();
  // the array keeps the previous call's contents: the moments start at zero
  if (e == hipSuccess) e = hipMemcpyAsync(w, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(m, 0, 2 * kNaParamBytes, s);
  const int64_t nb = n / batch;
  for (int st = 1; st <= steps && e == hipSuccess; st++) {
    const int64_t off = ((st - 1) % nb) * batch;
    e = launch_mlp_train_step(w, feats, targets, off, batch, gpart, grad, m, v, st, lr, dl, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(params, w, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, dl, steps * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? ATTN_OK : ATTN_ERR_HIP;
}
