// Kernels of the observable and disentangler-environment contractions: FP64
// matrix products over a work list (the contractions of an operator image
// through a tree node, the link Gram matrices, the closing products at the
// lowest common node), leg permutations and fixed-order sums of partials.
#include <hip/hip_runtime.h>

#include "measure.hpp"

namespace attn {

// One 64 x 64 tile of C per workgroup: K walked in steps of 16 through LDS,
// each thread accumulating a 4 x 4 block in FP64 (the vector FP64 rate of the
// chip equals its FP64 matrix-core rate).
__global__ __launch_bounds__(256) void k_gemm_jobs(const GMJob* __restrict__ jobs, const int4* __restrict__ wus) {
  __shared__ double As[16][64 + 2];
  __shared__ double Bs[16][64 + 2];
  const int4 wu = wus[blockIdx.x];
  const GMJob& J = jobs[wu.x];
  const double* A = J.A + (int64_t)wu.y * J.sa;
  const double* B = J.B + (int64_t)wu.y * J.sb;
  double* C = J.C + (int64_t)wu.y * J.sc;
  const int m0 = wu.z * 64, n0 = wu.w * 64;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int c = 0; c < 4; c++) acc[r][c] = 0.0;
  for (int k0 = 0; k0 < J.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = tid + 256 * q;
      int i, k;
      if (J.ta) { k = e >> 6; i = e & 63; } else { i = e >> 4; k = e & 15; }
      const int gi = m0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < J.M && gk < J.K) v = J.ta ? A[(int64_t)gk * J.lda + gi] : A[(int64_t)gi * J.lda + gk];
      As[k][i] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = tid + 256 * q;
      int j, k;
      if (J.tb) { j = e >> 4; k = e & 15; } else { k = e >> 6; j = e & 63; }
      const int gj = n0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < J.N && gk < J.K) v = J.tb ? B[(int64_t)gj * J.ldb + gk] : B[(int64_t)gk * J.ldb + gj];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; r++) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; c++) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int gi = m0 + ty * 4 + r;
    if (gi >= J.M) continue;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int gj = n0 + tx * 4 + c;
      if (gj >= J.N) continue;
      double* p = C + (int64_t)gi * J.ldc + gj;
      *p = J.accumulate ? *p + acc[r][c] : acc[r][c];
    }
  }
}

__global__ __launch_bounds__(256) void k_permute_jobs(const PMJob* __restrict__ jobs) {
  const PMJob& J = jobs[blockIdx.y];
  const int64_t M = (int64_t)J.d0 * J.d1 * J.d2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const int64_t a = e / ((int64_t)J.d1 * J.d2);
    const int64_t rem = e - a * J.d1 * J.d2;
    const int64_t b = rem / J.d2, c = rem - b * J.d2;
    J.out[(b * J.d0 + a) * J.d2 + c] = J.in[e];
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(const SPJob* __restrict__ jobs) {
  const SPJob& J = jobs[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < J.n; e += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int q = 0; q < J.nq; q++) acc += J.in[(int64_t)q * J.stride + e];
    J.out[e] = acc;
  }
}

// one workgroup per pair: a strided pass over the two vectors, then a
// reduction across the workgroup in a fixed order
__global__ __launch_bounds__(256) void k_pair_dots(const double* __restrict__ base, const int2* __restrict__ pairs,
                                                   int64_t M, double* __restrict__ out) {
  __shared__ double red[256];
  const int2 pr = pairs[blockIdx.x];
  const double* u = base + (int64_t)pr.x * M;
  const double* v = base + (int64_t)pr.y * M;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < M; e += 256) acc = fma(u[e], v[e], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g > 1024 ? 1024 : (g < 1 ? 1 : g));
}

hipError_t launch_gemm_jobs(const GMJob* jobs, const int4* wus, int nwu, hipStream_t s) {
  if (nwu <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_jobs, dim3(nwu), dim3(256), 0, s, jobs, wus);
  return hipGetLastError();
}

hipError_t launch_permute_jobs(const PMJob* jobs, int njob, int64_t maxM, hipStream_t s) {
  if (njob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_jobs, dim3(grid_for(maxM), njob), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const SPJob* jobs, int njob, int64_t maxn, hipStream_t s) {
  if (njob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(maxn), njob), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace attn

namespace attn {
hipError_t launch_pair_dots(const double* base, const int2* pairs, int npair, int64_t M, double* out, hipStream_t s) {
  if (npair <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_dots, dim3(npair), dim3(256), 0, s, base, pairs, M, out);
  return hipGetLastError();
}
}  // namespace attn
