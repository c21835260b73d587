// Work descriptors and launchers of the observable / disentangler-environment
// kernels (measure_kernels.hip): FP64 matrix products over work lists, leg
// permutations and fixed-order sums of partial results.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace attn {

// C (+)= op(A) op(B) for one job and batch index b: A + b sa, B + b sb, C + b sc.
// Row-major operands: op(A) is M x K (ta = 0: A[i lda + k]; ta = 1: A[k lda + i]),
// op(B) is K x N (tb = 0: B[k ldb + j]; tb = 1: B[j ldb + k]); C[i ldc + j].
struct GMJob {
  const double* A;
  const double* B;
  double* C;
  int64_t sa, sb, sc;
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t ta, tb;
  int32_t accumulate, pad;
};

// out[b][a][c] = in[a][b][c] for tensors of dims (d0, d1, d2)
struct PMJob {
  const double* in;
  double* out;
  int32_t d0, d1, d2, pad;
};

// out[e] = sum_{q < nq} in[q * stride + e] for e < n (q in increasing order)
struct SPJob {
  const double* in;
  double* out;
  int64_t n, stride;
  int32_t nq, pad;
};

// work units: int4 {job, batch index, 64-row tile, 64-column tile}
hipError_t launch_gemm_jobs(const GMJob* jobs, const int4* wus, int nwu, hipStream_t s);
hipError_t launch_permute_jobs(const PMJob* jobs, int njob, int64_t maxM, hipStream_t s);
hipError_t launch_sum_parts(const SPJob* jobs, int njob, int64_t maxn, hipStream_t s);
// out[p] = sum_e base[pairs[p].x * M + e] * base[pairs[p].y * M + e] (one workgroup per pair)
hipError_t launch_pair_dots(const double* base, const int2* pairs, int npair, int64_t M, double* out, hipStream_t s);

}  // namespace attn
