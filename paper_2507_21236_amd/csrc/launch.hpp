// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "kernels.hpp"

namespace attn {

// Lanczos / QR scalar state kept on the device (no host round trip per step).
struct KrylovState {
  double alpha[128];
  double beta[128];
  double h[128];
  double y[128];      // eigenvector of the tridiagonal matrix
  double scal[8];     // [0] = theta, [1] = norm scratch, [2] = shift
  int32_t kmax;       // number of matvecs requested
  int32_t keff;       // number of Lanczos vectors kept
  int32_t stop;       // breakdown reached
  int32_t status;     // 0 ok, 1 non-finite, 2 factorisation breakdown
};

// Reduction scratch: per vector, per block partial sums.
constexpr int kRedBlocks = 256;

hipError_t launch_sandwich(int dtype, int ma, int mb, const SWTask* tasks, const SWItem* items,
                           const int4* wus, int nwu, const void* xbase, hipStream_t s);
hipError_t launch_mode(int dtype, int mj, bool mfma, const MPTask* tasks, const MPJob* jobs,
                       const int2* wus, int nwu, const void* xbase, hipStream_t s);
hipError_t launch_gram(int mj, bool mfma, const GRTask* tasks, int ntask, hipStream_t s);
hipError_t launch_gram_reduce(const GRReduce* r, int nr, int maxm, hipStream_t s);
hipError_t launch_combine(const CBTask* tasks, const CBTerm* terms, int ntask, int maxn,
                          hipStream_t s);
hipError_t launch_reduce_out(int dtype_in, const RDSrc* srcs, int nsrc, void* y, int dtype_out,
                             int ml, int mr, int mp, hipStream_t s);
hipError_t launch_transpose_plr(int dtype, const void* x, void* xt, int ml, int mr, int mp,
                                hipStream_t s);
hipError_t launch_convert(int dtype, const CVTask* tasks, int ntask, int64_t maxn, hipStream_t s);
hipError_t launch_cast(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t n,
                       hipStream_t s);

// Krylov helpers (all FP64).  Vectors are length n, V is row-major [nv][n].
hipError_t launch_multidot(const double* V, int nv, const double* w, int64_t n, double* partial,
                           const KrylovState* st, hipStream_t s);
hipError_t launch_dot_final(const double* partial, int nv, double* out, int mode,
                            KrylovState* st, int j, hipStream_t s);
hipError_t launch_lanczos_update(double* w, const double* V, int64_t n, KrylovState* st, int j,
                                 double* partial, hipStream_t s);
hipError_t launch_axpy_dots(double* w, const double* V, int nv, int64_t n, KrylovState* st,
                            double* partial, int norm_only, hipStream_t s);
hipError_t launch_scale_into(const double* w, double* out, int64_t n, KrylovState* st, int which,
                             int j, hipStream_t s);
hipError_t launch_tridiag(KrylovState* st, hipStream_t s);
hipError_t launch_tiny_lanczos(const TinyPlan* plan, int M, double* H, double* T, double* V,
                               double* w, KrylovState* st, int k, hipStream_t s);
hipError_t launch_ritz(const double* V, int64_t n, double* out, KrylovState* st, double* partial,
                       hipStream_t s);
hipError_t launch_normalize(double* x, int64_t n, double* partial, KrylovState* st, hipStream_t s);
hipError_t launch_norm2(const double* x, int64_t n, double* partial, hipStream_t s);

hipError_t launch_state_init(KrylovState* st, int kmax, hipStream_t s);
hipError_t launch_lanczos_update2(double* w, const double* V, int64_t n, KrylovState* st, int j,
                                  const double* partial_a, double* partial, hipStream_t s);
hipError_t launch_axpy_dots2(double* w, const double* V, int nv, int64_t n, KrylovState* st,
                             const double* partial_in, double* partial, int norm_only,
                             hipStream_t s);
hipError_t launch_scale_beta(const double* w, double* out, int64_t n, KrylovState* st, int j,
                             const double* partial, hipStream_t s);
hipError_t launch_scale_norm(const double* x, double* out, int64_t n, const double* partial,
                             KrylovState* st, hipStream_t s);

// QR helpers
hipError_t launch_chol_inv(const double* G, int n, double* R, double* RinvRow, int shift_mode,
                           int64_t rows, KrylovState* st, hipStream_t s);
hipError_t launch_qr_small(double* T, int d0, int d1, int d2, int j, double* Rout, KrylovState* st,
                           hipStream_t s);
hipError_t launch_small_matmul(const double* A, const double* B, double* C, int n, hipStream_t s);

}  // namespace attn
