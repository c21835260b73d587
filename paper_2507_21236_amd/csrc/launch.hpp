// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "kernels.hpp"

namespace attn {

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

// Krylov steps (FP64) over a list of jobs, one launch for all of them.  Each
// job reads/writes its own partial-sum areas P0..P3 (see KJob).
hipError_t launch_kinit(const KJob* jobs, int nj, int kmax, hipStream_t s);
hipError_t launch_knorm(const KJob* jobs, int nj, hipStream_t s);
hipError_t launch_kscale(const KJob* jobs, int nj, int64_t nmax, int mode, hipStream_t s);
hipError_t launch_kdot(const KJob* jobs, int nj, int j, hipStream_t s);
hipError_t launch_kalpha(const KJob* jobs, int nj, int j, hipStream_t s);
hipError_t launch_kupdate(const KJob* jobs, int nj, int j, hipStream_t s);
hipError_t launch_kortho(const KJob* jobs, int nj, int j, int pin, int norm_only, hipStream_t s);
hipError_t launch_kbeta(const KJob* jobs, int nj, int j, int64_t nmax, hipStream_t s);
hipError_t launch_ktridiag(const KJob* jobs, int nj, hipStream_t s);
hipError_t launch_kritz(const KJob* jobs, int nj, hipStream_t s);
hipError_t launch_tiny(const TJob* jobs, int nj, int maxM, int kreq, hipStream_t s);

// Mixed-shape launches over the tasks of several nodes / problem instances
// (LDS in bytes: the largest any unit of the launch needs).
hipError_t launch_batch_sandwich(int dtype, const SWTask* tasks, const SWItem* items, const int4* wus,
                                 int nwu, size_t lds, hipStream_t s);
hipError_t launch_batch_mode(int dtype, const MPTask* tasks, const MPJob* jobs, const int2* wus, int nwu,
                             size_t lds, hipStream_t s);
hipError_t launch_transpose_list(int dtype, const TRTask* tasks, int ntask, int64_t maxM, hipStream_t s);
hipError_t launch_reduce_list(int dtype_in, const RDTask* tasks, int ntask, int64_t maxM, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t prepare_kernel_attributes();

// QR helpers
hipError_t launch_chol_inv(const double* G, int n, double* R, double* RinvRow, int shift_mode,
                           int64_t rows, KrylovState* st, hipStream_t s);
hipError_t launch_qr_small(double* T, int d0, int d1, int d2, int j, double* Rout, KrylovState* st,
                           hipStream_t s);
hipError_t launch_small_matmul(const double* A, const double* B, double* C, int n, hipStream_t s);

}  // namespace attn
