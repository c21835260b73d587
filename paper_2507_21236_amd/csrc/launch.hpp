// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "kernels.hpp"

namespace attn {

// Reduction scratch: per vector, per block partial sums.
constexpr int kRedBlocks = 256;

// outs (MFMA shapes only): tasks with pad = 1 write several outputs, items of
// output o = outs[task.item0 + k] going to its own y
hipError_t launch_sandwich(int dtype, int ma, int mb, const SWTask* tasks, const SWItem* items,
                           const int4* wus, int nwu, const void* xbase, hipStream_t s,
                           const SWOut* outs = nullptr);
// nt: every task has j in {0, 1} and 16 | d2 (register-direct kernel, m_j <= 64)
hipError_t launch_mode(int dtype, int mj, bool mfma, const MPTask* tasks, const MPJob* jobs,
                       const int2* wus, int nwu, const void* xbase, hipStream_t s, bool nt = false);
// nt: every task has j in {0, 1}, 16 | d2 and 16-aligned free ranges (register-direct kernel, mj <= 64)
hipError_t launch_gram(int mj, bool mfma, const GRTask* tasks, int ntask, hipStream_t s, bool nt = false);
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
hipError_t launch_kalpha(const KJob* jobs, int nj, int j, hipStream_t s);
// partial dots of basis vectors [i0, i0 + nv) with w into partial-sum area pin
hipError_t launch_kdots(const KJob* jobs, int nj, int i0, int nv, int pin, hipStream_t s);
// w = sum of a product's partial outputs, then launch_kdots' partial dots (one job)
hipError_t launch_reduce_dots(const RDSrc* srcs, int nsrc, const KJob* job, int ml, int mr, int mp, int i0,
                              int nv, int pin, hipStream_t s);
hipError_t launch_kortho(const KJob* jobs, int nj, int j, int pin, int norm_only, int set_alpha, hipStream_t s);
hipError_t launch_kbeta(const KJob* jobs, int nj, int j, int64_t nmax, hipStream_t s);
hipError_t launch_ktridiag(const KJob* jobs, int nj, hipStream_t s);
hipError_t launch_kritz(const KJob* jobs, int nj, hipStream_t s);
hipError_t launch_tiny(const TJob* jobs, int nj, int minM, int maxM, int kreq, hipStream_t s);

// Mixed-shape launches over the tasks of several nodes / problem instances
// (LDS in bytes: the largest any unit of the launch needs).
hipError_t launch_batch_sandwich(int dtype, const SWTask* tasks, const SWItem* items, const int4* wus,
                                 int nwu, size_t lds, hipStream_t s);
// One persistent launch of a whole batched matvec (grid workgroups; the
// counters of a.cnt must be zero, and are zero again when it ends).
hipError_t launch_batch_matvec(int dtype, const PMArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t batch_matvec_occupancy(int dtype, size_t lds, int* per_cu);
hipError_t launch_batch_mode(int dtype, const MPTask* tasks, const MPJob* jobs, const int2* wus, int nwu,
                             size_t lds, hipStream_t s);
hipError_t launch_transpose_list(int dtype, const TRTask* tasks, int ntask, int64_t maxM, hipStream_t s);
hipError_t launch_reduce_list(int dtype_in, const RDTask* tasks, int ntask, int64_t maxM, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
// dst = src (n doubles; the ranges do not overlap)
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
hipError_t prepare_kernel_attributes();
hipError_t prepare_sandwich_attributes();

// Davidson form.  op: 0 init, 1 start (arg = phase 0/1), 2 dots of W[k-1],
// 3 Rayleigh-Ritz (Jacobi eigensolver), 4 Ritz vector and residual, 5 Jacobi
// correction, 6 learned correction, 7 correction check, 8/9 Gram-Schmidt pass
// (arg = input area; 9 = last pass), 10 append (arg = slot), 11 restart
// (arg = vectors kept), 12 final Ritz vector into T.
hipError_t launch_heff_diag(const TinyPlan* plan, const DJob* job, int64_t n, hipStream_t s);
hipError_t launch_dav(int op, const DJob* job, int k, int arg, double tol, hipStream_t s);
hipError_t launch_to_half(const float* src, void* dst, int n, hipStream_t s);

// Correction model: one Adam training step on batch points [off, off + batch)
// (batch a multiple of 64; gpart: batch / 64 x (kMlpParams + 1) floats,
// grad: kMlpParams + 1); inference on given features; small vector kernels of
// the exact-correction solver.
hipError_t launch_mlp_train_step(float* w, const float* feats, const float* targets, int64_t off, int batch,
                                 float* gpart, float* grad, float* m, float* v, int step, float lr, float* loss,
                                 hipStream_t s);
hipError_t launch_mlp_eval(const void* w16, const float* feats, float* out, int64_t n, hipStream_t s);
hipError_t launch_vdot(const double* a, const double* b, int64_t n, double* partial, hipStream_t s);
hipError_t launch_axpby(double alpha, const double* x, double beta, double* y, int64_t n, hipStream_t s);
hipError_t launch_harvest_write(const double* diag, const double* r, const double* x, double theta, double sc,
                                double rinf, float* feats, float* targets, int64_t n, hipStream_t s);

// QR helpers.  ws: n (n + 1) doubles of device workspace, used (and required)
// when n > 128
hipError_t launch_chol_inv(const double* G, int n, double* R, double* RinvRow, int shift_mode,
                           int64_t rows, KrylovState* st, double* ws, hipStream_t s);
hipError_t launch_qr_small(double* T, int d0, int d1, int d2, int j, double* Rout, KrylovState* st,
                           hipStream_t s);
hipError_t launch_small_matmul(const double* A, const double* B, double* C, int n, hipStream_t s);

}  // namespace attn
