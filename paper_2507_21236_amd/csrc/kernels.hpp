// Work descriptors shared by the host runtime and the gfx950 kernels.
//
// Every kernel is driven by a device-resident list of work units so that one
// launch can cover many terms, output blocks or problem instances of uneven
// size.  All operator blocks are m x m, stored column-major: element O[i][i']
// (acting as (O x_j v)[.., i, ..] = sum_i' O[i][i'] v[.., i', ..]) lives at
// O + i' * m + i.  Tensors are row-major [d0][d1][d2].
#pragma once
#include <stdint.h>

namespace attn {

// ---------------------------------------------------------------- sandwich
// Y_s (+)= sum_items coef * A X_s B^T over slices s of a spectator leg:
// X_s[a][b] at x + s*xs_slice + a*xs_row + b (same for y).  A acts on the
// a leg (ma x ma), B on the b leg (mb x mb).
struct SWItem {
  const void* A;
  const void* B;
  double coef;
};

struct SWTask {
  const void* x;
  void* y;
  int64_t xs_slice, xs_row;
  int64_t ys_slice, ys_row;
  int32_t ma, mb;
  int32_t item0, nitem;   // items, or (pad = 1) outputs
  int32_t accumulate;
  int32_t pad;            // 1: several outputs per task (SWOut list)
};

// One output of a several-output task: items [item0, item0 + nitem) -> y (same geometry).
struct SWOut {
  void* y;
  int32_t item0, nitem;
};

// ---------------------------------------------------------------- mode product
// out (+)= sum_jobs coef * A x_j in, all tensors of dims (d0, d1, d2).
struct MPJob {
  const void* A;
  const void* in;
  double coef;
};

struct MPTask {
  void* out;
  int32_t d0, d1, d2, j;
  int32_t job0, njob;
  int32_t accumulate;
  int32_t pad;
};

// ---------------------------------------------------------------- gram
// partial[o][c] = sum_{f in chunk c} X[f][j] Z_o[f][j'] with f the two legs
// other than j of a (d0, d1, d2) tensor; reduced afterwards over c.
struct GRTask {
  const void* X;
  const void* Z;
  void* partial;      // m_j x m_j, column-major
  int32_t d0, d1, d2, j;
  int32_t f0, f1;     // free-index range of this unit
};

// Final block = coef * sum over npart partials (fixed order) (+ existing if accumulate)
struct GRReduce {
  const void* partial;   // npart consecutive m*m partials
  void* out;
  int32_t m, npart;
  double coef;
  int32_t accumulate;
  int32_t pad;
};

// ---------------------------------------------------------------- block combine
// out = sum_k coef_k * in_k (blocks of n elements)
struct CBTerm {
  const void* in;
  double coef;
};
struct CBTask {
  void* out;
  int32_t n, term0, nterm;
  int32_t pad;
};

// ---------------------------------------------------------------- reduction of partial outputs
// y[l][r][p] = sum_k src_k, src_k in layout 0 ([l][r][p]) or 1 ([p][l][r])
// LDS bytes of the slice form of the generic sandwich (slice, stage-1
// product and one item's blocks), or 0 where the per-element form is used
// (more than 256 entries per slice, or more than 32 KiB).  The work units of
// a generic group are one per 256 entries of a slice either way.
constexpr size_t gen_slice_lds(int ma, int mb, size_t esz) {
  return (ma * mb <= 256 && (size_t)(2 * ma * mb + ma * ma + mb * mb) * esz <= 32768)
             ? (size_t)(2 * ma * mb + ma * ma + mb * mb) * esz
             : 0;
}

struct RDSrc {
  const void* p;
  int32_t layout;
  int32_t pad;
};

// list forms (one task per tensor, several problem instances per launch)
struct RDTask {
  const RDSrc* srcs;
  void* y;             // FP64
  int32_t nsrc, ml, mr, mp;
};
struct TRTask {        // [l][r][p] -> [p][l][r]
  const void* x;
  void* xt;
  int32_t ml, mr, mp, pad;
};

// ---------------------------------------------------------------- persistent batched matvec
// One launch runs a whole matvec of several problem instances: a resident
// grid of workgroups takes units from one ordered work list by ticket.  The
// tickets are dealt to kPmQueues queues (ticket t to queue t mod kPmQueues,
// workgroup b takes from queue b mod kPmQueues, one atomic counter per queue),
// so that no single counter serialises every grab.  A unit may wait for a
// counter of units that come before it in the list (per instance:
// transposes before the sandwiches that read the transposed input, each chain
// stage before the next, every partial output before the reduction).  The
// launch cannot deadlock: each queue hands out its tickets in list order, so
// the earliest unfinished unit is either held by a running workgroup (and
// everything it waits for is earlier, hence finished) or is next in its
// queue, whose workgroups are then all free to take it.  One ticket covers a
// run of consecutive units with the same wait and signal, so that the ticket
// atomic and the device-scope release and acquire are paid once per run.
enum { PU_TRANSPOSE = 0, PU_MODE = 1, PU_SANDWICH = 2, PU_REDUCE = 3 };

struct PUnit {
  int32_t kind;     // PU_*
  int32_t a, b, c, d;
  // transpose / reduce: a = task, b = first element (kPmTileT / kPmTileR elements)
  // mode: a = chain stage, b = task of that stage, c = free tile or first element
  // sandwich: (a, b, c, d) = (task, slice, first 16-row strip, body)
  int32_t wait;     // counter that must reach `need` before the unit runs, or -1
  int32_t need;
  int32_t signal;   // counter incremented once the unit's results are visible, or -1
};

constexpr int kPmQueues = 8;              // ticket queues (counters 0 .. 7)
constexpr int kPmExit = kPmQueues;        // counter: workgroups that have left the loop
constexpr int kPmFirst = kPmQueues + 1;   // first dependency counter
constexpr int kPmStride = 32;             // ints between counters: one 128-byte line each
constexpr int kPmTileT = 2048;            // elements per transpose unit
constexpr int kPmTileR = 256;             // elements per reduction unit (one per lane: each sums every source)
// Spin limit of one wait: about a second; past it the launch sets its abort
// word, skips every unit that still has to wait, and ends.
constexpr int kPmSpin = 1 << 20;
constexpr int kPmMaxLds = 64 * 1024;   // dynamic LDS limit of the persistent launch
constexpr int kPmDefer = 4;             // tickets a workgroup may finish before publishing their count

struct PMArgs {
  const PUnit* units;
  const int32_t* tickets;   // [n_tickets + 1]: first unit of each ticket
  int32_t n_tickets;
  int32_t n_units;
  int32_t n_cnt;      // counters (queues, exit, dependencies); the last workgroup out zeroes them
  int32_t* cnt;       // counter c at cnt[c * kPmStride]
  int32_t* abort;     // sticky: a wait exceeded its limit
  const SWTask* sw_tasks;
  const SWItem* sw_items;
  const MPTask* mp_tasks[3];
  const MPJob* mp_jobs[3];
  const TRTask* tr;
  const RDTask* rd;
};

// ---------------------------------------------------------------- conversion
// fmt 1: FP64 -> FP32, same (column-major) layout.
// fmt 2: FP64 -> split BF16 (x = hi + lo up to ~2^-17 |x|) for m x m blocks,
//        m a multiple of 32: per block, the hi plane then the lo plane, each
//        row-major with the columns of every 32-wide chunk permuted into the
//        order in which the BF16 matrix-core kernels walk their K index.
struct CVTask {
  const double* src;
  void* dst;
  int64_t n;       // elements
  int32_t m;       // block dimension (fmt 2)
  int32_t fmt;
};

// ---------------------------------------------------------------- Krylov
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
  int32_t sticky;     // OR of every nonzero status set since it was last cleared
  int32_t pad;
};

// One Lanczos eigensolve (one node of one problem instance).
struct KJob {
  double* V;          // Krylov basis, row-major [k + 1][n]
  double* w;          // matvec output / residual
  double* T;          // node tensor: start vector in, normalised Ritz vector out
  double* red;        // four partial-sum areas P0..P3 of 64 x 256 values
  KrylovState* st;
  double* x64;        // optional copy of the newest basis vector (FP64)
  float* x32;         // optional copy of the newest basis vector (FP32)
  int64_t n;
};

// ---------------------------------------------------------------- tiny nodes
// Whole matvec plan of a node whose contractions all use the generic kernels,
// executed inside one workgroup (the tiny-node Lanczos kernels).
// Three-operator product item (one operator per leg) of a three-leg term.
struct Item3 {
  const void* op[3];
  double coef;
};

struct TinyPlan {
  const SWItem* items;  // two-leg terms and local operators, grouped by spectator
  const Item3* items3;  // three-leg terms expanded into products
  int32_t item0[3], nitem[3];
  int32_t n3;
  int32_t d0, d1, d2;
};

// Dense eigensolve of one tiny node: H (M x M scratch), basis V, residual w.
struct TJob {
  const TinyPlan* plan;
  double* H;
  double* T;
  double* V;
  double* w;
  KrylovState* st;
  int32_t M, pad;
};

// ---------------------------------------------------------------- Davidson form
constexpr int kDavMax = 32;          // largest basis
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 3 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1;   // 8641

// Davidson scalar state (device).  G and Y are column-major with leading dimension kDavMax.
struct DavState {
  double G[kDavMax * kDavMax];   // V^T H V
  double Y[kDavMax * kDavMax];   // its eigenvectors, columns by ascending eigenvalue
  double ev[kDavMax];
  double theta, rnorm, rinf, dinf, tnorm2;
  int32_t converged;             // ||r|| <= tol
  int32_t tbad;                  // correction not finite
  int32_t status;                // 1 non-finite, 2 breakdown
  int32_t pad;
};

// One Davidson eigensolve.  red holds 8 partial-sum areas of kDavMax x 256 values.
struct DJob {
  double* V;          // basis [kDavMax][n]
  double* W;          // H V  [kDavMax][n]
  double* Vt;         // restart scratch [2 * restart][n]
  double* u;          // Ritz vector
  double* r;          // residual
  double* t;          // correction
  double* diag;       // diag(H_eff)
  double* T;          // node tensor (start vector in, Ritz vector out)
  double* red;
  DavState* ds;
  const void* mlp;    // FP16 parameters of the correction model (learned mode)
  int64_t n;
};

}  // namespace attn
