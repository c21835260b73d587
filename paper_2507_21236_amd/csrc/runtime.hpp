// Internal declarations of the runtime shared by runtime.cpp (single-handle
// entry points) and batch.cpp (lock-step batches of handles): device plans,
// the handle itself and the helpers that enqueue its work.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "attn.h"
#include "kernels.hpp"
#include "launch.hpp"
#include "model.hpp"

namespace rt {
using namespace attn;


struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIPCHK(x)                                 \
  do {                                            \
    hipError_t _e = (x);                          \
    if (_e != hipSuccess) throw HipFail{_e, #x};  \
  } while (0)

struct StatusFail {
  attn_status st;
  std::string msg;
};

// A sandwich launch group: tasks with the same (ma, mb).
struct SWGroup {
  int ma = 0, mb = 0;
  int fmt = 0;        // low-precision plans: 1 = FP32 blocks, 2 = split-BF16 blocks
  double flops = 0;   // algorithmic flops of one launch
  std::vector<SWTask> tasks;
  std::vector<SWItem> items;
  std::vector<int4> wus;
  std::vector<SWOut> outs;   // tasks with several outputs
  SWTask* d_tasks = nullptr;
  SWItem* d_items = nullptr;
  int4* d_wus = nullptr;
  SWOut* d_outs = nullptr;
};

struct MPGroup {
  int mj = 0;
  bool mfma = false;
  bool nt = false;   // register-direct kernel
  std::vector<MPTask> tasks;
  std::vector<MPJob> jobs;
  std::vector<int2> wus;
  MPTask* d_tasks = nullptr;
  MPJob* d_jobs = nullptr;
  int2* d_wus = nullptr;
};

struct CBPlan {
  std::vector<CBTask> tasks;
  std::vector<CBTerm> terms;
  CBTask* d_tasks = nullptr;
  CBTerm* d_terms = nullptr;
  int maxn = 0;
};

struct GRPlan {
  int mj = 0;
  bool mfma = false;
  bool nt = false;   // register-direct gram kernel
  std::vector<GRTask> tasks;
  std::vector<GRReduce> reds;
  GRTask* d_tasks = nullptr;
  GRReduce* d_reds = nullptr;
};

struct MVDev {
  TinyPlan* d_plan = nullptr;   // every item written out (dense tiny H_eff, diagonal)
  TinyPlan* d_tiny = nullptr;   // == d_plan when the whole eigensolve runs in one workgroup
  std::vector<SWItem> tiny_items;
  int tiny_item0[3] = {0, 0, 0}, tiny_nitem[3] = {0, 0, 0};
  std::vector<Item3> tiny_items3;
  CBPlan comb;
  std::vector<SWGroup> sw;
  std::vector<MPGroup> chainA, chainB, chainC;   // one group per mj
  std::vector<RDSrc> srcs;
  RDSrc* d_srcs = nullptr;
  bool need_xt = false;
  int dims[3] = {0, 0, 0};
};

struct EnvChunk {
  std::vector<SWGroup> sw;
  GRPlan gr;
  std::vector<std::pair<double*, int64_t>> zero_blocks;
};

struct EnvDev {
  bool present = false;
  bool transpose = false;
  int dims[3] = {0, 0, 0};
  CBPlan comb;
  std::vector<EnvChunk> chunks;
  int node = -1, leg = -1, out_edge = -1, out_dir = 0;
};

// QR of a node tensor with one leg as the column index (three CholeskyQR passes)
struct QRDev {
  bool present = false;
  int mj = 0, nfc = 0, nwus = 0;
  bool gmf = false, mmf = false, gnt = false, mnt = false;
  int64_t rows = 0, Msz = 0;
  GRTask* d_gt[3] = {nullptr, nullptr, nullptr};
  GRReduce* d_gr = nullptr;
  MPTask* d_mt[3] = {nullptr, nullptr, nullptr};
  MPJob* d_mj[3] = {nullptr, nullptr, nullptr};
  int2* d_wus = nullptr;
  std::vector<GRTask> h_gt[3];
  std::vector<GRReduce> h_gr;
  MPGroup h_mp[3];   // host copies for validation
};

// T <- R x_leg T through a temporary
struct ABDev {
  bool present = false;
  int mj = 0, nwus = 0;
  bool mmf = false, mnt = false;
  int64_t Msz = 0;
  MPTask* d_mt = nullptr;
  MPJob* d_mj = nullptr;
  int2* d_wus = nullptr;
  MPGroup h_mp;   // host copy for validation
};

inline bool mode_mfma_ok(int mj, int64_t M) { return mj % 16 == 0 && mj <= 128 && (M / mj) % 64 == 0; }
inline bool gram_mfma_ok(int mj, int64_t M) { return mj % 16 == 0 && mj <= 128 && (M / mj) % 64 == 0; }

}  // namespace rt

using namespace attn;   // internal header: the runtime sources use both namespaces
using namespace rt;

// Host copy of the problem a handle was built from (every array deep-copied),
// kept for the problem hash of checkpoints and for rebuilding the rotated
// terms when the disentanglers change.
struct ProblemCopy {
  int32_t n_sites = 0, d = 0, m = 0;
  std::vector<int32_t> leaf_order, term_nsites, term_sites, de_sites;
  std::vector<double> term_ops, term_coef, de_u;
  uint32_t flags = 0;
  int32_t device = 0;
  void assign(const attn_problem* p);
  attn_problem view() const;
  // FNV-1a over everything that fixes the tree and the Hamiltonian: sizes,
  // leaf order, terms, disentangler sites and the strict flag (not the
  // disentangler matrices, which the optimisation changes, and not the device)
  uint64_t hash() const;
};

struct attn_handle {
  Model M;
  ProblemCopy prob;
  uint64_t problem_hash = 0;
  std::vector<double> sweep_energies;   // theta at the last node of every attn_sweep sweep
  std::string err;
  bool host_only = false;
  bool dryrun = false;
  bool dead = false;
  uintptr_t fake_next = (uintptr_t)1 << 40;
  std::vector<std::pair<uintptr_t, size_t>> allocs;
  int device = 0;
  std::vector<void*> owned;
  // tensors
  double* d_T = nullptr;
  std::vector<int64_t> T_off;
  std::vector<int64_t> T_len;
  // effective-operator stores per edge and direction
  std::vector<double*> store[2];
  std::vector<char> valid[2];
  std::vector<int> iso;       // per node: leg it is isometric toward, -1 = centre
  int center = -1;
  bool state_ready = false;
  // scratch
  int64_t Mmax = 0;
  int kcap = 65;   // at most 64 Krylov vectors (+1)
  double* d_V = nullptr;      // (kcap) x Mmax
  double* d_w = nullptr;
  double* d_xt = nullptr;
  double* d_tmp = nullptr;
  double* d_tmp2 = nullptr;
  float* d_x32 = nullptr;
  float* d_y32 = nullptr;
  double* d_part = nullptr;   // mv partial outputs
  int64_t part_cap = 0;
  double* d_chain = nullptr;
  int64_t chain_cap = 0;
  double* d_mvcomb = nullptr;
  double* d_envcomb = nullptr;
  double* d_Z = nullptr;
  double* d_grpart = nullptr;
  double* d_red = nullptr;    // 128 x kRedBlocks
  double* d_qrmat = nullptr;  // G, R0, R1, R2, Rinv, Rt (mmax^2 each), Cholesky workspace
  double* d_qrR = nullptr;    // R of the last QR (absorbed into the neighbour)
  void* d_cvtasks = nullptr;  // conversion work list (low-precision forms)
  int cv_cap = 0;
  int mmax = 1;
  KrylovState* d_st = nullptr;
  // sweeps: per-node status checks stay on the device (no host round trip per
  // node); every failure status also lands in d_st->sticky, read once per sweep
  bool defer_status = false;
  KJob* d_kjobs64 = nullptr;  // per node: eigensolve descriptors (FP64 / with FP32 copy)
  KJob* d_kjobs32 = nullptr;
  TJob* d_tjobs = nullptr;    // per node: dense tiny-node eigensolve
  std::vector<KJob> h_kjobs;  // host copies for validation
  // Davidson form (allocated at its first use)
  DJob* d_djobs = nullptr;    // per node
  std::vector<DJob> h_djobs;
  DavState* d_dav = nullptr;
  void* d_mlp = nullptr;      // FP16 parameters of the learned correction model
  bool mlp_ready = false;
  double jacobi_rate = 0.9;   // running per-iteration residual reduction of Jacobi-mode solves
  int64_t n_dav_iter = 0, n_fallback = 0;
  double last_rnorm = 0;
  std::vector<TJob> h_tjobs;
  // plans
  std::vector<MVDev> mv;
  // low-precision forms: 4-byte-per-element mirrors of the FP64 stores (FP32,
  // or BF16 hi/lo planes per block) and copies of every matvec work list
  bool lowp_ready[2] = {false, false};
  std::vector<void*> mir[2][2];     // [format - 1][direction][edge]
  std::vector<int64_t> store_elems[2];
  void* comb_lp[2] = {nullptr, nullptr};
  int64_t mvcomb_elems = 0;
  std::vector<MVDev> mvlp[2];
  std::vector<std::vector<std::pair<int64_t, int>>> comb_blocks;   // per node: (offset, dim)
  std::vector<EnvDev> env_up, env_down[2];
  std::vector<QRDev> qr[3];   // per leg, per node
  std::vector<ABDev> ab[3];   // absorb into node along leg
  // FP64 Lanczos sweeps captured as HIP graphs (attn_sweep_opts.use_graphs):
  // a graph replays the launches of one whole sweep from the host state it was
  // captured in (centre, isometry legs, valid stores) and leaves the state it
  // left then, so it is replayed only from an identical start state
  struct SweepState {
    int center = -1;
    std::vector<int> iso;
    std::vector<char> valid0, valid1;
    bool operator==(const SweepState& o) const {
      return center == o.center && iso == o.iso && valid0 == o.valid0 && valid1 == o.valid1;
    }
  };
  struct SweepGraph {
    hipGraphExec_t exec = nullptr;
    int krylov_k = 0;
    SweepState pre, post;
    int64_t d_matvec = 0, d_env = 0, d_qr = 0;
    double d_flops = 0;
  };
  hipStream_t gstream = nullptr;
  std::vector<SweepGraph> sgraphs;   // at most two (the first sweep from a fresh state, then the steady one)
  // counters
  int64_t n_matvec = 0, n_env = 0, n_qr = 0;
  double mv_flops = 0;
  // live timing of the matvec sandwich launches (HIP events on the launch stream)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct ProfRec { int a, b; double flops; int ma, mb, dtype; };
  std::vector<ProfRec> prof_recs;
};


// ---------------------------------------------------------------- shared helpers (runtime.cpp)
namespace rt {
void* dev_alloc(attn_handle* h, size_t bytes);
template <typename T>
T* upload(attn_handle* h, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  void* p = dev_alloc(h, v.size() * sizeof(T));
  if (!h->dryrun) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return (T*)p;
}
double* block_ptr(attn_handle* h, const BRef& b, double* comb_base, const std::vector<int64_t>& comb_off);
void slice_geom(int spect, const int* dm, int& ma, int& mb, int& ns, int64_t& sl, int64_t& row);
// item chunks per spectator of the matvec plan of a node with dims dm
// (target workgroups per launch, per spectator's slice shape)
// matvec work units per spectator group (three groups per node): 3 x 768 =
// three rounds of the 768 workgroups resident at three per CU.  Measured
// against 1024 (four rounds) and 512: sweep 0.581 vs 0.584 and 0.582 s, and a
// quarter fewer partial outputs to write and sum than with 1024.  The batched
// form takes the same split unless it is autotuned.
constexpr int64_t kMvTarget = 768;
void mv_chunks(const MatvecPlan& P, const int* dm, const int64_t target[3], int out[3]);
bool sw_mfma(int ma, int mb);
// Doubles of the QR matrices of a handle whose widest link is mmax: G, R0, R1,
// R2, R^-1, R products (mmax^2 each) and the Cholesky workspace of links wider
// than 128 (two packed triangles, mmax (mmax + 1)).
inline int64_t qrmat_doubles(int64_t mmax) { return 6 * mmax * mmax + mmax * (mmax + 1); }
// Most item chunks (workgroup sets with their own partial output) of one
// sandwich group of a matvec: small nodes get more, so that their few slices
// still spread over the chip.
inline int64_t chunk_cap(int64_t Msz) {
  return Msz >= 65536 ? 32 : std::min<int64_t>(128, std::max<int64_t>(32, ((int64_t)1 << 19) / Msz));
}
// Item chunks per spectator of a matvec plan.  Spectators whose slices have
// the same shape share one launch; the launch gets C = (number of such
// spectators) x target / units item chunks in total (units = workgroups per
// chunk), shared out in proportion to the spectators' item counts by largest
// remainders, so that every chunk carries about the same number of items and
// the chunks add up to exactly C (a launch of C x units workgroups: with the
// default target, whole rounds of the chip's workgroup slots, and no round
// that starts only a few of them).  nitems[sp] = 0: no chunk.
inline void mv_chunk_counts(const int64_t nitems[3], const int ma[3], const int mb[3], const int64_t units[3],
                            int64_t Msz, const int64_t target[3], int out[3]) {
  for (int sp = 0; sp < 3; sp++) out[sp] = 0;
  bool done[3] = {false, false, false};
  for (int sp = 0; sp < 3; sp++) {
    if (nitems[sp] <= 0 || done[sp]) continue;
    int grp[3], ng = 0;
    int64_t tot = 0;
    for (int q = 0; q < 3; q++)
      if (nitems[q] > 0 && ma[q] == ma[sp] && mb[q] == mb[sp]) { grp[ng++] = q; tot += nitems[q]; done[q] = true; }
    const int64_t C = ng * std::max<int64_t>(1, target[sp] / std::max<int64_t>(1, units[sp]));
    int64_t c[3], rem[3], sum = 0;
    for (int g = 0; g < ng; g++) {
      const int q = grp[g];
      c[g] = C * nitems[q] / tot;
      rem[g] = C * nitems[q] - c[g] * tot;   // remainder of the exact share, in units of 1 / tot
      if (c[g] == 0) { c[g] = 1; rem[g] -= tot; }   // every spectator with items gets a chunk
      sum += c[g];
    }
    while (sum < C) {   // the largest remainders get one more chunk (lowest spectator first on ties)
      int best = 0;
      for (int g = 1; g < ng; g++)
        if (rem[g] > rem[best]) best = g;
      c[best]++;
      rem[best] -= tot;
      sum++;
    }
    while (sum > C) {   // the smallest remainders among spectators with two chunks or more give one back
      int worst = -1;
      for (int g = 0; g < ng; g++)
        if (c[g] > 1 && (worst < 0 || rem[g] < rem[worst])) worst = g;
      if (worst < 0) break;
      c[worst]--;
      rem[worst] += tot;
      sum--;
    }
    for (int g = 0; g < ng; g++) {
      const int q = grp[g];
      out[q] = (int)std::max<int64_t>(1, std::min<int64_t>(c[g], std::min<int64_t>(nitems[q], chunk_cap(Msz))));
    }
  }
}
void run_comb(CBPlan& P, hipStream_t s);
void* to_mirror(attn_handle* h, const void* p, int fmt);
void ensure_lowp(attn_handle* h, int dtype);
std::vector<CVTask> lowp_conversions(attn_handle* h, int n, int dtype);
int leg_toward(const Tree& tr, int a, int b);
void run_env(attn_handle* h, EnvDev& D, hipStream_t s);
void qr_node(attn_handle* h, int n, int leg, hipStream_t s);
void absorb(attn_handle* h, int q, int leg, hipStream_t s);
attn_status guard(attn_handle* h, const std::function<attn_status()>& f);
attn_status need_device(attn_handle* h);
void check_state(attn_handle* h, hipStream_t s, const char* where);
void reset_state(attn_handle* h, int kmax, hipStream_t s);
// Mark every effective-operator store stale, then recompute every store that
// points toward the current centre (children before parents off the centre's
// path, then down the path from the root).  Requires every node other than the
// centre to be isometric toward the centre.
void rebuild_envs(attn_handle* h, hipStream_t s);
}  // namespace rt
