/*
 * attn.h -- C interface of the MI355X (gfx950) library for the hot path of the
 * augmented tree tensor network (aTTN) ground-state search.
 *
 * The method (Reinic, Pavesic, Jaschke, Montangero, "The Augmented Tree Tensor
 * Network Cookbook"):
 *   |psi_aTTN> = D(u) |psi_TTN>, D(u) = prod_k u_k two-site unitaries on the
 *   bottom of a binary TTN (Sec. 2, eq. 1).  The ground-state sweep maps the
 *   Hamiltonian (a sum of local terms stored term by term as a TPO, Sec. 3.3)
 *   to H' with the disentangler layer contracted into every term (Sec. 4.3,
 *   algorithm "Contract disentangler layer"), then runs a DMRG sweep of
 *   single-tensor updates on the TTN (Sec. 4, step 3): QR isometrisation
 *   (Sec. 3.1), effective operators kept term by term (Sec. 3.3.2), and the
 *   generalised matvec (Sec. 3.3.2, cost in Sec. 4.4.2) inside the Lanczos
 *   eigensolver (Sec. 4.4.2).
 *
 * Conventions shared by every call:
 *   - Every call returns attn_status: 0 = ATTN_OK, negative = error.  No C++
 *     exception crosses this interface.  attn_last_error(h) gives a message.
 *   - Validation errors leave the handle unchanged.  After ATTN_ERR_HIP or
 *     ATTN_ERR_NUMERIC only attn_last_error and attn_destroy may be called.
 *   - A handle is not thread-safe; separate handles are independent.
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Work is enqueued asynchronously on that stream; only
 *     calls that return host scalars synchronise it.
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied.  Device pointers passed in (attn_heff_apply) are owned by the
 *     caller and must live on the handle's device.
 *   - Tensors are real, row-major T[l][r][p]: l = left child leg, r = right
 *     child leg, p = parent leg.  Node ids are the post-order of the binary
 *     tree (left subtree, right subtree, node); the root is n_sites - 2 and
 *     its parent leg has dimension 1.  Legs are numbered 0 = l, 1 = r, 2 = p.
 *   - Bond dimension of the link above a k-site subtree: min(m, d^k, d^(N-k)).
 */
#ifndef ATTN_H
#define ATTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t attn_status;

#define ATTN_OK                  0
#define ATTN_ERR_ARG            -1   /* null pointer, out-of-range or duplicate value */
#define ATTN_ERR_NOT_UNITARY    -2   /* ||u^T u - 1||_max > 1e-12 for a disentangler */
#define ATTN_ERR_NOT_HERMITIAN  -3   /* a term's operator is not symmetric (1e-12) */
#define ATTN_ERR_DE_OVERLAP     -4   /* a site belongs to two disentanglers */
#define ATTN_ERR_DE_RESTRICTION -5   /* ATTN_DE_STRICT: a placement restriction is broken */
#define ATTN_ERR_OOM            -6   /* device or host allocation failed */
#define ATTN_ERR_HIP            -7   /* a HIP runtime call failed */
#define ATTN_ERR_STATE          -8   /* call not valid in the current state (see each call) */
#define ATTN_ERR_SHAPE          -9   /* buffer length does not match the tensor size */
#define ATTN_ERR_NUMERIC       -10   /* NaN / Inf, or a factorisation broke down */
#define ATTN_ERR_UNSUPPORTED   -11   /* valid input outside what this library implements */
#define ATTN_ERR_IO            -12   /* a file cannot be opened, read or written, or is corrupt */
#define ATTN_ERR_MISMATCH      -13   /* a checkpoint belongs to another problem */

/* attn_problem.flags */
#define ATTN_DE_STRICT     1u  /* enforce both placement restrictions of Sec. 6.1.1 */
#define ATTN_HOST_ONLY     2u  /* build host-side structures only, touch no GPU */
#define ATTN_DRYRUN        4u  /* build every device work list against a fake address
                                  space without touching the GPU (for attn_validate) */
#define ATTN_COMPRESS_TERMS 8u /* sum the terms that act on the same set of sites into
                                  one term before the factorisation (Sec. 6.2.2, closing
                                  paragraph: fewer TPO terms, one bond <= d^2 per cut
                                  for a two-site sum under one disentangler) */

typedef enum attn_dtype {
  ATTN_F64 = 0,     /* FP64 operands, FP64 accumulation */
  ATTN_F32 = 1,     /* FP32 operands on MFMA, FP32 accumulation */
  ATTN_BF16X2 = 2   /* operands split hi+lo in BF16, three products, FP32 accumulation */
} attn_dtype;

/*
 * The problem: a lattice Hamiltonian as a sum of local terms (Sec. 3.3), a
 * binary tree over the sites in `leaf_order` (Sec. 3.1), bond dimension m and
 * a layer of two-site disentanglers (Sec. 3.2).
 *
 *   n_sites, d, m     number of sites (>= 2), local dimension (>= 2), maximal
 *                     bond dimension (>= 1).
 *   leaf_order        [n_sites] permutation of 0..n_sites-1: site at each leaf.
 *   n_terms           number of terms.
 *   term_nsites       [n_terms] sites per term, 1..4.
 *   term_sites        concatenated site ids of every term (distinct per term).
 *   term_ops          concatenated d x d row-major real operators, one per
 *                     site of every term, in the order of term_sites.
 *   term_coef         [n_terms] real coefficient; term = coef * (op_0 x op_1 ..).
 *   n_de              number of disentanglers.
 *   de_sites          [n_de][2] site pairs (no site in two pairs).
 *   de_u              [n_de][d*d][d*d] row-major real orthogonal matrices acting on
 *                     |s_a s_b> with the first listed site the major index.
 *   flags             ATTN_DE_STRICT, ATTN_HOST_ONLY, ATTN_DRYRUN,
 *                     ATTN_COMPRESS_TERMS.
 *   device            HIP device ordinal for all device memory of the handle.
 */
typedef struct attn_problem {
  int32_t n_sites, d, m;
  const int32_t* leaf_order;
  int32_t n_terms;
  const int32_t* term_nsites;
  const int32_t* term_sites;
  const double* term_ops;
  const double* term_coef;
  int32_t n_de;
  const int32_t* de_sites;
  const double* de_u;
  uint32_t flags;
  int32_t device;
} attn_problem;

typedef struct attn_handle attn_handle;

/* Local eigensolver options (Sec. 4.4.2: Lanczos inside the sweep). */
#define ATTN_SOLVER_LANCZOS  0
#define ATTN_SOLVER_DAVIDSON 1
#define ATTN_PRECOND_NONE    0
#define ATTN_PRECOND_JACOBI  1
#define ATTN_PRECOND_LEARNED 2

typedef struct attn_solver_opts {
  int32_t solver;      /* ATTN_SOLVER_LANCZOS (default) or ATTN_SOLVER_DAVIDSON */
  int32_t krylov_k;    /* Lanczos: number of matvecs k (capped at the tensor size);
                          Davidson: maximal subspace size */
  double tol;          /* Davidson: residual norm tolerance; Lanczos: unused */
  int32_t precision;   /* attn_dtype of the H_eff contractions; Krylov stays FP64 */
  int32_t precond;     /* Davidson preconditioner: NONE, JACOBI or LEARNED */
  int32_t max_iter;    /* Davidson: maximal number of matvecs */
  int32_t restart;     /* Davidson: vectors kept at a restart */
} attn_solver_opts;

typedef struct attn_sweep_opts {
  attn_solver_opts solver;
  int32_t use_graphs;  /* 1: FP64 Lanczos sweeps run from HIP graphs on a stream of
                          the handle: the first sweep from a given host state
                          (centre, isometries, valid effective operators) is
                          captured, later sweeps from the same state replay it
                          (two graphs kept); same results as without graphs */
} attn_sweep_opts;

/*
 * a1. Rotated TPO build (Sec. 4.3, algorithm "Contract disentangler layer"):
 * validates the problem, builds the tree and bond dimensions, contracts the
 * disentanglers touching each term into it (h' = U^T h U on the extended
 * support), factorises every rotated term across each tree link it crosses
 * (operator-Schmidt decompositions: minimal TPO bonds, at most d^2 for a term
 * touching one disentangler, d^4 for two), classifies terms per node as local
 * (summed into one operator per leg) or crossing, and allocates all device
 * storage.  Tensors must then be given with attn_init_state or attn_set_tensor.
 * *out is owned by the caller; release it with attn_destroy.
 * Errors: ARG, NOT_UNITARY, NOT_HERMITIAN, DE_OVERLAP, DE_RESTRICTION
 * (strict mode), UNSUPPORTED (supports beyond 6 sites), OOM, HIP.
 */
attn_status attn_build_tpo(const attn_problem* p, attn_handle** out);

/* Release every resource of the handle.  NULL is accepted. */
attn_status attn_destroy(attn_handle* h);

/* Message of the last error on this handle (owned by h); "" if none.
 * With h == NULL: the last error of a failed attn_build_tpo in this thread. */
const char* attn_last_error(const attn_handle* h);

/* Structure of node `node` and the cost of its matvec (Sec. 4.4.2: each TPO
 * term of the effective operators is contracted into the tensor in turn, so
 * the cost is set by the bond dimensions, the TPO bonds t and the number of
 * terms): dims[3] = (m_l, m_r, m_p); *n_cross = number of
 * crossing terms; *flops = algorithmic flops of one matvec (summed local legs
 * 2 m_j M, two-leg terms 2 M t (m_a + m_b), three-leg terms the cheapest chain
 * 2 M (t_a m_a + t_a t_c m_b + t_c m_c); M = m_l m_r m_p, t = minimal bonds).
 * Any output pointer may be NULL.  Works on host-only handles.  Errors: ARG. */
attn_status attn_node_info(const attn_handle* h, int32_t node, int32_t dims[3],
                           int32_t* n_cross, double* flops);

/* Tree and storage summary: n_nodes, root id, total device bytes of
 * effective-operator storage.  Any pointer may be NULL. */
attn_status attn_tree_info(const attn_handle* h, int32_t* n_nodes, int32_t* root,
                           int64_t* env_bytes);

/* Initial state (reading of the paper's random start): `raw` holds one block of
 * m_l*m_r*m_p values per node in post-order (concatenated, row-major).  Every
 * non-root block, viewed as an (m_l m_r) x m_p matrix, is replaced by Q of its
 * QR decomposition with diag(R) >= 0; the root block is normalised.  The
 * isometry centre is the root and all effective operators toward it are built.
 * Synchronises the stream.  Errors: SHAPE (len), STATE (host-only), NUMERIC, HIP. */
attn_status attn_init_state(attn_handle* h, const double* raw, int64_t len, void* stream);

/* Load / read back T_node (host buffer of exactly m_l*m_r*m_p doubles).
 * attn_set_tensor invalidates every effective operator that depends on the
 * node; the node keeps its isometry direction.  attn_get_tensor synchronises.
 * Errors: ARG, SHAPE, STATE (host-only), HIP. */
attn_status attn_set_tensor(attn_handle* h, int32_t node, const double* host, int64_t len);
attn_status attn_get_tensor(attn_handle* h, int32_t node, double* host, int64_t len);

/* Current isometry centre (node id). */
attn_status attn_get_center(const attn_handle* h, int32_t* node);

/*
 * a2. Effective-operator update (Sec. 3.3.2): renormalise every term through
 * T_node onto the link at leg `leg` (0 = l, 1 = r, 2 = p), in the direction
 * pointing away from `node`.  Terms confined to node's side are summed into
 * the link's local operator; terms reaching across it keep one m x m block per
 * TPO bond index.  Requires T_node isometric toward `leg` and the node's two
 * other incoming effective operators current.  Child legs that are sites
 * carry no tensor: leg must lead to a tree node.
 * Errors: ARG, STATE (not isometric toward leg / stale inputs / host-only), HIP.
 */
attn_status attn_update_env(attn_handle* h, int32_t node, int32_t leg, void* stream);

/*
 * a3. H_eff matvec (Sec. 3.3.2; its cost, Sec. 4.4.2): y <- H_eff(node) x, with
 * H_eff = E_l x 1 x 1 + 1 x E_r x 1 + 1 x 1 x E_p + sum over crossing terms of
 * their leg blocks contracted into x over the TPO bonds.  x and y are device
 * pointers of M = m_l m_r m_p elements, row-major [l][r][p]: double for
 * ATTN_F64, float for ATTN_F32 and ATTN_BF16X2 (split into hi/lo inside).
 * They must not alias.  Asynchronous on `stream`.
 * Errors: STATE (node is not the centre, or its incoming effective operators
 * are stale, or host-only), ARG (NULL pointer or dtype), HIP.
 */
attn_status attn_heff_apply(attn_handle* h, int32_t node, int32_t dtype, const void* x,
                            void* y, void* stream);

/*
 * a4. Local eigensolve (Sec. 4: the variational sweep minimises the energy
 * of one tensor at a time; Sec. 4.4.2: with the Lanczos algorithm, one matvec
 * per iteration): lowest eigenpair of H_eff(node), warm-started from
 * T_node.  Lanczos: k = min(opts->krylov_k, M) matvecs, three-term recurrence
 * plus two passes of classical Gram-Schmidt in FP64, stop when
 * beta_j <= 1e-14 max|alpha|; lowest eigenpair of the tridiagonal matrix; the
 * normalised Ritz vector (sign: non-negative overlap with the start vector)
 * replaces T_node.  Davidson (optional form): Jacobi or learned pointwise
 * preconditioner, stops at residual norm <= tol.  Synchronises `stream` and
 * returns theta and the number of matvecs.  opts may be NULL (Lanczos, k = 20,
 * FP64).  Errors: STATE (as heff_apply), NUMERIC (non-finite values), HIP.
 */
attn_status attn_eigsolve_node(attn_handle* h, int32_t node, const attn_solver_opts* opts,
                               double* theta, int32_t* n_matvec, void* stream);

/*
 * a5. Isometrisation (Sec. 3.1): move the centre from `from` to the adjacent
 * node `to`.  QR of T_from matricised (other two legs) x (leg toward `to`),
 * with diag(R) >= 0; Q replaces T_from, R is absorbed into T_to along that
 * link.  Does not update effective operators: follow with
 * attn_update_env(from, leg toward to).
 * Errors: ARG (not adjacent), STATE (from is not the centre), NUMERIC, HIP.
 */
attn_status attn_isometrize(attn_handle* h, int32_t from, int32_t to, void* stream);

/* Move the isometry centre to `target` link by link (attn_isometrize then
 * attn_update_env for every link of the tree path).  Errors: as those calls. */
attn_status attn_move_center(attn_handle* h, int32_t target, void* stream);

/*
 * a6. Sweep (Sec. 4, step 3): n_sweeps sweeps over all nodes in post-order;
 * the centre moves link by link (attn_isometrize then attn_update_env) and
 * every node is optimised with attn_eigsolve_node.  energies[s] = theta at the
 * last node of sweep s, seconds[s] = wall time of sweep s (device synchronised).
 * Output arrays are caller-owned, n_sweeps entries each (either may be NULL).
 * Errors: any of the calls above.
 */
attn_status attn_sweep(attn_handle* h, int32_t n_sweeps, const attn_sweep_opts* opts,
                       double* energies, double* seconds);

/*
 * Davidson form (not from the paper, which uses Lanczos): attn_eigsolve_node
 * with opts->solver = ATTN_SOLVER_DAVIDSON runs Davidson's method in FP64
 * (contractions in opts->precision): basis of at most min(krylov_k, 32)
 * vectors, restart to the lowest opts->restart Ritz vectors, stop at residual
 * norm <= opts->tol or after opts->max_iter matvecs.  Corrections:
 * ATTN_PRECOND_JACOBI, t_i = -r_i / (diag_i - theta) with the H_eff diagonal
 * assembled from the diagonals of the operators of every term; or
 * ATTN_PRECOND_LEARNED, a pointwise model t_i = o(f_i) ||r||_inf / ||diag||_inf
 * of the features f_i = ((diag_i - theta)/||diag||_inf, r_i/||r||_inf,
 * theta/||diag||_inf): three tanh layers of width 64, FP16 parameters, FP32
 * arithmetic.  The learned correction falls back to Jacobi for the rest of a
 * solve when it is not finite, adds nothing to the basis, or reduces the
 * residual less than the running Jacobi rate for two consecutive iterations.
 */

/* Number of model parameters: W1[3][64], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[64], b4 (row-major; layer k maps h to tanh(h W + b)). */
#define ATTN_MLP_PARAMS 8641

/* Load the model (FP32 host array of ATTN_MLP_PARAMS values, stored as FP16).
 * Errors: SHAPE (n), STATE (no device), HIP. */
attn_status attn_precond_set_weights(attn_handle* h, const float* params, int64_t n);

/* Davidson counters since the handle was built: iterations, fallbacks to
 * Jacobi, residual norm at the end of the last Davidson solve and the running
 * Jacobi reduction rate.  Pointers may be NULL. */
attn_status attn_solver_stats(const attn_handle* h, int64_t* dav_iters, int64_t* fallbacks,
                              double* last_rnorm, double* jacobi_rate);

/* diag(H_eff(node)) into the device array `diag` (M doubles, layout of T_n).
 * node must be the centre with current effective operators.  Asynchronous. */
attn_status attn_heff_diagonal(attn_handle* h, int32_t node, double* diag, void* stream);

/* Training data of the learned correction at the centre `node`: n_pairs
 * Davidson iterations with Jacobi corrections from T_n; at each, the exact
 * Jacobi-Davidson correction t* (solution of (1 - uu^T)(H - theta)(1 - uu^T) t = -r,
 * t orthogonal to u) by projected conjugate gradients to relative residual
 * cg_tol (at most cg_max matvecs).  Writes the features (device float
 * [n_pairs][M][3]) and the scaled targets t* ||diag||_inf / ||r||_inf (device
 * float [n_pairs][M]); cg_res[p] (host, may be NULL) = achieved relative CG
 * residual.  T_n is left unchanged.  Synchronises `stream`. */
attn_status attn_precond_harvest(attn_handle* h, int32_t node, int32_t n_pairs, double cg_tol,
                                 int32_t cg_max, float* feats, float* targets, double* cg_res,
                                 void* stream);

/* Train the model on n points (device features [n][3], targets [n]): `steps`
 * Adam steps (lr; beta 0.9, 0.999; eps 1e-8) on consecutive batches of `batch`
 * points (a multiple of 64; batch k uses points [(k mod (n / batch)) batch, +batch)),
 * mean-squared-error loss, hand-written FP32 kernels.  params (host,
 * ATTN_MLP_PARAMS) is the start point and receives the result; loss (host,
 * `steps` values, may be NULL) the batch losses.  Errors: ARG, HIP. */
attn_status attn_mlp_train(const float* feats, const float* targets, int64_t n, int32_t steps,
                           int32_t batch, float lr, float* params, float* loss, void* stream);

/* attn_mlp_train without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, work and results as
 * attn_mlp_train; its working memory (parameters, Adam moments, gradient,
 * per-workgroup partial sums, per-step losses: 9.25 MB) is a fixed device
 * array of the library, one per device, held until the process ends, on the
 * device current at the call.  Limits: batch <= 16384 and steps <= 65536,
 * else UNSUPPORTED.  Every call on a device shares that device's array:
 * calls that overlap on one device (other host threads, other streams) race,
 * so serialise them.  Synchronises `stream`.  Errors: ARG, UNSUPPORTED, HIP. */
attn_status attn_mlp_train_noalloc(const float* feats, const float* targets, int64_t n, int32_t steps,
                                   int32_t batch, float lr, float* params, float* loss, void* stream);

/* Model outputs o for n feature triples (device in/out) with the FP16-rounded
 * parameters (host FP32).  Synchronises `stream`. */
attn_status attn_mlp_eval(const float* params, const float* feats, float* out, int64_t n,
                          void* stream);

/*
 * Batched form (not from the paper): independent problem instances, each its
 * own handle (sizes and bond dimensions may differ, d must agree, legs <= 64),
 * swept in lock step.  Step t of a batch sweep moves every instance's centre to
 * its node t (post-order; instances with fewer nodes idle) and optimises it.
 * The eigensolver work of all instances in a step runs in mixed-shape launches
 * over one work list (all terms of every active node: two-leg terms and local
 * operators in one launch, each stage of the three-leg chains in one launch,
 * every Krylov vector step in one launch); the centre moves of different
 * instances run concurrently on four streams.  With persistent, each matvec
 * of a step is instead ONE launch: a resident grid takes the units of all
 * instances (transposes, chain stages, two-leg tiles, reduction tiles) from
 * one ordered work list by ticket, and a unit that needs earlier results waits
 * on a per-instance counter of the units it depends on, which always come
 * earlier in the list (persistent = 2: each step takes whichever of the two
 * forms ran its matvec faster when timed at creation).  With use_graphs each
 * step is captured once as a HIP graph and replayed in later sweeps.  With
 * autotune the work split of the two-leg launches (and, for FP32 legs 64 x 64
 * in the staged launches, the tile of a wave: one or two 16-row strips) is
 * chosen per leg shape (ma, mb) by timing the candidates over all steps at
 * creation.  Without autotuning the split is the one the single-handle path
 * uses, and batch sweeps then reproduce attn_sweep of each handle bit for
 * bit.
 * The batch borrows the handles (they must outlive it and must not be used
 * while it sweeps).  Each handle must be in the sweep start state: after
 * attn_init_state or after full sweeps.
 */
typedef struct attn_batch attn_batch;

typedef struct attn_batch_opts {
  int32_t krylov_k;    /* Lanczos matvecs per node (20) */
  int32_t precision;   /* ATTN_F64 or ATTN_F32 operands; Krylov steps stay FP64 */
  int32_t use_graphs;  /* 1: capture every step as a HIP graph */
  int32_t autotune;    /* 1: time candidate work splits (and FP32 tiles) per leg shape at creation */
  int32_t persistent;  /* 0: staged launches; 1: each matvec of a step is one
                          launch of a resident grid over an ordered work list
                          of all instances' units; 2: per step, whichever of
                          the two timed faster at creation (every choice gives
                          the same results bit for bit) */
} attn_batch_opts;

/* opts may be NULL (k = 20, FP32, graphs, no autotuning, staged launches).
 * *out is owned by the caller (attn_batch_destroy).  Errors: ARG (also
 * persistent outside 0..2), STATE (handle not on a device), UNSUPPORTED (mixed
 * d or devices, legs above 64, BF16X2), HIP, OOM. */
attn_status attn_batch_create(attn_handle* const* hs, int32_t n, const attn_batch_opts* opts,
                              attn_batch** out);

/* n_sweeps lock-step sweeps.  energies[i * n_sweeps + s] = theta at the last
 * node (root) of instance i in sweep s; seconds[s] = wall time of sweep s.
 * Either array may be NULL.  Errors: STATE (a handle is not in the sweep start
 * state), NUMERIC, HIP (also when a wait inside a persistent matvec ran past
 * its limit of about a second; the batch is then unusable). */
attn_status attn_batch_sweep(attn_batch* b, int32_t n_sweeps, double* energies, double* seconds);

/* Number of steps, sandwich work units per sweep-step matvec summed over steps,
 * and the autotuned choices per leg shape: tuned[4k..4k+3] = (ma, mb, target
 * workgroups, rows per wave: 16, or 32 for the two-strip FP32 tile at legs
 * 64 x 64).  tuned holds 4 * cap values. */
attn_status attn_batch_info(const attn_batch* b, int32_t* n_steps, int64_t* n_launch_units,
                            int32_t* n_tuned, int32_t* tuned, int32_t cap);

/* Steps that run matvecs, and how many of them use the persistent launch. */
attn_status attn_batch_forms(const attn_batch* b, int32_t* n_matvec_steps, int32_t* n_persistent_steps);

/* Message of the last error of b (of the last failed attn_batch_create when b
 * is NULL); owned by the library. */
const char* attn_batch_last_error(const attn_batch* b);

attn_status attn_batch_destroy(attn_batch* b);

/*
 * Checkpoint and restore of the variational state (the sweep is an iteration,
 * Sec. 4: the state after any number of sweeps is the starting point of the
 * next, so it can be saved and resumed).
 *
 * attn_checkpoint writes `path` (through `path`.tmp and a rename): a hash of
 * the problem the handle was built from (sizes, leaf order, terms,
 * disentangler sites, strict flag), the disentangler matrices, every tensor
 * T_n, the isometry centre and the isometry direction of every node, and the
 * energies of every sweep run so far through attn_sweep; the file ends with a
 * checksum.  Synchronises the device.  Errors: ARG (NULL path), STATE (no
 * state: attn_init_state not called; host-only handle), IO, HIP.
 *
 * attn_restore loads such a file into a handle built from the same problem
 * (same hash) with the same disentanglers: tensors, centre, isometry
 * directions and sweep history are replaced, and every effective operator
 * pointing toward the centre is recomputed from the restored tensors, so the
 * handle continues exactly as the saved one would have (sweeps after a
 * restore repeat those of the uninterrupted run bit for bit).  Synchronises
 * the device.  Errors: ARG, IO (unreadable, truncated or corrupt file,
 * directions that do not point to the centre), MISMATCH (another problem or
 * other disentanglers), STATE (host-only), HIP.
 */
attn_status attn_checkpoint(attn_handle* h, const char* path);
attn_status attn_restore(attn_handle* h, const char* path);

/* Header of a checkpoint file, read and checksum-verified on the host (no
 * handle or GPU needed).  Any output pointer may be NULL.  Errors: ARG, IO. */
attn_status attn_checkpoint_info(const char* path, uint64_t* problem_hash, int32_t* n_nodes,
                                 int32_t* center, int64_t* n_sweeps);

/* Problem hash of the handle (the value a checkpoint records). */
attn_status attn_problem_hash(const attn_handle* h, uint64_t* hash);

/* Energies of every sweep run on the handle (including those restored from a
 * checkpoint): *n_sweeps = count, energies[0 .. min(cap, count)) written. */
attn_status attn_sweep_history(const attn_handle* h, int64_t* n_sweeps, double* energies, int64_t cap);

/*
 * Observables (Sec. 5).  Every call moves the isometry centre to the root
 * first (attn_move_center; the state is unchanged, only its gauge) and
 * synchronises the device.  Operators are d x d row-major real matrices,
 * element [i][k] = <i|A|k>.
 *
 * attn_expect_products: out[p] = <psi_TTN| prod_i A_(p,i) |psi_TTN> for n_prod
 * products of one-site operators on distinct sites (the TTN alone, no
 * disentanglers; Sec. 5.1: only the subtree holding the operators is
 * contracted).  nsites[p] sites per product; sites and ops concatenated over
 * the products (d*d values per site).  Errors: ARG, STATE, HIP.
 *
 * attn_measure: out[o] = <psi_aTTN| coef_o prod_i A_(o,i) |psi_aTTN> for n_obs
 * observables on 1..4 distinct sites each: the disentanglers touching an
 * observable are contracted into it, o' = U^T o U (Sec. 5.2, eq. 6, read with
 * the state D|psi_TTN> as for the Hamiltonian), and o' is measured on the TTN
 * as a sum of products of one-site operators (nested operator-Schmidt
 * decompositions).  coef may be NULL (all 1).  Errors: ARG, STATE, UNSUPPORTED
 * (rotated support beyond 6 sites), HIP.
 *
 * attn_correlation: the two-body correlation matrix of eq. 7 (Sec. 5.3),
 * C[i * N + j] = <psi_aTTN| o^a_i o^b_j |psi_aTTN> for all sites i, j (N x N,
 * row-major, caller-owned), the diagonal being the one-site product
 * o^a o^b; every entry is the rotated pair measured as above, the rotated
 * one-site factors shared between entries.  Errors: ARG, STATE, HIP.
 */
attn_status attn_expect_products(attn_handle* h, int32_t n_prod, const int32_t* nsites, const int32_t* sites,
                                 const double* ops, double* out);
attn_status attn_measure(attn_handle* h, int32_t n_obs, const int32_t* nsites, const int32_t* sites,
                         const double* ops, const double* coef, double* out);
attn_status attn_correlation(attn_handle* h, const double* oa, const double* ob, double* C);

/*
 * Disentangler optimisation (Sec. 4.1, MERA-like variant of Sec. 4.1.1) and
 * the aTTN ground-state recipe of Sec. 4 (each sweep: optimise the layer,
 * contract it into the Hamiltonian, sweep the TTN).  Needs the placement
 * restriction of Sec. 4.1 (no term acts on two disentanglers: problems built
 * with ATTN_DE_STRICT placements), else DE_RESTRICTION.
 *
 * attn_optimize_disentanglers: for every gate k, the energy of the terms on
 * its sites with the bra copy of u_k fixed at u~ is Tr(u_k Gamma_k) (eq. 4);
 * Gamma_k is built from expectation values of the current TTN state (the
 * environment, computed once on the GPU with the centre moved to the root);
 * u_k <- -V U^T for Gamma_k = U sigma V^T (eq. 5), repeated with the new u as
 * u~ until the gate's energy changes by <= rel_tol * max(1, |E|) or max_iter
 * steps.  With shift = 1 the gate's terms are shifted by an upper bound of
 * their largest eigenvalue (sum of |coef| prod ||op||_2) first: the energy is
 * then a concave function of u_k, its linearisation an upper bound, and no
 * step raises the energy (the paper does not fix a safeguard; shift = 0 is
 * the plain linearisation).  Gates are independent under the restriction, so
 * all are optimised from the same state.  Writes the new matrices
 * (de_u_out, [n_de][d^2][d^2] row-major, the layout of attn_problem.de_u),
 * and per gate the energy of its terms before and after and the number of
 * steps (any output may be NULL).  The handle keeps its disentanglers: apply
 * the result with attn_set_disentanglers.  opts may be NULL (MERA-like,
 * 20 steps, rel_tol 1e-12, shift on).  Errors: ARG, STATE, DE_RESTRICTION, HIP.
 *
 * attn_set_disentanglers: replaces the disentangler matrices (same sites):
 * the rotated TPO is rebuilt (attn_build_tpo on the stored problem), the TTN
 * tensors, centre and sweep history are kept, and every effective operator
 * toward the centre is recomputed.  Batches that borrow the handle become
 * invalid.  Errors: ARG, NOT_UNITARY, OOM, HIP.
 *
 * attn_sweep_attn: n_sweeps sweeps; from sweep s_ttn on (counted in this
 * call), each sweep is preceded by attn_optimize_disentanglers and
 * attn_set_disentanglers (Sec. 6.3: the first S_TTN sweeps run on the TTN
 * with the given layer, e.g. the identity, S_TTN = 1 being the paper's best
 * schedule).  energies[s] / seconds[s] as attn_sweep (seconds include the
 * layer update).  Errors: as the calls it makes.
 *
 * attn_get_disentanglers: the current matrices (len = n_de d^4 values).
 */
typedef struct attn_de_opts {
  int32_t max_iter;   /* steps per gate (20) */
  double rel_tol;     /* stop at |dE| <= rel_tol * max(1, |E|) (1e-12) */
  int32_t shift;      /* MERA-like: 1 shifted terms (monotone steps); 0 plain linearisation */
  int32_t method;     /* ATTN_DE_MERA (default) or ATTN_DE_RCG */
} attn_de_opts;

/* attn_de_opts.method.  ATTN_DE_RCG: gradient optimisation of Sec. 4.1.2, both
 * copies of u_k varied together, as Riemannian conjugate gradient on the
 * orthogonal group (the paper names Riemannian nonlinear CG): skew directions
 * in the frame of u, Polak-Ribiere+ coefficient, steps u <- u cay(t D) with
 * cay(X) = (I - X/2)^-1 (I + X/2) and t halved from 1 until the Armijo
 * condition E_new <= E + 1e-4 t <g, D> holds, restart along -g when D is not
 * a descent direction; the energy never rises.  Real orthogonal gates only:
 * every tensor of this library is real. */
#define ATTN_DE_MERA 0
#define ATTN_DE_RCG  1

attn_status attn_optimize_disentanglers(attn_handle* h, const attn_de_opts* opts, double* de_u_out,
                                        double* e_before, double* e_after, int32_t* iters);
attn_status attn_set_disentanglers(attn_handle* h, const double* de_u);
attn_status attn_sweep_attn(attn_handle* h, int32_t n_sweeps, int32_t s_ttn, const attn_sweep_opts* sopts,
                            const attn_de_opts* dopts, double* energies, double* seconds);
attn_status attn_get_disentanglers(const attn_handle* h, double* de_u, int64_t len);

/* Checks on the host that every work unit of every device work list of the
 * handle reads and writes only inside the buffer it was built for.  Meant for
 * ATTN_DRYRUN handles (no GPU needed).  Errors: STATE (message names the first
 * violation), ARG. */
attn_status attn_validate(const attn_handle* h);

/* Counters since the handle was built: matvecs, env updates, QR moves and the
 * algorithmic flops of all matvecs (attn_node_info's count per matvec).  Any
 * pointer may be NULL. */
attn_status attn_counters(const attn_handle* h, int64_t* n_matvec, int64_t* n_env,
                          int64_t* n_qr, double* matvec_flops);

/* Live timing of the matvec's two-leg contraction kernel.  enable = 1 starts
 * recording: every launch of that kernel is bracketed by HIP events on its own
 * stream.  enable = 0 synchronises the device, stops recording and returns the
 * summed event time (*ms), algorithmic flops (*flops) and number of launches
 * (*launches) of the launches whose two contracted legs are both >= min_dim.
 * Errors: STATE (host-only / dry-run handle), HIP. */
attn_status attn_profile(attn_handle* h, int32_t enable, int32_t min_dim, double* ms,
                         double* flops, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* ATTN_H */
