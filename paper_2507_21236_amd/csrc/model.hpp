// Host-side structure of an aTTN problem: tree, rotated terms, operator-Schmidt
// splits, per-link block slots and per-node contraction plans.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "attn.h"

namespace attn {

struct Node {
  int lo, mid, hi;   // leaf-position interval; left child covers [lo, mid)
  int child[2];      // >= 0: node id, < 0: -(site + 1)
  int parent;        // -1 for the root
  int side;          // position in the parent (0 = left, 1 = right)
  int dims[3];       // (m_l, m_r, m_p)
};

// Edges are the links below every node or site: edge id = site for a site's
// link to its parent, n_sites + node for a node's link to its parent.
struct Tree {
  int N = 0, m = 0, d = 0, root = 0;
  std::vector<int> leaf;   // leaf position -> site
  std::vector<int> pos;    // site -> leaf position
  std::vector<int> site_parent, site_side;
  std::vector<Node> nodes;
  int dim_of(int k) const;
  int n_edges() const { return N + (int)nodes.size(); }
  int edge_of_child(int n, int side) const {
    int c = nodes[n].child[side];
    return c >= 0 ? N + c : -(c + 1);
  }
  int edge_of_node(int n) const { return N + n; }
  bool edge_is_site(int e) const { return e < N; }
  int edge_lo(int e) const { return e < N ? pos[e] : nodes[e - N].lo; }
  int edge_hi(int e) const { return e < N ? pos[e] + 1 : nodes[e - N].hi; }
  int edge_dim(int e) const { return e < N ? d : nodes[e - N].dims[2]; }
  int edge_upper(int e) const;  // node above the edge
};

// Operator-Schmidt decomposition of a rotated term across the bipartition
// {K, S \ K} of its support (K holds position 0): h = sum_k sigma_k X_k (x) Y_k,
// X_k orthonormal operators on K, Y_k orthonormal operators on S \ K.
// Operator vectors: index (out digits of the positions in increasing order,
// then in digits), base d.
struct Split {
  uint32_t K = 0;
  int t = 0;
  int lenK = 0, lenC = 0;
  std::vector<double> sigma, X, Y;
};

struct RTerm {
  std::vector<int> S;       // support, sorted site ids
  std::vector<double> h;    // d^s x d^s row-major, S[0] most significant
  std::map<uint32_t, Split> splits;
};

// A reference to an m x m block on the device.
//   kind 0: effective-operator store of an edge (dir 0 = from below, 1 = from
//           above), slot -1 = summed local operator, slot >= 0 = term block.
//   kind 1: combined block in the node scratch area (index = slot).
//   kind 2: no operator (identity).
//   kind 3: zero operator (the product vanishes).
struct BRef {
  int kind = 2, edge = -1, dir = 0, slot = -1;
  static BRef none() { return BRef(); }
  static BRef store(int e, int dir, int slot) { BRef b; b.kind = 0; b.edge = e; b.dir = dir; b.slot = slot; return b; }
  static BRef comb(int idx) { BRef b; b.kind = 1; b.slot = idx; return b; }
  static BRef zero() { BRef b; b.kind = 3; return b; }
  bool is_none() const { return kind == 2; }
  bool is_zero() const { return kind == 3; }
};

struct Combine {
  int dim = 0;
  std::vector<std::pair<BRef, double>> in;
};

// Product item on two legs: coef * (opA on leg a) (x) (opB on leg b), identity
// on the third (spectator) leg.  Spectator l: (a, b) = (r, p); spectator r:
// (l, p); spectator p: (l, r).
struct Item2 {
  int spect;
  BRef A, B;
  double coef;
};

// Three-leg term as a chain o2 -> mid -> o1:
//   W_c = O2_c x_o2 x;  V_a = sum_c Mid_{a,c} x_mid W_c;  y += sum_a O1_a x_o1 V_a
struct Chain {
  int o1, mid, o2;
  std::vector<BRef> O1, O2;
  std::vector<BRef> Mid;   // t1 * t2, index a * t2 + c
};

struct MatvecPlan {
  std::vector<Item2> items;      // local operators and two-leg terms
  std::vector<Chain> chains;     // three-leg terms
  std::vector<Combine> combines; // blocks combined on the device before use
  int64_t flops = 0;
  int n_cross = 0;
};

// Effective-operator update at node q toward leg j: for each output block o
// (slot -1 = the summed local operator), Z_o = sum items (A (x) B (x) 1_j) T_q,
// O_o = contraction of T_q with Z_o over the two legs other than j.
struct EnvOut {
  int slot;
  std::vector<Item2> items;   // spect = j
};

struct EnvPlan {
  int node = -1, leg = -1, out_edge = -1, out_dir = 0;
  std::vector<EnvOut> outs;
  std::vector<Combine> combines;
};

struct EdgeCross {
  int term;
  uint32_t mask;   // support positions below the edge
  int slot0, t;
};

struct Model {
  Tree tree;
  std::vector<RTerm> terms;
  // per edge: crossing terms with their slots, total slots, local-op flags
  std::vector<std::vector<EdgeCross>> cross;
  std::vector<int> n_slots;
  std::vector<char> has_local[2];   // per edge, per direction
  std::vector<MatvecPlan> mv;       // per node
  std::vector<EnvPlan> env_up;      // per node (toward parent), root unused
  std::vector<EnvPlan> env_down[2]; // per node, into child side (node children only)
  // site-edge constant blocks (column-major d x d): E then slots
  std::vector<std::vector<double>> site_blocks;
};

// Builds everything; returns ATTN_OK or an error code with a message.
attn_status build_model(const attn_problem* p, Model& M, std::string& err);

// helpers shared with tests of the host build
int mask_popcount(uint32_t m);

// The disentanglers touching a term contracted into it (Sec. 4.3): S = the
// term's sites plus the partner sites of every gate touching them (sorted),
// H = U^T (h (x) 1) U, d^|S| x d^|S| row-major with S[0] most significant;
// tdense = the term's own dense operator on tsites (in that order); de_of[site]
// = index of its gate or -1.  Errors: UNSUPPORTED (support beyond 6 sites).
attn_status rotate_term_dense(const std::vector<int>& tsites, const std::vector<double>& tdense, int d,
                              const std::vector<int>& de_of, const int32_t* de_sites, const double* de_u,
                              std::vector<int>& S, std::vector<double>& H, std::string& err);

// One-sided Jacobi SVD of the r x c row-major A: A = U diag(s) V^T (U r x k,
// V c x k row-major, k = min(r, c), singular values descending).
void svd_jacobi(const std::vector<double>& A, int r, int c, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& V);

}  // namespace attn
