// Host build of an aTTN problem (no GPU work): validation, the binary tree,
// the disentangler layer contracted into every term (paper Sec. 4.3, algorithm "Contract disentangler layer"),
// operator-Schmidt factorisation of every rotated term across each tree link it
// crosses (minimal TPO bonds), block slots per link, and per-node plans for the
// matvec (Sec. 3.3.2, cost in Sec. 4.4.2) and the effective-operator updates (Sec. 3.3.2).
#include "model.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <set>
#include <unordered_map>

namespace attn {

int mask_popcount(uint32_t m) { return __builtin_popcount(m); }

int Tree::dim_of(int k) const {
  if (k == N) return 1;
  auto capped = [&](int e) {
    long long v = 1;
    for (int i = 0; i < e; i++) {
      v *= d;
      if (v > m) return (long long)m + 1;
    }
    return v;
  };
  return (int)std::min<long long>(m, std::min(capped(k), capped(N - k)));
}

int Tree::edge_upper(int e) const { return e < N ? site_parent[e] : nodes[e - N].parent; }

namespace {

// ------------------------------------------------------------------ small dense algebra
int ipow(int b, int e) {
  int v = 1;
  for (int i = 0; i < e; i++) v *= b;
  return v;
}

// One-sided Jacobi SVD (Hestenes) of the r x c row-major matrix A:
// A = U diag(s) V^T, k = min(r, c) columns, singular values descending.
void svd(const std::vector<double>& A, int r, int c, std::vector<double>& U,
         std::vector<double>& s, std::vector<double>& V) {
  if (r < c) {
    std::vector<double> At((size_t)r * c);
    for (int i = 0; i < r; i++)
      for (int j = 0; j < c; j++) At[(size_t)j * r + i] = A[(size_t)i * c + j];
    svd(At, c, r, V, s, U);   // A^T = V' s U'^T  =>  A = U' s V'^T
    return;
  }
  // columns of W (r x c) stored contiguously
  std::vector<double> W((size_t)r * c), Vc((size_t)c * c, 0.0);
  for (int i = 0; i < r; i++)
    for (int j = 0; j < c; j++) W[(size_t)j * r + i] = A[(size_t)i * c + j];
  for (int j = 0; j < c; j++) Vc[(size_t)j * c + j] = 1.0;
  for (int sweep = 0; sweep < 80; sweep++) {
    double off = 0.0;
    for (int p = 0; p < c; p++)
      for (int q = p + 1; q < c; q++) {
        double* wp = &W[(size_t)p * r];
        double* wq = &W[(size_t)q * r];
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < r; i++) {
          a += wp[i] * wp[i];
          b += wq[i] * wq[i];
          g += wp[i] * wq[i];
        }
        if (a == 0.0 || b == 0.0 || g == 0.0) continue;
        double rel = std::fabs(g) / std::sqrt(a * b);
        if (rel <= 1e-16) continue;
        off = std::max(off, rel);
        double zeta = (b - a) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < r; i++) {
          double x = wp[i], y = wq[i];
          wp[i] = cs * x - sn * y;
          wq[i] = sn * x + cs * y;
        }
        double* vp = &Vc[(size_t)p * c];
        double* vq = &Vc[(size_t)q * c];
        for (int i = 0; i < c; i++) {
          double x = vp[i], y = vq[i];
          vp[i] = cs * x - sn * y;
          vq[i] = sn * x + cs * y;
        }
      }
    if (off < 1e-15) break;
  }
  std::vector<int> order(c);
  std::vector<double> nrm(c);
  for (int j = 0; j < c; j++) {
    double a = 0;
    for (int i = 0; i < r; i++) a += W[(size_t)j * r + i] * W[(size_t)j * r + i];
    nrm[j] = std::sqrt(a);
    order[j] = j;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  U.assign((size_t)r * c, 0.0);
  V.assign((size_t)c * c, 0.0);
  s.assign(c, 0.0);
  for (int k = 0; k < c; k++) {
    int j = order[k];
    s[k] = nrm[j];
    for (int i = 0; i < r; i++) U[(size_t)i * c + k] = nrm[j] > 0 ? W[(size_t)j * r + i] / nrm[j] : 0.0;
    for (int i = 0; i < c; i++) V[(size_t)i * c + k] = Vc[(size_t)j * c + i];
  }
}

// positions (bit indices) of a mask in increasing order
std::vector<int> bits_of(uint32_t m) {
  std::vector<int> p;
  for (int i = 0; i < 32; i++)
    if (m & (1u << i)) p.push_back(i);
  return p;
}

// index of the operator-vector layout over mask `sub` from per-position
// out/in digits
inline int compose(const std::vector<int>& P, const int* od, const int* id, int d) {
  int x = 0;
  for (int p : P) x = x * d + od[p];
  for (int p : P) x = x * d + id[p];
  return x;
}

// For every index e of the layout over `U`, the index over each part (parts
// partition U; an empty part maps to 0).
void index_maps(int s, int d, uint32_t U, const std::vector<uint32_t>& parts,
                std::vector<std::vector<int>>& maps) {
  std::vector<int> PU = bits_of(U);
  int k = (int)PU.size();
  int len = ipow(d, 2 * k);
  maps.assign(parts.size(), std::vector<int>(len, 0));
  std::vector<std::vector<int>> Pp;
  for (uint32_t m : parts) Pp.push_back(bits_of(m));
  int od[32] = {0}, id[32] = {0};
  for (int e = 0; e < len; e++) {
    int x = e;
    for (int t = k - 1; t >= 0; t--) { id[PU[t]] = x % d; x /= d; }
    for (int t = k - 1; t >= 0; t--) { od[PU[t]] = x % d; x /= d; }
    for (size_t q = 0; q < parts.size(); q++) maps[q][e] = compose(Pp[q], od, id, d);
  }
  (void)s;
}

// Realign h over S into (K | S \ K): rows over K's layout, columns over the rest.
std::vector<double> realign(const RTerm& T, uint32_t K, int d) {
  int s = (int)T.S.size();
  uint32_t full = (s == 32) ? 0xffffffffu : ((1u << s) - 1);
  uint32_t C = full ^ K;
  std::vector<int> PK = bits_of(K), PC = bits_of(C);
  int lenK = ipow(d, 2 * (int)PK.size()), lenC = ipow(d, 2 * (int)PC.size());
  int D = ipow(d, s);
  std::vector<double> A((size_t)lenK * lenC, 0.0);
  int od[32], id[32];
  for (int o = 0; o < D; o++) {
    int x = o;
    for (int t = s - 1; t >= 0; t--) { od[t] = x % d; x /= d; }
    for (int i = 0; i < D; i++) {
      int y = i;
      for (int t = s - 1; t >= 0; t--) { id[t] = y % d; y /= d; }
      A[(size_t)compose(PK, od, id, d) * lenC + compose(PC, od, id, d)] = T.h[(size_t)o * D + i];
    }
  }
  return A;
}

const double kRankTol = 1e-12;   // singular values kept: > kRankTol * largest
const double kCoefTol = 1e-13;   // coupling entries dropped: <= kCoefTol * largest

const Split& get_split(RTerm& T, uint32_t A, int d) {
  uint32_t K = (A & 1u) ? A : (((1u << T.S.size()) - 1) ^ A);
  auto it = T.splits.find(K);
  if (it != T.splits.end()) return it->second;
  Split sp;
  sp.K = K;
  int s = (int)T.S.size();
  uint32_t C = ((1u << s) - 1) ^ K;
  sp.lenK = ipow(d, 2 * mask_popcount(K));
  sp.lenC = ipow(d, 2 * mask_popcount(C));
  std::vector<double> A2 = realign(T, K, d), U, sv, V;
  svd(A2, sp.lenK, sp.lenC, U, sv, V);
  int kmax = (int)sv.size();
  int t = 0;
  while (t < kmax && sv[t] > kRankTol * sv[0]) t++;
  if (sv.empty() || sv[0] == 0.0) t = 0;
  sp.t = t;
  sp.sigma.assign(sv.begin(), sv.begin() + t);
  sp.X.resize((size_t)t * sp.lenK);
  sp.Y.resize((size_t)t * sp.lenC);
  for (int k = 0; k < t; k++) {
    for (int i = 0; i < sp.lenK; i++) sp.X[(size_t)k * sp.lenK + i] = U[(size_t)i * kmax + k];
    for (int i = 0; i < sp.lenC; i++) sp.Y[(size_t)k * sp.lenC + i] = V[(size_t)i * kmax + k];
  }
  return T.splits.emplace(K, std::move(sp)).first->second;
}

// Orthonormal operator basis on the side A of the bipartition {A, S \ A}.
struct Basis {
  int t = 1, len = 1;
  std::vector<double> v{1.0};   // trivial basis: the scalar 1 (empty side)
  std::vector<double> sigma{1.0};
};

Basis side_basis(RTerm& T, uint32_t A, int d) {
  Basis b;
  if (A == 0) return b;
  const Split& sp = get_split(T, A, d);
  b.t = sp.t;
  if (A == sp.K) {
    b.len = sp.lenK;
    b.v = sp.X;
  } else {
    b.len = sp.lenC;
    b.v = sp.Y;
  }
  b.sigma = sp.sigma;
  return b;
}

// <P_a (x) Q_b (x) R_c, V> for all (a, b, c); parts partition U.
std::vector<double> couplings3(int s, int d, uint32_t mp, const Basis& P, uint32_t mq,
                               const Basis& Q, uint32_t mr, const Basis& R, const double* V) {
  uint32_t U = mp | mq | mr;
  std::vector<std::vector<int>> maps;
  index_maps(s, d, U, {mp, mq, mr}, maps);
  int len = (int)maps[0].size();
  std::vector<double> G((size_t)P.t * Q.t * R.t, 0.0);
  for (int a = 0; a < P.t; a++)
    for (int b = 0; b < Q.t; b++)
      for (int c = 0; c < R.t; c++) {
        double acc = 0;
        const double* pa = &P.v[(size_t)a * P.len];
        const double* qb = &Q.v[(size_t)b * Q.len];
        const double* rc = &R.v[(size_t)c * R.len];
        for (int e = 0; e < len; e++) acc += pa[maps[0][e]] * qb[maps[1][e]] * rc[maps[2][e]] * V[e];
        G[((size_t)a * Q.t + b) * R.t + c] = acc;
      }
  return G;
}

double max_abs(const std::vector<double>& v) {
  double m = 0;
  for (double x : v) m = std::max(m, std::fabs(x));
  return m;
}

}  // namespace

// Disentanglers contracted into one term (Sec. 4.3, algorithm "Contract
// disentangler layer"): S = the term's sites plus the partner sites of every
// gate that touches them (sorted), H = U^T (h (x) 1) U on S with U the product
// of those gates; tdense is the term's dense operator on its own site order.
attn_status rotate_term_dense(const std::vector<int>& tsites_t, const std::vector<double>& tdense_t, int d,
                              const std::vector<int>& de_of, const int32_t* de_sites, const double* de_u,
                              std::vector<int>& S_out, std::vector<double>& H_out, std::string& err) {
  const int dd = d * d;
    std::vector<int> S = tsites_t;
    std::vector<int> touch;
    for (int s : tsites_t)
      if (de_of[s] >= 0 && std::find(touch.begin(), touch.end(), de_of[s]) == touch.end()) touch.push_back(de_of[s]);
    for (int k : touch)
      for (int q = 0; q < 2; q++) {
        int x = de_sites[2 * k + q];
        if (std::find(S.begin(), S.end(), x) == S.end()) S.push_back(x);
      }
    if (S.size() > 6) { err = "rotated term support beyond 6 sites"; return ATTN_ERR_UNSUPPORTED; }
    std::sort(S.begin(), S.end());
    int s = (int)S.size();
    int D = ipow(d, s);
    // the original term embedded on S
    int k0 = (int)tsites_t.size();
    int D0 = ipow(d, k0);
    std::vector<int> tpos(k0);
    for (int i = 0; i < k0; i++) tpos[i] = (int)(std::find(S.begin(), S.end(), tsites_t[i]) - S.begin());
    auto digits = [&](int x, int* dg) { for (int q = s - 1; q >= 0; q--) { dg[q] = x % d; x /= d; } };
    std::vector<double> H((size_t)D * D, 0.0);
    int od[8], id[8];
    for (int o = 0; o < D; o++) {
      digits(o, od);
      for (int i = 0; i < D; i++) {
        digits(i, id);
        bool ok = true;
        for (int q = 0; q < s && ok; q++)
          if (std::find(tpos.begin(), tpos.end(), q) == tpos.end() && od[q] != id[q]) ok = false;
        if (!ok) continue;
        int ro = 0, ri = 0;
        for (int q = 0; q < k0; q++) { ro = ro * d + od[tpos[q]]; ri = ri * d + id[tpos[q]]; }
        H[(size_t)o * D + i] = tdense_t[(size_t)ro * D0 + ri];
      }
    }
    // U = product of the touching gates embedded on S; h' = U^T H U
    for (int k : touch) {
      int a = (int)(std::find(S.begin(), S.end(), de_sites[2 * k]) - S.begin());
      int b = (int)(std::find(S.begin(), S.end(), de_sites[2 * k + 1]) - S.begin());
      const double* u = de_u + (size_t)k * dd * dd;
      // G = embed(u): G[o][i] = u[(o_a o_b)][(i_a i_b)] prod_{q != a, b} delta(o_q, i_q)
      auto apply_right = [&](std::vector<double>& X) {   // X <- X G
        std::vector<double> Y((size_t)D * D, 0.0);
        for (int i = 0; i < D; i++) {
          digits(i, id);
          for (int xa = 0; xa < d; xa++)
            for (int xb = 0; xb < d; xb++) {
              int o2[8];
              for (int q = 0; q < s; q++) o2[q] = id[q];
              o2[a] = xa; o2[b] = xb;
              int o = 0;
              for (int q = 0; q < s; q++) o = o * d + o2[q];
              double g = u[(xa * d + xb) * dd + (id[a] * d + id[b])];
              if (g == 0.0) continue;
              for (int r = 0; r < D; r++) Y[(size_t)r * D + i] += X[(size_t)r * D + o] * g;
            }
        }
        X.swap(Y);
      };
      apply_right(H);                  // H G
      // G^T (H G): transpose, right-multiply by G, transpose back
      std::vector<double> Ht((size_t)D * D);
      for (int i = 0; i < D; i++) for (int j = 0; j < D; j++) Ht[(size_t)j * D + i] = H[(size_t)i * D + j];
      apply_right(Ht);
      for (int i = 0; i < D; i++) for (int j = 0; j < D; j++) H[(size_t)j * D + i] = Ht[(size_t)i * D + j];
    }
  S_out = S;
  H_out = std::move(H);
  return ATTN_OK;
}

void svd_jacobi(const std::vector<double>& A, int r, int c, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& V) {
  svd(A, r, c, U, s, V);
}

// ====================================================================== build
attn_status build_model(const attn_problem* p, Model& M, std::string& err) {
  if (!p) { err = "problem is NULL"; return ATTN_ERR_ARG; }
  const int N = p->n_sites, d = p->d, m = p->m;
  if (N < 2 || d < 2 || m < 1) { err = "need n_sites >= 2, d >= 2, m >= 1"; return ATTN_ERR_ARG; }
  if (!p->leaf_order || (p->n_terms > 0 && (!p->term_nsites || !p->term_sites || !p->term_ops || !p->term_coef)) ||
      (p->n_de > 0 && (!p->de_sites || !p->de_u)) || p->n_terms < 0 || p->n_de < 0) {
    err = "NULL array or negative count";
    return ATTN_ERR_ARG;
  }
  // ---- leaf order
  Tree& tr = M.tree;
  tr.N = N; tr.m = m; tr.d = d;
  tr.leaf.assign(p->leaf_order, p->leaf_order + N);
  tr.pos.assign(N, -1);
  for (int i = 0; i < N; i++) {
    int s = tr.leaf[i];
    if (s < 0 || s >= N || tr.pos[s] != -1) { err = "leaf_order is not a permutation"; return ATTN_ERR_ARG; }
    tr.pos[s] = i;
  }
  // ---- disentanglers: sites, overlap, unitarity
  const int dd = d * d;
  std::vector<int> de_of(N, -1);
  for (int k = 0; k < p->n_de; k++) {
    int a = p->de_sites[2 * k], b = p->de_sites[2 * k + 1];
    if (a < 0 || a >= N || b < 0 || b >= N || a == b) { err = "disentangler site out of range"; return ATTN_ERR_ARG; }
    if (de_of[a] != -1 || de_of[b] != -1) { err = "a site belongs to two disentanglers"; return ATTN_ERR_DE_OVERLAP; }
    de_of[a] = de_of[b] = k;
    const double* u = p->de_u + (size_t)k * dd * dd;
    for (int i = 0; i < dd; i++)
      for (int j = 0; j < dd; j++) {
        double acc = 0;
        for (int r = 0; r < dd; r++) acc += u[r * dd + i] * u[r * dd + j];
        if (!std::isfinite(acc) || std::fabs(acc - (i == j ? 1.0 : 0.0)) > 1e-12) {
          err = "disentangler " + std::to_string(k) + " is not orthogonal";
          return ATTN_ERR_NOT_UNITARY;
        }
      }
  }
  // ---- terms
  std::vector<std::vector<int>> tsites(p->n_terms);
  std::vector<std::vector<double>> tdense(p->n_terms);
  {
    size_t off = 0;
    for (int t = 0; t < p->n_terms; t++) {
      int k = p->term_nsites[t];
      if (k < 1 || k > 4) { err = "term_nsites must be 1..4"; return ATTN_ERR_UNSUPPORTED; }
      for (int i = 0; i < k; i++) {
        int s = p->term_sites[off + i];
        if (s < 0 || s >= N) { err = "term site out of range"; return ATTN_ERR_ARG; }
        for (int j = 0; j < i; j++)
          if (p->term_sites[off + j] == s) { err = "repeated site in a term"; return ATTN_ERR_ARG; }
        tsites[t].push_back(s);
      }
      off += k;
    }
    size_t opoff = 0;
    for (int t = 0; t < p->n_terms; t++) {
      int k = (int)tsites[t].size();
      int D = ipow(d, k);
      std::vector<double> h(1, p->term_coef[t]);
      int cur = 1;
      for (int i = 0; i < k; i++) {
        const double* o = p->term_ops + opoff + (size_t)i * dd;
        std::vector<double> nh((size_t)cur * d * cur * d);
        for (int a = 0; a < cur; a++)
          for (int b = 0; b < cur; b++)
            for (int x = 0; x < d; x++)
              for (int y = 0; y < d; y++)
                nh[(size_t)(a * d + x) * (cur * d) + (b * d + y)] = h[(size_t)a * cur + b] * o[x * d + y];
        h.swap(nh);
        cur *= d;
      }
      opoff += (size_t)k * dd;
      for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++) {
          double x = h[(size_t)i * D + j], y = h[(size_t)j * D + i];
          if (!std::isfinite(x) || std::fabs(x - y) > 1e-12 * (1.0 + std::fabs(x))) {
            err = "term " + std::to_string(t) + " is not symmetric";
            return ATTN_ERR_NOT_HERMITIAN;
          }
        }
      tdense[t] = std::move(h);
    }
  }
  // ---- tree (balanced split, single root with a dimension-1 parent leg)
  tr.nodes.clear();
  tr.site_parent.assign(N, -1);
  tr.site_side.assign(N, 0);
  {
    struct Frame { int lo, hi; };
    std::function<int(int, int)> build = [&](int lo, int hi) -> int {
      if (hi - lo == 1) return -(tr.leaf[lo] + 1);
      int k = hi - lo, kl = (k + 1) / 2;
      int cl = build(lo, lo + kl);
      int cr = build(lo + kl, hi);
      Node n;
      n.lo = lo; n.mid = lo + kl; n.hi = hi;
      n.child[0] = cl; n.child[1] = cr;
      n.parent = -1; n.side = 0;
      n.dims[0] = tr.dim_of(kl); n.dims[1] = tr.dim_of(k - kl); n.dims[2] = tr.dim_of(k);
      int id = (int)tr.nodes.size();
      tr.nodes.push_back(n);
      for (int s2 = 0; s2 < 2; s2++) {
        int c = s2 == 0 ? cl : cr;
        if (c >= 0) { tr.nodes[c].parent = id; tr.nodes[c].side = s2; }
        else { tr.site_parent[-(c + 1)] = id; tr.site_side[-(c + 1)] = s2; }
      }
      return id;
    };
    build(0, N);
    tr.root = (int)tr.nodes.size() - 1;
  }
  for (const Node& n : tr.nodes)
    if ((long long)n.dims[2] > (long long)n.dims[0] * n.dims[1] ||
        (long long)n.dims[0] > (long long)n.dims[1] * n.dims[2] ||
        (long long)n.dims[1] > (long long)n.dims[0] * n.dims[2]) {
      err = "inconsistent bond dimensions";
      return ATTN_ERR_UNSUPPORTED;
    }
  // ---- strict placement restrictions (Sec. 6.1.1)
  if (p->flags & ATTN_DE_STRICT) {
    for (int t = 0; t < p->n_terms; t++) {
      std::set<int> ks;
      for (int s : tsites[t]) if (de_of[s] >= 0) ks.insert(de_of[s]);
      if (ks.size() > 1) { err = "term touches more than one disentangler"; return ATTN_ERR_DE_RESTRICTION; }
    }
    for (int k = 0; k < p->n_de; k++) {
      int pa = tr.pos[p->de_sites[2 * k]], pb = tr.pos[p->de_sites[2 * k + 1]];
      if (pa > pb) std::swap(pa, pb);
      int n = tr.root;
      while (true) {
        const Node& nd = tr.nodes[n];
        if (pb < nd.mid && nd.child[0] >= 0) n = nd.child[0];
        else if (pa >= nd.mid && nd.child[1] >= 0) n = nd.child[1];
        else break;
      }
      const Node& nd = tr.nodes[n];
      auto maxdim = [&](int k2) {
        long long a = 1, b = 1;
        for (int i = 0; i < k2 && a <= m; i++) a *= d;
        for (int i = 0; i < N - k2 && b <= m; i++) b *= d;
        return std::min(a, b);
      };
      if (maxdim(nd.mid - nd.lo) <= m || maxdim(nd.hi - nd.mid) <= m) {
        err = "disentangler supports an untruncated link";
        return ATTN_ERR_DE_RESTRICTION;
      }
    }
  }
  // ---- rotated terms: h' = U^T (h (x) 1) U on the support extended by the
  //      partner sites of the disentanglers that touch the term
  M.terms.assign(p->n_terms, RTerm());
  for (int t = 0; t < p->n_terms; t++) {
    std::vector<int> S;
    std::vector<double> H;
    if (attn_status st = rotate_term_dense(tsites[t], tdense[t], d, de_of, p->de_sites, p->de_u, S, H, err))
      return st;
    M.terms[t].S = S;
    M.terms[t].h = std::move(H);
  }
  // ---- compression of terms acting on the same sites (Sec. 6.2.2, closing
  //      paragraph): terms with the same support meet the same disentanglers,
  //      so their rotated operators live on the same extended support and are
  //      summed into one term before the factorisation, which then finds the
  //      minimal bonds of the sum (e.g. XX + YY + ZZ on a bond: one term of
  //      bond <= d^2 across any cut instead of three)
  if (p->flags & ATTN_COMPRESS_TERMS) {
    std::map<std::vector<int>, int> first;
    std::vector<RTerm> merged;
    for (int t = 0; t < p->n_terms; t++) {
      std::vector<int> key = tsites[t];
      std::sort(key.begin(), key.end());
      auto it = first.find(key);
      if (it == first.end()) {
        first[key] = (int)merged.size();
        merged.push_back(std::move(M.terms[t]));
      } else {
        RTerm& R = merged[it->second];
        for (size_t i = 0; i < R.h.size(); i++) R.h[i] += M.terms[t].h[i];
      }
    }
    M.terms.swap(merged);
  }
  // ---- crossing terms per edge, slots
  const int NE = tr.n_edges();
  M.cross.assign(NE, {});
  M.n_slots.assign(NE, 0);
  std::vector<std::unordered_map<int, int>> slot_of(NE);
  auto edge_mask = [&](int e, const RTerm& T) {
    int lo = tr.edge_lo(e), hi = tr.edge_hi(e);
    uint32_t mk = 0;
    for (size_t q = 0; q < T.S.size(); q++) {
      int ps = tr.pos[T.S[q]];
      if (ps >= lo && ps < hi) mk |= 1u << q;
    }
    return mk;
  };
  for (int t = 0; t < (int)M.terms.size(); t++) {
    RTerm& T = M.terms[t];
    uint32_t full = (1u << T.S.size()) - 1;
    std::set<int> edges;
    for (int s0 : T.S) {
      int e = s0;
      while (true) {
        uint32_t mk = edge_mask(e, T);
        if (mk == full) break;
        edges.insert(e);
        int up = tr.edge_upper(e);
        if (up == tr.root) break;
        e = tr.edge_of_node(up);
      }
    }
    for (int e : edges) {
      uint32_t mk = edge_mask(e, T);
      const Split& sp = get_split(T, mk, d);
      if (sp.t == 0) continue;   // zero term
      EdgeCross ec{t, mk, M.n_slots[e], sp.t};
      slot_of[e][t] = (int)M.cross[e].size();
      M.cross[e].push_back(ec);
      M.n_slots[e] += sp.t;
    }
  }
  // ---- site edges: constant blocks (E then the Schmidt operators), column-major
  M.has_local[0].assign(NE, 0);
  M.has_local[1].assign(NE, 0);
  M.site_blocks.assign(N, {});
  for (int s0 = 0; s0 < N; s0++) {
    std::vector<double>& B = M.site_blocks[s0];
    B.assign((size_t)(1 + M.n_slots[s0]) * dd, 0.0);
    for (int t = 0; t < (int)M.terms.size(); t++) {
      const RTerm& T = M.terms[t];
      if (T.S.size() == 1 && T.S[0] == s0) {
        for (int o = 0; o < d; o++)
          for (int i = 0; i < d; i++) B[(size_t)i * d + o] += T.h[(size_t)o * d + i];
        M.has_local[0][s0] = 1;
      }
    }
    for (const EdgeCross& ec : M.cross[s0]) {
      Basis b = side_basis(M.terms[ec.term], ec.mask, d);
      for (int k = 0; k < b.t; k++)
        for (int o = 0; o < d; o++)
          for (int i = 0; i < d; i++)
            B[(size_t)(1 + ec.slot0 + k) * dd + (size_t)i * d + o] = b.v[(size_t)k * b.len + o * d + i];
    }
  }

  auto ref_of = [&](int e, int dir, int term, int k) {
    auto it = slot_of[e].find(term);
    return BRef::store(e, dir, M.cross[e][it->second].slot0 + k);
  };
  auto masks3 = [&](int n, const RTerm& T, uint32_t& ml, uint32_t& mr, uint32_t& mp) {
    const Node& nd = tr.nodes[n];
    ml = mr = mp = 0;
    for (size_t q = 0; q < T.S.size(); q++) {
      int ps = tr.pos[T.S[q]];
      if (ps >= nd.lo && ps < nd.mid) ml |= 1u << q;
      else if (ps >= nd.mid && ps < nd.hi) mr |= 1u << q;
      else mp |= 1u << q;
    }
  };
  // terms relevant at node n: those crossing any of its three links
  auto terms_at = [&](int n) {
    std::set<int> ts;
    for (int sd = 0; sd < 2; sd++)
      for (const EdgeCross& ec : M.cross[tr.edge_of_child(n, sd)]) ts.insert(ec.term);
    if (n != tr.root)
      for (const EdgeCross& ec : M.cross[tr.edge_of_node(n)]) ts.insert(ec.term);
    return ts;
  };
  auto add_items = [&](std::vector<Item2>& items, std::vector<Combine>& combs, int spect,
                       const std::vector<BRef>& ra, const std::vector<BRef>& rb,
                       const std::vector<double>& G, int ta, int tb, int dimb) {
    // items for sum_{a,b} G[a][b] (A_a (x) B_b); several b per a are combined
    double gmax = max_abs(G);
    for (int a = 0; a < ta; a++) {
      std::vector<std::pair<int, double>> nz;
      for (int b = 0; b < tb; b++) {
        double g = G[(size_t)a * tb + b];
        if (std::fabs(g) > kCoefTol * gmax) nz.push_back({b, g});
      }
      if (nz.empty()) continue;
      if (nz.size() == 1 || rb[0].is_none()) {
        for (auto& z : nz) items.push_back({spect, ra[a], rb[z.first], z.second});
      } else {
        Combine c;
        c.dim = dimb;
        for (auto& z : nz) c.in.push_back({rb[z.first], z.second});
        combs.push_back(c);
        items.push_back({spect, ra[a], BRef::comb((int)combs.size() - 1), 1.0});
      }
    }
  };

  const int nn = (int)tr.nodes.size();
  M.env_up.assign(nn, EnvPlan());
  M.env_down[0].assign(nn, EnvPlan());
  M.env_down[1].assign(nn, EnvPlan());
  // ---- upward updates (post-order so that child flags are known)
  for (int q = 0; q < nn; q++) {
    if (q == tr.root) continue;
    const Node& nd = tr.nodes[q];
    int el = tr.edge_of_child(q, 0), er = tr.edge_of_child(q, 1), eo = tr.edge_of_node(q);
    EnvPlan& P = M.env_up[q];
    P.node = q; P.leg = 2; P.out_edge = eo; P.out_dir = 0;
    EnvOut E;
    E.slot = -1;
    if (M.has_local[0][el]) E.items.push_back({2, BRef::store(el, 0, -1), BRef::none(), 1.0});
    if (M.has_local[0][er]) E.items.push_back({2, BRef::none(), BRef::store(er, 0, -1), 1.0});
    for (int t : terms_at(q)) {
      RTerm& T = M.terms[t];
      uint32_t ml, mr, mp;
      masks3(q, T, ml, mr, mp);
      int s = (int)T.S.size();
      if (mp == 0 && ml && mr) {   // term confined to subtree(q), meeting both children
        Basis bl = side_basis(T, ml, d), br = side_basis(T, mr, d), one;
        std::vector<double> G = couplings3(s, d, ml, bl, mr, br, 0, one, T.h.data());
        std::vector<BRef> ra, rb;
        for (int a = 0; a < bl.t; a++) ra.push_back(ref_of(el, 0, t, a));
        for (int b = 0; b < br.t; b++) rb.push_back(ref_of(er, 0, t, b));
        add_items(E.items, P.combines, 2, ra, rb, G, bl.t, br.t, nd.dims[1]);
      }
    }
    M.has_local[0][eo] = !E.items.empty();
    P.outs.push_back(E);
    for (const EdgeCross& ec : M.cross[eo]) {
      RTerm& T = M.terms[ec.term];
      uint32_t ml, mr, mp;
      masks3(q, T, ml, mr, mp);
      int s = (int)T.S.size();
      Basis bl = side_basis(T, ml, d), br = side_basis(T, mr, d);
      Basis bo = side_basis(T, ml | mr, d);
      std::vector<BRef> ra, rb;
      for (int a = 0; a < bl.t; a++) ra.push_back(ml ? ref_of(el, 0, ec.term, a) : BRef::none());
      for (int b = 0; b < br.t; b++) rb.push_back(mr ? ref_of(er, 0, ec.term, b) : BRef::none());
      for (int c = 0; c < bo.t; c++) {
        Basis one_c;
        one_c.t = 1; one_c.len = bo.len;
        one_c.v.assign(bo.v.begin() + (size_t)c * bo.len, bo.v.begin() + (size_t)(c + 1) * bo.len);
        Basis one;
        std::vector<double> G = couplings3(s, d, ml, bl, mr, br, 0, one, one_c.v.data());
        EnvOut O;
        O.slot = ec.slot0 + c;
        add_items(O.items, P.combines, 2, ra, rb, G, bl.t, br.t, nd.dims[1]);
        P.outs.push_back(O);
      }
    }
  }
  // ---- downward updates (reverse post-order: parents first)
  for (int q = nn - 1; q >= 0; q--) {
    const Node& nd = tr.nodes[q];
    for (int sd = 0; sd < 2; sd++) {
      if (nd.child[sd] < 0) continue;   // sites carry no tensor
      int es = tr.edge_of_child(q, sd), eo_ = tr.edge_of_child(q, 1 - sd);
      int ep = q == tr.root ? -1 : tr.edge_of_node(q);
      EnvPlan& P = M.env_down[sd][q];
      P.node = q; P.leg = sd; P.out_edge = es; P.out_dir = 1;
      int dim_o = nd.dims[1 - sd], dim_p = nd.dims[2];
      EnvOut E;
      E.slot = -1;
      if (M.has_local[0][eo_]) E.items.push_back({sd, BRef::store(eo_, 0, -1), BRef::none(), 1.0});
      if (ep >= 0 && M.has_local[1][ep]) E.items.push_back({sd, BRef::none(), BRef::store(ep, 1, -1), 1.0});
      for (int t : terms_at(q)) {
        RTerm& T = M.terms[t];
        uint32_t m3[3];
        masks3(q, T, m3[0], m3[1], m3[2]);
        uint32_t ms = m3[sd], mo = m3[1 - sd], mpm = m3[2];
        int s = (int)T.S.size();
        if (ms == 0 && mo && mpm) {   // confined to the outside of the child, crossing q
          Basis bo = side_basis(T, mo, d);
          Basis bp = side_basis(T, mpm, d);   // orthonormal ops on the part above q
          std::vector<double> G = couplings3(s, d, mo, bo, mpm, bp, 0, Basis(), T.h.data());
          // the down store of edge(q) holds sigma_c * w_c: divide
          for (int b = 0; b < bo.t; b++)
            for (int c = 0; c < bp.t; c++) G[(size_t)b * bp.t + c] /= bp.sigma[c];
          std::vector<BRef> ra, rb;
          for (int b = 0; b < bo.t; b++) ra.push_back(ref_of(eo_, 0, t, b));
          for (int c = 0; c < bp.t; c++) rb.push_back(ref_of(ep, 1, t, c));
          add_items(E.items, P.combines, sd, ra, rb, G, bo.t, bp.t, dim_p);
        }
      }
      M.has_local[1][es] = !E.items.empty();
      P.outs.push_back(E);
      for (const EdgeCross& ec : M.cross[es]) {
        RTerm& T = M.terms[ec.term];
        uint32_t m3[3];
        masks3(q, T, m3[0], m3[1], m3[2]);
        uint32_t ms = m3[sd], mo = m3[1 - sd], mpm = m3[2];
        int s = (int)T.S.size();
        Basis bc = side_basis(T, mo | mpm, d);   // orthonormal ops on the child's outside
        Basis cs = side_basis(T, ms, d);        // for sigma of the child's split
        Basis bo = side_basis(T, mo, d);
        Basis bp = side_basis(T, mpm, d);
        std::vector<BRef> ra, rb;
        for (int b = 0; b < bo.t; b++) ra.push_back(mo ? ref_of(eo_, 0, ec.term, b) : BRef::none());
        for (int c = 0; c < bp.t; c++) rb.push_back(mpm ? ref_of(ep, 1, ec.term, c) : BRef::none());
        for (int a = 0; a < bc.t; a++) {
          Basis one_a;
          one_a.t = 1; one_a.len = bc.len;
          one_a.v.assign(bc.v.begin() + (size_t)a * bc.len, bc.v.begin() + (size_t)(a + 1) * bc.len);
          std::vector<double> G = couplings3(s, d, mo, bo, mpm, bp, 0, Basis(), one_a.v.data());
          for (int b = 0; b < bo.t; b++)
            for (int c = 0; c < bp.t; c++)
              G[(size_t)b * bp.t + c] *= cs.sigma[a] / (mpm ? bp.sigma[c] : 1.0);
          EnvOut O;
          O.slot = ec.slot0 + a;
          add_items(O.items, P.combines, sd, ra, rb, G, bo.t, bp.t, dim_p);
          P.outs.push_back(O);
        }
        (void)dim_o;
      }
    }
  }
  // ---- matvec plans
  M.mv.assign(nn, MatvecPlan());
  for (int n = 0; n < nn; n++) {
    const Node& nd = tr.nodes[n];
    MatvecPlan& P = M.mv[n];
    int el = tr.edge_of_child(n, 0), er = tr.edge_of_child(n, 1);
    int ep = n == tr.root ? -1 : tr.edge_of_node(n);
    const int64_t ml = nd.dims[0], mr = nd.dims[1], mpd = nd.dims[2];
    const int64_t Msz = ml * mr * mpd;
    const int64_t dm[3] = {ml, mr, mpd};
    if (M.has_local[0][el]) { P.items.push_back({1, BRef::store(el, 0, -1), BRef::none(), 1.0}); P.flops += 2 * ml * Msz; }
    if (M.has_local[0][er]) { P.items.push_back({0, BRef::store(er, 0, -1), BRef::none(), 1.0}); P.flops += 2 * mr * Msz; }
    if (ep >= 0 && M.has_local[1][ep]) { P.items.push_back({1, BRef::none(), BRef::store(ep, 1, -1), 1.0}); P.flops += 2 * mpd * Msz; }
    for (int t : terms_at(n)) {
      RTerm& T = M.terms[t];
      uint32_t m3[3];
      masks3(n, T, m3[0], m3[1], m3[2]);
      int present = (m3[0] ? 1 : 0) + (m3[1] ? 1 : 0) + (m3[2] ? 1 : 0);
      if (present < 2) continue;
      P.n_cross++;
      int s = (int)T.S.size();
      Basis b3[3];
      b3[0] = side_basis(T, m3[0], d);
      b3[1] = side_basis(T, m3[1], d);
      Basis bpw = side_basis(T, m3[2], d);   // orthonormal ops above n
      b3[2] = bpw;
      std::vector<double> G = couplings3(s, d, m3[0], b3[0], m3[1], b3[1], m3[2], b3[2], T.h.data());
      if (m3[2])
        for (int a = 0; a < b3[0].t; a++)
          for (int b = 0; b < b3[1].t; b++)
            for (int c = 0; c < b3[2].t; c++) G[((size_t)a * b3[1].t + b) * b3[2].t + c] /= bpw.sigma[c];
      std::vector<BRef> r3[3];
      for (int a = 0; a < b3[0].t; a++) r3[0].push_back(m3[0] ? ref_of(el, 0, t, a) : BRef::none());
      for (int b = 0; b < b3[1].t; b++) r3[1].push_back(m3[1] ? ref_of(er, 0, t, b) : BRef::none());
      for (int c = 0; c < b3[2].t; c++) r3[2].push_back(m3[2] ? ref_of(ep, 1, t, c) : BRef::none());
      if (present == 2) {
        int x, y, spect;
        if (!m3[0]) { spect = 0; x = 1; y = 2; }
        else if (!m3[1]) { spect = 1; x = 0; y = 2; }
        else { spect = 2; x = 0; y = 1; }
        // flatten G over (x, y) with the absent leg of size 1
        int tx = b3[x].t, ty = b3[y].t;
        std::vector<double> G2((size_t)tx * ty);
        for (int a = 0; a < tx; a++)
          for (int b = 0; b < ty; b++) {
            int idx[3] = {0, 0, 0};
            idx[x] = a; idx[y] = b;
            G2[(size_t)a * ty + b] = G[((size_t)idx[0] * b3[1].t + idx[1]) * b3[2].t + idx[2]];
          }
        add_items(P.items, P.combines, spect, r3[x], r3[y], G2, tx, ty, (int)dm[y]);
        uint32_t mx = m3[x];
        int tb = get_split(T, mx, d).t;
        P.flops += 2 * Msz * tb * (dm[x] + dm[y]);
      } else {
        // chain with the cheapest middle leg
        int t3[3];
        for (int j = 0; j < 3; j++) t3[j] = b3[j].t;
        int best = -1;
        int64_t bestc = 0;
        for (int mid = 0; mid < 3; mid++) {
          int o1 = mid == 0 ? 1 : 0, o2 = mid == 2 ? 1 : 2;
          int64_t c = t3[o1] * dm[o1] + (int64_t)t3[o1] * t3[o2] * dm[mid] + t3[o2] * dm[o2];
          if (best < 0 || c < bestc) { best = mid; bestc = c; }
        }
        P.flops += 2 * Msz * bestc;
        Chain ch;
        ch.mid = best;
        ch.o1 = best == 0 ? 1 : 0;
        ch.o2 = best == 2 ? 1 : 2;
        ch.O1 = r3[ch.o1];
        ch.O2 = r3[ch.o2];
        int t1 = t3[ch.o1], t2 = t3[ch.o2], tm = t3[best];
        double gmax = max_abs(G);
        for (int a = 0; a < t1; a++)
          for (int c = 0; c < t2; c++) {
            Combine cb;
            cb.dim = (int)dm[best];
            for (int b = 0; b < tm; b++) {
              int idx[3];
              idx[ch.o1] = a; idx[ch.o2] = c; idx[best] = b;
              double g = G[((size_t)idx[0] * t3[1] + idx[1]) * t3[2] + idx[2]];
              if (std::fabs(g) > kCoefTol * gmax) cb.in.push_back({r3[best][b], g});
            }
            if (cb.in.empty()) { ch.Mid.push_back(BRef::zero()); continue; }
            P.combines.push_back(cb);
            ch.Mid.push_back(BRef::comb((int)P.combines.size() - 1));
          }
        P.chains.push_back(ch);
      }
    }
  }
  // ---- the root's parent leg has dimension 1: an item with no operator on it
  //      is the same contraction with p as the (single-slice) spectator, which
  //      keeps both contracted legs at full size
  auto to_spect_p = [](Item2& it) {
    if (it.spect == 2 || !it.B.is_none()) return;
    if (it.spect == 0) { it.B = it.A; it.A = BRef::none(); }   // op on r
    it.spect = 2;                                             // spect 1: op on l stays A
  };
  if (tr.nodes[tr.root].dims[2] == 1) {
    for (Item2& it : M.mv[tr.root].items) to_spect_p(it);
    for (int sd = 0; sd < 2; sd++)
      for (EnvOut& o : M.env_down[sd][tr.root].outs)
        for (Item2& it : o.items) to_spect_p(it);
  }
  return ATTN_OK;
}

}  // namespace attn
