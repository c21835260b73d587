// Observables of the augmented state (Sec. 5) and the MERA-like optimisation
// of the disentangler layer (Sec. 4.1.1, 4.2), both built on one device
// engine: expectation values <psi_TTN| prod_s A_s |psi_TTN> of many products
// of one-site operators, with the isometry centre at the root.
//
// Engine (all FP64, launches of measure_kernels.hip):
//  * image of the factors below a link: at the link above node q,
//    R = T_q^T (R_l (x) R_r) T_q with R_l / R_r the images on q's child links
//    (a site link carries the operator itself, a factor-free side the
//    identity); images are shared between products by content and computed
//    level by level from the leaves up;
//  * Gram matrix of every link from above, G_child = sum T G_p T^T over the
//    other two legs, from the root (G = 1 above it) down;
//  * at the lowest node n holding all factors of a product, with the left
//    image R_l and right image R_r: <P> = <R_l^T x_l T_n, R_r x_r (G_p x_p T_n)>,
//    all pairs of a node's left and right images in one product of the two
//    stacked lists (split over the summed index, partials summed in order).
#include <array>
#include <map>

#include "measure.hpp"
#include "runtime.hpp"

using namespace attn;
using namespace rt;

namespace {

struct Buf {
  std::vector<void*> ptrs;
  double* get(int64_t n) {
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<int64_t>(n, 1) * sizeof(double)));
    ptrs.push_back(p);
    return (double*)p;
  }
  ~Buf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

template <typename T>
T* upload_tmp(Buf& b, const std::vector<T>& v) {
  double* p = b.get((int64_t)((v.size() * sizeof(T) + 7) / 8));
  HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return (T*)p;
}

// GEMM jobs of one launch and their work units
struct GemmList {
  std::vector<GMJob> jobs;
  std::vector<int4> wus;
  void add(const GMJob& j, int batch) {
    const int id = (int)jobs.size();
    jobs.push_back(j);
    const int tm = (j.M + 63) / 64, tn = (j.N + 63) / 64;
    for (int b = 0; b < batch; b++)
      for (int x = 0; x < tm; x++)
        for (int y = 0; y < tn; y++) wus.push_back(int4{id, b, x, y});
  }
  void run(Buf& buf, hipStream_t s) {
    if (jobs.empty()) return;
    GMJob* dj = upload_tmp(buf, jobs);
    int4* dw = upload_tmp(buf, wus);
    HIPCHK(launch_gemm_jobs(dj, dw, (int)wus.size(), s));
    jobs.clear();
    wus.clear();
  }
};

GMJob gm(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc, int ta = 0,
         int tb = 0, int64_t sa = 0, int64_t sb = 0, int64_t sc = 0) {
  GMJob j;
  j.A = A; j.B = B; j.C = C;
  j.sa = sa; j.sb = sb; j.sc = sc;
  j.M = M; j.N = N; j.K = K;
  j.lda = lda; j.ldb = ldb; j.ldc = ldc;
  j.ta = ta; j.tb = tb;
  j.accumulate = 0; j.pad = 0;
  return j;
}

}  // namespace

namespace rt {

// A product of one-site operators: (site, operator id), sites distinct.
struct XProd {
  std::vector<std::pair<int, int>> f;
};

struct XEngine {
  attn_handle* h;
  int d;
  std::vector<double> ops;   // d x d row-major per operator id
  std::map<std::vector<double>, int> op_ids;

  explicit XEngine(attn_handle* hh) : h(hh), d(hh->M.tree.d) {}

  int op_id(const double* m) {
    std::vector<double> key(m, m + d * d);
    auto it = op_ids.find(key);
    if (it != op_ids.end()) return it->second;
    const int id = (int)(ops.size() / (d * d));
    ops.insert(ops.end(), key.begin(), key.end());
    op_ids.emplace(std::move(key), id);
    return id;
  }

  struct Img {
    int edge, node, opid, left, right, dim;
    double* dev;
  };

  void run(const std::vector<XProd>& prods, std::vector<double>& out, hipStream_t s);
};

void XEngine::run(const std::vector<XProd>& prods, std::vector<double>& out, hipStream_t s) {
  const Tree& tr = h->M.tree;
  const int nn = (int)tr.nodes.size();
  const int dd = d * d;
  out.assign(prods.size(), 0.0);
  if (prods.empty()) return;
  Buf buf;
  double* d_ops = upload_tmp(buf, ops.empty() ? std::vector<double>(1, 0.0) : ops);
  auto Tptr = [&](int n) { return h->d_T + h->T_off[n]; };

  // ---- images (content-keyed) and, per product, its lowest common node
  std::vector<Img> imgs;
  std::map<std::pair<int, std::vector<std::pair<int, int>>>, int> memo;
  std::function<int(int, const std::vector<std::pair<int, int>>&)> image =
      [&](int edge, const std::vector<std::pair<int, int>>& fs) -> int {
    auto key = std::make_pair(edge, fs);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    Img im;
    im.edge = edge;
    im.dev = nullptr;
    if (tr.edge_is_site(edge)) {
      if (fs.size() != 1) throw StatusFail{ATTN_ERR_ARG, "internal: several factors on one site"};
      im.node = -1;
      im.opid = fs[0].second;
      im.left = im.right = -1;
      im.dim = d;
    } else {
      const int q = edge - tr.N;
      const Node& nd = tr.nodes[q];
      std::vector<std::pair<int, int>> fl, fr;
      for (auto& x : fs) (tr.pos[x.first] < nd.mid ? fl : fr).push_back(x);
      im.node = q;
      im.opid = -1;
      im.left = fl.empty() ? -1 : image(tr.edge_of_child(q, 0), fl);
      im.right = fr.empty() ? -1 : image(tr.edge_of_child(q, 1), fr);
      im.dim = nd.dims[2];
    }
    const int id = (int)imgs.size();
    imgs.push_back(im);
    memo.emplace(std::move(key), id);
    return id;
  };
  struct Eval {
    std::vector<int> L, R;   // distinct image ids (-1 = identity)
    std::map<int, int> li, ri;
  };
  std::map<int, Eval> evals;
  std::vector<std::array<int, 3>> where(prods.size());   // (node, left index, right index)
  for (size_t p = 0; p < prods.size(); p++) {
    std::vector<std::pair<int, int>> fs = prods[p].f;
    if (fs.empty()) throw StatusFail{ATTN_ERR_ARG, "empty product"};
    std::sort(fs.begin(), fs.end());
    for (size_t i = 1; i < fs.size(); i++)
      if (fs[i].first == fs[i - 1].first) throw StatusFail{ATTN_ERR_ARG, "repeated site in a product"};
    int n = tr.root;
    while (true) {
      const Node& nd = tr.nodes[n];
      bool all_l = true, all_r = true;
      for (auto& x : fs) {
        if (tr.pos[x.first] < nd.mid) all_r = false;
        else all_l = false;
      }
      if (all_l && nd.child[0] >= 0) { n = nd.child[0]; continue; }
      if (all_r && nd.child[1] >= 0) { n = nd.child[1]; continue; }
      break;
    }
    const Node& nd = tr.nodes[n];
    std::vector<std::pair<int, int>> fl, fr;
    for (auto& x : fs) (tr.pos[x.first] < nd.mid ? fl : fr).push_back(x);
    const int il = fl.empty() ? -1 : image(tr.edge_of_child(n, 0), fl);
    const int ir = fr.empty() ? -1 : image(tr.edge_of_child(n, 1), fr);
    Eval& ev = evals[n];
    if (!ev.li.count(il)) { ev.li[il] = (int)ev.L.size(); ev.L.push_back(il); }
    if (!ev.ri.count(ir)) { ev.ri[ir] = (int)ev.R.size(); ev.R.push_back(ir); }
    where[p] = {n, ev.li[il], ev.ri[ir]};
  }

  // ---- image storage; site images point into the operator table
  {
    int64_t tot = 0;
    for (auto& im : imgs)
      if (im.node >= 0) tot += (int64_t)im.dim * im.dim;
    double* store = buf.get(tot);
    int64_t off = 0;
    for (auto& im : imgs) {
      if (im.node >= 0) { im.dev = store + off; off += (int64_t)im.dim * im.dim; }
      else im.dev = d_ops + (int64_t)im.opid * dd;
    }
  }
  // node heights (a node above two sites has height 1)
  std::vector<int> height(nn, 0), depth(nn, 0);
  int hmax = 0, dmax = 0;
  for (int n = 0; n < nn; n++) {   // post-order: children first
    int hh = 0;
    for (int sd = 0; sd < 2; sd++)
      if (tr.nodes[n].child[sd] >= 0) hh = std::max(hh, height[tr.nodes[n].child[sd]]);
    height[n] = hh + 1;
    hmax = std::max(hmax, height[n]);
  }
  for (int n = nn - 1; n >= 0; n--) {   // reverse post-order: parents first
    const int p = tr.nodes[n].parent;
    depth[n] = p < 0 ? 0 : depth[p] + 1;
    dmax = std::max(dmax, depth[n]);
  }
  const int64_t kScratch = (int64_t)1 << 25;   // doubles of intermediate tensors per launch group
  // ---- images, level by level from the leaves
  for (int lev = 1; lev <= hmax; lev++) {
    std::vector<int> todo;
    for (int i = 0; i < (int)imgs.size(); i++)
      if (imgs[i].node >= 0 && height[imgs[i].node] == lev) todo.push_back(i);
    size_t k = 0;
    while (k < todo.size()) {
      std::vector<int> chunk;
      int64_t need = 0;
      while (k < todo.size()) {
        const Node& nd = tr.nodes[imgs[todo[k]].node];
        const int64_t M = (int64_t)nd.dims[0] * nd.dims[1] * nd.dims[2];
        if (!chunk.empty() && need + 2 * M > kScratch) break;
        need += 2 * M;
        chunk.push_back(todo[k++]);
      }
      Buf lb;   // freed (after the device has finished with it) at the end of the chunk
      double* z = lb.get(need);
      GemmList ga, gb, gc;
      int64_t off = 0;
      for (int i : chunk) {
        const Img& im = imgs[i];
        const Node& nd = tr.nodes[im.node];
        const int dl = nd.dims[0], dr = nd.dims[1], dp = nd.dims[2];
        const int64_t M = (int64_t)dl * dr * dp;
        double* z1 = z + off;
        double* z2 = z + off + M;
        off += 2 * M;
        const double* T = Tptr(im.node);
        const double* cur = T;
        if (im.right >= 0) {
          ga.add(gm(imgs[im.right].dev, T, z1, dr, dp, dr, dr, dp, dp, 0, 0, 0, (int64_t)dr * dp, (int64_t)dr * dp), dl);
          cur = z1;
        }
        if (im.left >= 0) {
          gb.add(gm(imgs[im.left].dev, cur, z2, dl, dr * dp, dl, dl, dr * dp, dr * dp), 1);
          cur = z2;
        }
        gc.add(gm(T, cur, im.dev, dp, dp, dl * dr, dp, dp, dp, 1, 0), 1);
      }
      ga.run(lb, s);
      gb.run(lb, s);
      gc.run(lb, s);
    }
  }
  // ---- Gram matrices of the parent links, from the root down
  std::vector<double*> G(nn, nullptr);
  std::vector<double*> W(nn, nullptr);   // T_n x_p G_p, kept for the closing products
  {
    int64_t gtot = 0;
    for (int n = 0; n < nn; n++) gtot += (int64_t)tr.nodes[n].dims[2] * tr.nodes[n].dims[2];
    double* gs = buf.get(gtot);
    int64_t off = 0;
    for (int n = 0; n < nn; n++) { G[n] = gs + off; off += (int64_t)tr.nodes[n].dims[2] * tr.nodes[n].dims[2]; }
    const double one = 1.0;
    HIPCHK(hipMemcpy(G[tr.root], &one, sizeof(double), hipMemcpyHostToDevice));
  }
  for (int dep = 0; dep <= dmax; dep++) {
    std::vector<int> lvl;
    for (int n = 0; n < nn; n++)
      if (depth[n] == dep) lvl.push_back(n);
    GemmList gw, gg;
    std::vector<PMJob> pm;
    int64_t maxM = 0;
    Buf lb;
    for (int n : lvl) {
      const Node& nd = tr.nodes[n];
      const int dl = nd.dims[0], dr = nd.dims[1], dp = nd.dims[2];
      const int64_t M = (int64_t)dl * dr * dp;
      const bool need_down = nd.child[0] >= 0 || nd.child[1] >= 0;
      if (!need_down && !evals.count(n)) continue;
      W[n] = buf.get(M);
      gw.add(gm(Tptr(n), G[n], W[n], dl * dr, dp, dp, dp, dp, dp, 0, 1), 1);
      if (nd.child[0] >= 0) gg.add(gm(Tptr(n), W[n], G[nd.child[0]], dl, dl, dr * dp, dr * dp, dr * dp, dl, 0, 1), 1);
      if (nd.child[1] >= 0) {
        double* tp = lb.get(M);
        double* wp = lb.get(M);
        pm.push_back(PMJob{Tptr(n), tp, dl, dr, dp, 0});
        pm.push_back(PMJob{W[n], wp, dl, dr, dp, 0});
        maxM = std::max(maxM, M);
        gg.add(gm(tp, wp, G[nd.child[1]], dr, dr, dl * dp, dl * dp, dl * dp, dr, 0, 1), 1);
      }
    }
    gw.run(lb, s);
    if (!pm.empty()) {
      PMJob* dpm = upload_tmp(lb, pm);
      HIPCHK(launch_permute_jobs(dpm, (int)pm.size(), maxM, s));
    }
    gg.run(lb, s);
  }
  // ---- closing products at every lowest common node.  The needed (left,
  // right) pairs of a node are evaluated either as all pairs of two stacked
  // lists (one matrix product, when most pairs are needed) or pair by pair
  // (when the images are specific to single products); the stacked images
  // are formed in groups that fit kUVBudget doubles.
  const int64_t kUVBudget = (int64_t)1 << 28;
  std::map<int, std::map<std::pair<int, int>, double>> vals;
  std::map<int, std::vector<std::pair<int, int>>> needed;
  for (size_t p = 0; p < prods.size(); p++) needed[where[p][0]].push_back({where[p][1], where[p][2]});
  for (auto& kv : needed) {
    std::sort(kv.second.begin(), kv.second.end());
    kv.second.erase(std::unique(kv.second.begin(), kv.second.end()), kv.second.end());
  }
  for (auto& kv : evals) {
    const int n = kv.first;
    const Eval& ev = kv.second;
    const Node& nd = tr.nodes[n];
    const int dl = nd.dims[0], dr = nd.dims[1], dp = nd.dims[2];
    const int64_t M = (int64_t)dl * dr * dp;
    const int nl = (int)ev.L.size(), nr = (int)ev.R.size();
    const std::vector<std::pair<int, int>>& pairs = needed[n];
    std::map<std::pair<int, int>, double>& out_n = vals[n];
    Buf nb;   // this node's stacked images and partials
    // U_i = R_l^T x_l T (or T), V_j = R_r x_r W (or W), written at given addresses
    auto make_u = [&](GemmList& g, int i, double* dst) {
      if (ev.L[i] < 0) HIPCHK(launch_copy(dst, Tptr(n), M, s));
      else g.add(gm(imgs[ev.L[i]].dev, Tptr(n), dst, dl, dr * dp, dl, dl, dr * dp, dr * dp, 1, 0), 1);
    };
    auto make_v = [&](GemmList& g, int j, double* dst) {
      if (ev.R[j] < 0) HIPCHK(launch_copy(dst, W[n], M, s));
      else
        g.add(gm(imgs[ev.R[j]].dev, W[n], dst, dr, dp, dr, dr, dp, dp, 0, 0, 0, (int64_t)dr * dp, (int64_t)dr * dp),
              dl);
    };
    const int64_t cap = std::max<int64_t>(2, kUVBudget / M);   // stacked vectors held at once
    if ((int64_t)nl * nr <= 4 * (int64_t)pairs.size()) {
      // all pairs: C (nl x nr) block by block
      const int cl = (int)std::max<int64_t>(1, std::min<int64_t>(nl, cap / 2));
      const int cr = (int)std::max<int64_t>(1, std::min<int64_t>(nr, cap - cl));
      double* U = nb.get((int64_t)cl * M);
      double* V = nb.get((int64_t)cr * M);
      std::vector<double> Cn((size_t)nl * nr);
      for (int i0 = 0; i0 < nl; i0 += cl) {
        const int ml = std::min(cl, nl - i0);
        GemmList gu;
        for (int i = 0; i < ml; i++) make_u(gu, i0 + i, U + (int64_t)i * M);
        gu.run(nb, s);
        for (int j0 = 0; j0 < nr; j0 += cr) {
          const int mr = std::min(cr, nr - j0);
          GemmList gv;
          for (int j = 0; j < mr; j++) make_v(gv, j0 + j, V + (int64_t)j * M);
          gv.run(nb, s);
          const int64_t tiles = (int64_t)((ml + 63) / 64) * ((mr + 63) / 64);
          int nq = (int)std::max<int64_t>(1, std::min<int64_t>({256, M / 2048, std::max<int64_t>(1, 1024 / tiles)}));
          const int64_t kc = (M + nq - 1) / nq;
          nq = (int)((M + kc - 1) / kc);
          double* part = nb.get((int64_t)nq * ml * mr);
          double* Cb = nb.get((int64_t)ml * mr);
          GemmList gp;
          for (int q = 0; q < nq; q++) {
            const int64_t k0 = (int64_t)q * kc;
            const int K = (int)std::min<int64_t>(kc, M - k0);
            gp.add(gm(U + k0, V + k0, part + (int64_t)q * ml * mr, ml, mr, K, (int)M, (int)M, mr, 0, 1), 1);
          }
          gp.run(nb, s);
          std::vector<SPJob> sp(1, SPJob{part, Cb, (int64_t)ml * mr, (int64_t)ml * mr, nq, 0});
          SPJob* dsp = upload_tmp(nb, sp);
          HIPCHK(launch_sum_parts(dsp, 1, (int64_t)ml * mr, s));
          std::vector<double> hb((size_t)ml * mr);
          HIPCHK(hipMemcpyAsync(hb.data(), Cb, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          for (int i = 0; i < ml; i++)
            for (int j = 0; j < mr; j++) Cn[(size_t)(i0 + i) * nr + j0 + j] = hb[(size_t)i * mr + j];
        }
      }
      for (auto& pr : pairs) out_n[pr] = Cn[(size_t)pr.first * nr + pr.second];
    } else {
      // pair by pair, in groups whose distinct images fit the budget
      size_t k = 0;
      double* UV = nb.get(cap * M);
      while (k < pairs.size()) {
        std::map<int, int> su, sv;
        std::vector<int2> pl;
        size_t k1 = k;
        while (k1 < pairs.size()) {
          const int nu = (int)su.size() + (su.count(pairs[k1].first) ? 0 : 1);
          const int nv = (int)sv.size() + (sv.count(pairs[k1].second) ? 0 : 1);
          if (nu + nv > cap && k1 > k) break;
          if (!su.count(pairs[k1].first)) { const int id = (int)su.size(); su[pairs[k1].first] = id; }
          if (!sv.count(pairs[k1].second)) { const int id = (int)sv.size(); sv[pairs[k1].second] = id; }
          k1++;
        }
        const int nu = (int)su.size();
        GemmList gu;
        for (auto& x : su) make_u(gu, x.first, UV + (int64_t)x.second * M);
        for (auto& x : sv) make_v(gu, x.first, UV + (int64_t)(nu + x.second) * M);
        gu.run(nb, s);
        for (size_t q = k; q < k1; q++) pl.push_back(int2{su[pairs[q].first], nu + sv[pairs[q].second]});
        int2* dpl = upload_tmp(nb, pl);
        double* res = nb.get((int64_t)pl.size());
        HIPCHK(launch_pair_dots(UV, dpl, (int)pl.size(), M, res, s));
        std::vector<double> hr(pl.size());
        HIPCHK(hipMemcpyAsync(hr.data(), res, hr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t q = k; q < k1; q++) out_n[pairs[q]] = hr[q - k];
        k = k1;
      }
    }
  }
  for (size_t p = 0; p < prods.size(); p++) {
    const auto& w = where[p];
    out[p] = vals[w[0]].at({w[1], w[2]});
  }
}

}  // namespace rt

// ====================================================================== host helpers
namespace {

// Products of one-site operators whose sum is the dense operator H on the
// sorted sites S (first site most significant): nested operator-Schmidt
// decompositions, one site split off at a time (singular values above 1e-13
// of the largest kept).
struct HostProd {
  double coef;
  std::vector<std::pair<int, std::vector<double>>> f;
};

void decompose(const std::vector<int>& S, const std::vector<double>& H, int d, double coef, HostProd prefix,
               std::vector<HostProd>& out) {
  const int s = (int)S.size();
  if (s == 1) {
    prefix.coef *= coef;
    prefix.f.push_back({S[0], H});
    out.push_back(prefix);
    return;
  }
  int Dr = 1;
  for (int i = 1; i < s; i++) Dr *= d;
  const int D = d * Dr;
  // rows (o0, i0), columns (o_rest, i_rest)
  std::vector<double> A((size_t)d * d * Dr * Dr);
  for (int o = 0; o < D; o++)
    for (int i = 0; i < D; i++) {
      const int o0 = o / Dr, orr = o % Dr, i0 = i / Dr, ir = i % Dr;
      A[(size_t)(o0 * d + i0) * (Dr * Dr) + (size_t)orr * Dr + ir] = H[(size_t)o * D + i];
    }
  std::vector<double> U, sv, V;
  svd_jacobi(A, d * d, Dr * Dr, U, sv, V);
  const int k = (int)sv.size();
  const std::vector<int> rest(S.begin() + 1, S.end());
  for (int t = 0; t < k; t++) {
    if (!(sv[t] > 1e-13 * sv[0])) break;
    std::vector<double> X((size_t)d * d), Y((size_t)Dr * Dr);
    for (int e = 0; e < d * d; e++) X[e] = U[(size_t)e * k + t];
    for (int e = 0; e < Dr * Dr; e++) Y[e] = V[(size_t)e * k + t];
    HostProd p = prefix;
    p.f.push_back({S[0], X});
    decompose(rest, Y, d, coef * sv[t], p, out);
  }
}

// rotated dense operator of coef * prod ops on sites (Sec. 5.2): o' = U^T o U
void rotate_obs(attn_handle* h, const std::vector<int>& sites, const std::vector<const double*>& ops, double coef,
                std::vector<int>& S, std::vector<double>& H) {
  const ProblemCopy& P = h->prob;
  const int d = P.d;
  std::vector<int> de_of(P.n_sites, -1);
  for (size_t k = 0; k < P.de_sites.size() / 2; k++) de_of[P.de_sites[2 * k]] = de_of[P.de_sites[2 * k + 1]] = (int)k;
  std::vector<double> t(1, coef);
  int cur = 1;
  for (const double* o : ops) {
    std::vector<double> nt((size_t)cur * d * cur * d);
    for (int a = 0; a < cur; a++)
      for (int b = 0; b < cur; b++)
        for (int x = 0; x < d; x++)
          for (int y = 0; y < d; y++) nt[(size_t)(a * d + x) * (cur * d) + (b * d + y)] = t[(size_t)a * cur + b] * o[x * d + y];
    t.swap(nt);
    cur *= d;
  }
  std::string err;
  if (attn_status st = rotate_term_dense(sites, t, d, de_of, P.de_sites.data(), P.de_u.data(), S, H, err))
    throw StatusFail{st, err};
}

void to_engine(XEngine& E, const std::vector<HostProd>& hp, std::vector<XProd>& prods, std::vector<double>& coefs) {
  for (const HostProd& p : hp) {
    XProd x;
    for (auto& f : p.f) x.f.push_back({f.first, E.op_id(f.second.data())});
    prods.push_back(x);
    coefs.push_back(p.coef);
  }
}

attn_status need_root(attn_handle* h) {
  if (!h->state_ready) { h->err = "no state (attn_init_state not called)"; return ATTN_ERR_STATE; }
  const int root = h->M.tree.root;
  if (h->center != root) {
    attn_status st = attn_move_center(h, root, nullptr);
    if (st) return st;
  }
  return ATTN_OK;
}

}  // namespace

extern "C" {

attn_status attn_expect_products(attn_handle* h, int32_t n_prod, const int32_t* nsites, const int32_t* sites,
                                 const double* ops, double* out) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (n_prod < 0 || (n_prod > 0 && (!nsites || !sites || !ops || !out))) { h->err = "bad arguments"; return ATTN_ERR_ARG; }
    HIPCHK(hipSetDevice(h->device));
    if (attn_status e = need_root(h)) return e;
    const Tree& tr = h->M.tree;
    const int d = tr.d;
    XEngine E(h);
    std::vector<XProd> prods(n_prod);
    int64_t off = 0;
    for (int p = 0; p < n_prod; p++) {
      if (nsites[p] < 1 || nsites[p] > tr.N) { h->err = "product size out of range"; return ATTN_ERR_ARG; }
      for (int i = 0; i < nsites[p]; i++, off++) {
        const int s = sites[off];
        if (s < 0 || s >= tr.N) { h->err = "site out of range"; return ATTN_ERR_ARG; }
        prods[p].f.push_back({s, E.op_id(ops + off * d * d)});
      }
    }
    std::vector<double> v;
    E.run(prods, v, nullptr);
    for (int p = 0; p < n_prod; p++) out[p] = v[p];
    return ATTN_OK;
  });
}

attn_status attn_measure(attn_handle* h, int32_t n_obs, const int32_t* nsites, const int32_t* sites,
                         const double* ops, const double* coef, double* out) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (n_obs < 0 || (n_obs > 0 && (!nsites || !sites || !ops || !out))) { h->err = "bad arguments"; return ATTN_ERR_ARG; }
    HIPCHK(hipSetDevice(h->device));
    if (attn_status e = need_root(h)) return e;
    const Tree& tr = h->M.tree;
    const int d = tr.d;
    XEngine E(h);
    std::vector<XProd> prods;
    std::vector<double> coefs;
    std::vector<int> owner;
    int64_t off = 0;
    for (int o = 0; o < n_obs; o++) {
      if (nsites[o] < 1 || nsites[o] > 4) { h->err = "observables act on 1..4 sites"; return ATTN_ERR_ARG; }
      std::vector<int> st;
      std::vector<const double*> op;
      for (int i = 0; i < nsites[o]; i++, off++) {
        const int s = sites[off];
        if (s < 0 || s >= tr.N || std::find(st.begin(), st.end(), s) != st.end()) { h->err = "bad observable site"; return ATTN_ERR_ARG; }
        st.push_back(s);
        op.push_back(ops + off * d * d);
      }
      std::vector<int> S;
      std::vector<double> H;
      rotate_obs(h, st, op, coef ? coef[o] : 1.0, S, H);
      std::vector<HostProd> hp;
      decompose(S, H, d, 1.0, HostProd{1.0, {}}, hp);
      const size_t before = prods.size();
      to_engine(E, hp, prods, coefs);
      owner.resize(prods.size(), o);
      (void)before;
    }
    std::vector<double> v;
    E.run(prods, v, nullptr);
    for (int o = 0; o < n_obs; o++) out[o] = 0.0;
    for (size_t p = 0; p < prods.size(); p++) out[owner[p]] += coefs[p] * v[p];
    return ATTN_OK;
  });
}

attn_status attn_correlation(attn_handle* h, const double* oa, const double* ob, double* C) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (!oa || !ob || !C) { h->err = "NULL argument"; return ATTN_ERR_ARG; }
    HIPCHK(hipSetDevice(h->device));
    if (attn_status e = need_root(h)) return e;
    const Tree& tr = h->M.tree;
    const int N = tr.N, d = tr.d;
    const ProblemCopy& P = h->prob;
    std::vector<int> de_of(N, -1);
    for (size_t k = 0; k < P.de_sites.size() / 2; k++) de_of[P.de_sites[2 * k]] = de_of[P.de_sites[2 * k + 1]] = (int)k;
    std::vector<double> ab((size_t)d * d, 0.0);
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++)
        for (int k = 0; k < d; k++) ab[(size_t)i * d + j] += oa[i * d + k] * ob[k * d + j];
    // decompositions of the rotated one-site observables o' (shared by every pair)
    auto one = [&](int i, const double* o) {
      std::vector<int> S;
      std::vector<double> H;
      rotate_obs(h, {i}, {o}, 1.0, S, H);
      std::vector<HostProd> hp;
      decompose(S, H, d, 1.0, HostProd{1.0, {}}, hp);
      return hp;
    };
    std::vector<std::vector<HostProd>> da(N), db(N);
    for (int i = 0; i < N; i++) { da[i] = one(i, oa); db[i] = one(i, ob); }
    XEngine E(h);
    // operator ids of the shared factors
    auto ids = [&](const std::vector<HostProd>& hp) {
      std::vector<std::vector<std::pair<int, int>>> r;
      for (const HostProd& p : hp) {
        std::vector<std::pair<int, int>> f;
        for (auto& x : p.f) f.push_back({x.first, E.op_id(x.second.data())});
        r.push_back(f);
      }
      return r;
    };
    std::vector<std::vector<std::vector<std::pair<int, int>>>> ia(N), ib(N);
    for (int i = 0; i < N; i++) { ia[i] = ids(da[i]); ib[i] = ids(db[i]); }
    std::vector<XProd> prods;
    std::vector<double> coefs;
    std::vector<int64_t> owner;
    for (int i = 0; i < N; i++)
      for (int j = 0; j < N; j++) {
        const int64_t e = (int64_t)i * N + j;
        const bool same = i == j || (de_of[i] >= 0 && de_of[i] == de_of[j]);
        if (same) {
          // the pair acts on one gate's sites (or one site): rotate it as a whole
          std::vector<int> S;
          std::vector<double> H;
          if (i == j) rotate_obs(h, {i}, {ab.data()}, 1.0, S, H);
          else rotate_obs(h, {i, j}, {oa, ob}, 1.0, S, H);
          std::vector<HostProd> hp;
          decompose(S, H, d, 1.0, HostProd{1.0, {}}, hp);
          const size_t b0 = prods.size();
          to_engine(E, hp, prods, coefs);
          owner.resize(prods.size(), e);
          (void)b0;
          continue;
        }
        for (size_t k = 0; k < da[i].size(); k++)
          for (size_t l = 0; l < db[j].size(); l++) {
            XProd x;
            x.f = ia[i][k];
            x.f.insert(x.f.end(), ib[j][l].begin(), ib[j][l].end());
            prods.push_back(x);
            coefs.push_back(da[i][k].coef * db[j][l].coef);
            owner.push_back(e);
          }
      }
    std::vector<double> v;
    E.run(prods, v, nullptr);
    for (int64_t e = 0; e < (int64_t)N * N; e++) C[e] = 0.0;
    for (size_t p = 0; p < prods.size(); p++) C[owner[p]] += coefs[p] * v[p];
    return ATTN_OK;
  });
}

}  // extern "C"

// ====================================================================== disentangler optimisation
namespace {

struct DeTerm {
  double coef;
  std::vector<std::pair<int, std::vector<double>>> rest;   // the term's operators off the gate
  std::vector<double> Q;                                    // its operators on the gate's sites, (a b), a major
};

// Terms acting on the sites of every gate; ATTN_ERR_DE_RESTRICTION when a term
// acts on two gates (the optimisation of Sec. 4.1 needs that restriction).
attn_status gate_terms(const ProblemCopy& P, std::vector<std::vector<DeTerm>>& out, std::string& err) {
  const int d = P.d, dd = d * d;
  const int nde = (int)P.de_sites.size() / 2;
  std::vector<int> de_of(P.n_sites, -1);
  for (int k = 0; k < nde; k++) de_of[P.de_sites[2 * k]] = de_of[P.de_sites[2 * k + 1]] = k;
  out.assign(nde, {});
  int64_t off = 0;
  for (size_t t = 0; t < P.term_nsites.size(); t++) {
    const int ns = P.term_nsites[t];
    int k = -1;
    for (int i = 0; i < ns; i++) {
      const int g = de_of[P.term_sites[off + i]];
      if (g < 0) continue;
      if (k >= 0 && g != k) {
        err = "a term acts on two disentanglers (the optimisation needs ATTN_DE_STRICT placements)";
        return ATTN_ERR_DE_RESTRICTION;
      }
      k = g;
    }
    if (k >= 0) {
      const int a = P.de_sites[2 * k], b = P.de_sites[2 * k + 1];
      DeTerm dt;
      dt.coef = P.term_coef[t];
      std::vector<double> A(dd, 0.0), B(dd, 0.0);   // one-site factors on a and b (identity if absent)
      for (int x = 0; x < d; x++) A[x * d + x] = B[x * d + x] = 1.0;
      for (int i = 0; i < ns; i++) {
        const int s = P.term_sites[off + i];
        const double* o = P.term_ops.data() + (off + i) * dd;
        if (s == a) A.assign(o, o + dd);
        else if (s == b) B.assign(o, o + dd);
        else dt.rest.push_back({s, std::vector<double>(o, o + dd)});
      }
      dt.Q.assign((size_t)dd * dd, 0.0);
      for (int xa = 0; xa < d; xa++)
        for (int xb = 0; xb < d; xb++)
          for (int ya = 0; ya < d; ya++)
            for (int yb = 0; yb < d; yb++) dt.Q[(size_t)(xa * d + xb) * dd + ya * d + yb] = A[xa * d + ya] * B[xb * d + yb];
      out[k].push_back(std::move(dt));
    }
    off += ns;
  }
  return ATTN_OK;
}

void matmul(const double* A, const double* B, double* C, int n) {   // C = A B, n x n row-major
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      double acc = 0;
      for (int k = 0; k < n; k++) acc += A[i * n + k] * B[k * n + j];
      C[i * n + j] = acc;
    }
}

void transpose(const double* A, double* At, int n) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) At[j * n + i] = A[i * n + j];
}

}  // namespace

extern "C" {

attn_status attn_optimize_disentanglers(attn_handle* h, const attn_de_opts* opts, double* de_u_out, double* e_before,
                                        double* e_after, int32_t* iters) {
  return guard(h, [&]() -> attn_status {
    const ProblemCopy& P = h->prob;
    const int d = P.d, dd = d * d;
    const int nde = (int)P.de_sites.size() / 2;
    attn_de_opts o;
    if (opts) o = *opts;
    else { o.max_iter = 20; o.rel_tol = 1e-12; o.shift = 1; o.method = ATTN_DE_MERA; }
    if (o.max_iter < 0) { h->err = "max_iter < 0"; return ATTN_ERR_ARG; }
    if (o.method != ATTN_DE_MERA && o.method != ATTN_DE_RCG) { h->err = "unknown method"; return ATTN_ERR_ARG; }
    std::vector<std::vector<DeTerm>> gt;
    if (attn_status e = gate_terms(P, gt, h->err)) return e;
    if (attn_status e = need_device(h)) return e;
    HIPCHK(hipSetDevice(h->device));
    if (attn_status e = need_root(h)) return e;
    // products: for every gate, the d^2 x d^2 units |y><x| on (a, b) times each
    // term's operators off the gate, and alone (rho_ab)
    XEngine E(h);
    std::vector<int> unit_a(dd * dd), unit_b(dd * dd);
    std::vector<std::vector<double>> units(dd, std::vector<double>(dd, 0.0));
    for (int o2 = 0; o2 < d; o2++)
      for (int i2 = 0; i2 < d; i2++) units[o2 * d + i2][o2 * d + i2] = 1.0;
    std::vector<XProd> prods;
    for (int k = 0; k < nde; k++) {
      const int a = P.de_sites[2 * k], b = P.de_sites[2 * k + 1];
      for (int t = -1; t < (int)gt[k].size(); t++)
        for (int x = 0; x < dd; x++)
          for (int y = 0; y < dd; y++) {
            const int ya = y / d, yb = y % d, xa = x / d, xb = x % d;
            XProd pr;
            pr.f.push_back({a, E.op_id(units[ya * d + xa].data())});
            pr.f.push_back({b, E.op_id(units[yb * d + xb].data())});
            if (t >= 0)
              for (auto& r : gt[k][t].rest) pr.f.push_back({r.first, E.op_id(r.second.data())});
            prods.push_back(pr);
          }
    }
    std::vector<double> v;
    E.run(prods, v, nullptr);
    // the self-consistent iteration of every gate on the host (d^2 x d^2 algebra)
    size_t pi = 0;
    for (int k = 0; k < nde; k++) {
      std::vector<double> rho(v.begin() + pi, v.begin() + pi + dd * dd);
      pi += dd * dd;
      const int nt = (int)gt[k].size();
      std::vector<std::vector<double>> sig(nt);
      double c = 0.0;
      for (int t = 0; t < nt; t++) {
        sig[t].assign(v.begin() + pi, v.begin() + pi + dd * dd);
        for (double& z : sig[t]) z *= gt[k][t].coef;
        pi += dd * dd;
        if (o.shift) {
          // |coef| prod ||op||_2 over the term's operators (spectral norms by SVD)
          double nrm = std::fabs(gt[k][t].coef);
          std::vector<std::vector<double>> fs;
          for (auto& r : gt[k][t].rest) fs.push_back(r.second);
          std::vector<double> U, s, V;
          svd_jacobi(gt[k][t].Q, dd, dd, U, s, V);
          nrm *= s.empty() ? 0.0 : s[0];
          for (auto& f : fs) { svd_jacobi(f, d, d, U, s, V); nrm *= s.empty() ? 0.0 : s[0]; }
          c += nrm;
        }
      }
      std::vector<double> u(P.de_u.begin() + (size_t)k * dd * dd, P.de_u.begin() + (size_t)(k + 1) * dd * dd);
      // energy of the gate's terms: sum_t Tr(u sigma_t u^T Q_t)
      auto energy = [&](const std::vector<double>& uu) {
        std::vector<double> ut(dd * dd), t1(dd * dd), t2(dd * dd), t3(dd * dd);
        transpose(uu.data(), ut.data(), dd);
        double e = 0;
        for (int t = 0; t < nt; t++) {
          matmul(uu.data(), sig[t].data(), t1.data(), dd);
          matmul(t1.data(), ut.data(), t2.data(), dd);
          matmul(t2.data(), gt[k][t].Q.data(), t3.data(), dd);
          for (int i = 0; i < dd; i++) e += t3[i * dd + i];
        }
        return e;
      };
      double e0 = energy(u), e_prev = e0;
      int it = 0;
      if (o.method == ATTN_DE_RCG) {
        // Riemannian gradient in the frame of u: Omega = skew(u^T G), with the
        // gradient of E in both copies G = sum_t (Q_t^T u sigma_t^T + Q_t u sigma_t)
        auto rgrad = [&](const std::vector<double>& uu) {
          std::vector<double> G(dd * dd, 0.0), t1(dd * dd), t2(dd * dd), qt(dd * dd), st(dd * dd);
          for (int t = 0; t < nt; t++) {
            transpose(gt[k][t].Q.data(), qt.data(), dd);
            transpose(sig[t].data(), st.data(), dd);
            matmul(qt.data(), uu.data(), t1.data(), dd);
            matmul(t1.data(), st.data(), t2.data(), dd);
            for (int i = 0; i < dd * dd; i++) G[i] += t2[i];
            matmul(gt[k][t].Q.data(), uu.data(), t1.data(), dd);
            matmul(t1.data(), sig[t].data(), t2.data(), dd);
            for (int i = 0; i < dd * dd; i++) G[i] += t2[i];
          }
          std::vector<double> ut(dd * dd), A(dd * dd), W(dd * dd);
          transpose(uu.data(), ut.data(), dd);
          matmul(ut.data(), G.data(), A.data(), dd);
          for (int i = 0; i < dd; i++)
            for (int j = 0; j < dd; j++) W[i * dd + j] = 0.5 * (A[i * dd + j] - A[j * dd + i]);
          return W;
        };
        // u cay(X), cay(X) = (I - X/2)^-1 (I + X/2) by Gaussian elimination with partial pivoting
        auto retract = [&](const std::vector<double>& uu, const std::vector<double>& X) {
          std::vector<double> L(dd * dd), R(dd * dd);
          for (int i = 0; i < dd; i++)
            for (int j = 0; j < dd; j++) {
              L[i * dd + j] = (i == j ? 1.0 : 0.0) - 0.5 * X[i * dd + j];
              R[i * dd + j] = (i == j ? 1.0 : 0.0) + 0.5 * X[i * dd + j];
            }
          for (int c = 0; c < dd; c++) {
            int pv = c;
            for (int r = c + 1; r < dd; r++)
              if (std::fabs(L[r * dd + c]) > std::fabs(L[pv * dd + c])) pv = r;
            if (pv != c)
              for (int j = 0; j < dd; j++) { std::swap(L[c * dd + j], L[pv * dd + j]); std::swap(R[c * dd + j], R[pv * dd + j]); }
            for (int r = c + 1; r < dd; r++) {
              const double f = L[r * dd + c] / L[c * dd + c];
              for (int j = 0; j < dd; j++) { L[r * dd + j] -= f * L[c * dd + j]; R[r * dd + j] -= f * R[c * dd + j]; }
            }
          }
          std::vector<double> C(dd * dd);
          for (int j = 0; j < dd; j++)
            for (int r = dd - 1; r >= 0; r--) {
              double acc = R[r * dd + j];
              for (int q = r + 1; q < dd; q++) acc -= L[r * dd + q] * C[q * dd + j];
              C[r * dd + j] = acc / L[r * dd + r];
            }
          std::vector<double> out(dd * dd);
          matmul(uu.data(), C.data(), out.data(), dd);
          return out;
        };
        auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
          double acc = 0;
          for (int i = 0; i < dd * dd; i++) acc += a[i] * b[i];
          return acc;
        };
        std::vector<double> g = rgrad(u), D(dd * dd);
        for (int i = 0; i < dd * dd; i++) D[i] = -g[i];
        double E = e0;
        for (; it < o.max_iter; it++) {
          const double gg = dot(g, g);
          if (gg == 0.0) break;
          double slope = dot(g, D);
          if (slope >= 0.0) {
            for (int i = 0; i < dd * dd; i++) D[i] = -g[i];
            slope = -gg;
          }
          double t = 1.0, En;
          std::vector<double> un, X(dd * dd);
          while (true) {
            for (int i = 0; i < dd * dd; i++) X[i] = t * D[i];
            un = retract(u, X);
            En = energy(un);
            if (En <= E + 1e-4 * t * slope || t < 1e-12) break;
            t *= 0.5;
          }
          if (En > E) break;
          std::vector<double> gn = rgrad(un);
          double num = 0;
          for (int i = 0; i < dd * dd; i++) num += gn[i] * (gn[i] - g[i]);
          const double beta = std::max(0.0, num / gg);
          for (int i = 0; i < dd * dd; i++) D[i] = -gn[i] + beta * D[i];
          const bool done = std::fabs(En - E) <= o.rel_tol * std::max(1.0, std::fabs(En));
          u = un;
          E = En;
          g = gn;
          if (done) { it++; break; }
        }
        e_prev = E;
      }
      for (; o.method == ATTN_DE_MERA && it < o.max_iter; it++) {
        // Gamma = sum_t sigma_t u^T Q_t - c rho u^T  (eq. 4, bra copy fixed)
        std::vector<double> ut(dd * dd), G(dd * dd, 0.0), t1(dd * dd), t2(dd * dd);
        transpose(u.data(), ut.data(), dd);
        for (int t = 0; t < nt; t++) {
          matmul(sig[t].data(), ut.data(), t1.data(), dd);
          matmul(t1.data(), gt[k][t].Q.data(), t2.data(), dd);
          for (int i = 0; i < dd * dd; i++) G[i] += t2[i];
        }
        matmul(rho.data(), ut.data(), t1.data(), dd);
        for (int i = 0; i < dd * dd; i++) G[i] -= c * t1[i];
        // u = -V U^T for Gamma = U s V^T (eq. 5)
        std::vector<double> U, s, V;
        svd_jacobi(G, dd, dd, U, s, V);
        std::vector<double> nu(dd * dd, 0.0);
        for (int i = 0; i < dd; i++)
          for (int j = 0; j < dd; j++) {
            double acc = 0;
            for (int q = 0; q < dd; q++) acc += V[i * dd + q] * U[j * dd + q];
            nu[i * dd + j] = -acc;
          }
        u = nu;
        const double e1 = energy(u);
        const bool done = std::fabs(e1 - e_prev) <= o.rel_tol * std::max(1.0, std::fabs(e1));
        e_prev = e1;
        if (done) { it++; break; }
      }
      if (de_u_out) std::copy(u.begin(), u.end(), de_u_out + (size_t)k * dd * dd);
      if (e_before) e_before[k] = e0;
      if (e_after) e_after[k] = e_prev;
      if (iters) iters[k] = it;
    }
    return ATTN_OK;
  });
}

attn_status attn_set_disentanglers(attn_handle* h, const double* de_u) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (!de_u) { h->err = "de_u is NULL"; return ATTN_ERR_ARG; }
    ProblemCopy np = h->prob;
    np.de_u.assign(de_u, de_u + np.de_u.size());
    attn_problem pv = np.view();
    pv.flags &= ~(ATTN_HOST_ONLY | ATTN_DRYRUN);
    attn_handle* h2 = nullptr;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipDeviceSynchronize());
    const attn_status st = attn_build_tpo(&pv, &h2);
    if (st) { h->err = attn_last_error(nullptr); return st; }
    try {
      int64_t tot = 0;
      for (int64_t l : h->T_len) tot += l;
      HIPCHK(hipMemcpy(h2->d_T, h->d_T, tot * sizeof(double), hipMemcpyDeviceToDevice));
      h2->iso = h->iso;
      h2->center = h->center;
      h2->state_ready = h->state_ready;
      h2->sweep_energies = h->sweep_energies;
      h2->n_matvec = h->n_matvec; h2->n_env = h->n_env; h2->n_qr = h->n_qr; h2->mv_flops = h->mv_flops;
      h2->jacobi_rate = h->jacobi_rate; h2->n_dav_iter = h->n_dav_iter; h2->n_fallback = h->n_fallback;
      if (h->mlp_ready) {
        h2->d_mlp = dev_alloc(h2, kMlpParams * 2);
        HIPCHK(hipMemcpy(h2->d_mlp, h->d_mlp, kMlpParams * 2, hipMemcpyDeviceToDevice));
        h2->mlp_ready = true;
      }
      if (h2->state_ready) {
        reset_state(h2, 0, nullptr);
        rebuild_envs(h2, nullptr);
        check_state(h2, nullptr, "attn_set_disentanglers");
      }
    } catch (...) {
      attn_destroy(h2);
      throw;
    }
    std::swap(*h, *h2);
    std::swap(h->err, h2->err);
    attn_destroy(h2);
    return ATTN_OK;
  });
}

attn_status attn_sweep_attn(attn_handle* h, int32_t n_sweeps, int32_t s_ttn, const attn_sweep_opts* sopts,
                            const attn_de_opts* dopts, double* energies, double* seconds) {
  if (!h) return ATTN_ERR_ARG;
  if (n_sweeps < 0 || s_ttn < 0) { h->err = "n_sweeps and s_ttn must be >= 0"; return ATTN_ERR_ARG; }
  const int dd = h->prob.d * h->prob.d;
  std::vector<double> u(h->prob.de_u.size());
  for (int s = 0; s < n_sweeps; s++) {
    auto t0 = std::chrono::steady_clock::now();
    if (s >= s_ttn && !u.empty()) {
      attn_status st = attn_optimize_disentanglers(h, dopts, u.data(), nullptr, nullptr, nullptr);
      if (st) return st;
      st = attn_set_disentanglers(h, u.data());
      if (st) return st;
    }
    double e = 0;
    attn_status st = attn_sweep(h, 1, sopts, &e, nullptr);
    if (st) return st;
    auto t1 = std::chrono::steady_clock::now();
    if (energies) energies[s] = e;
    if (seconds) seconds[s] = std::chrono::duration<double>(t1 - t0).count();
    (void)dd;
  }
  return ATTN_OK;
}

attn_status attn_get_disentanglers(const attn_handle* h, double* de_u, int64_t len) {
  if (!h || !de_u) return ATTN_ERR_ARG;
  if (len != (int64_t)h->prob.de_u.size()) return ATTN_ERR_SHAPE;
  std::copy(h->prob.de_u.begin(), h->prob.de_u.end(), de_u);
  return ATTN_OK;
}

}  // extern "C"
