// Runtime of the aTTN hot path: device memory, per-node device plans and the
// C interface declared in attn.h.  All arithmetic of the path runs in the
// kernels of kernels.hip; this file only allocates, uploads work lists and
// enqueues launches.
#include "runtime.hpp"

using namespace attn;
using namespace rt;

namespace {
thread_local std::string g_build_error;
}  // namespace

namespace rt {

// ------------------------------------------------------------------ device memory
// Every device buffer goes through dev_alloc so that a dry-run build can lay
// out all work lists in a fake address space and check them on the host.
void* dev_alloc(attn_handle* h, size_t bytes) {
  bytes = std::max<size_t>(bytes, 8);
  void* p = nullptr;
  if (h->dryrun) {
    p = (void*)h->fake_next;
    h->fake_next += (bytes + (1u << 20) - 1) / (1u << 20) * (1u << 20) + (1u << 20);
  } else {
    HIPCHK(hipMalloc(&p, bytes));
    h->owned.push_back(p);
  }
  h->allocs.push_back({(uintptr_t)p, bytes});
  return p;
}

// ------------------------------------------------------------------ pointers
double* block_ptr(attn_handle* h, const BRef& b, double* comb_base, const std::vector<int64_t>& comb_off) {
  if (b.kind == 0) {
    int dim = h->M.tree.edge_dim(b.edge);
    return h->store[b.dir][b.edge] + (int64_t)(b.slot + 1) * dim * dim;
  }
  if (b.kind == 1) return comb_base + comb_off[b.slot];
  return nullptr;
}

void build_comb(attn_handle* h, const std::vector<Combine>& cs, double* base, CBPlan& P,
                std::vector<int64_t>& off, int64_t& total) {
  off.clear();
  total = 0;
  for (const Combine& c : cs) {
    off.push_back(total);
    total += (int64_t)c.dim * c.dim;
  }
  for (size_t i = 0; i < cs.size(); i++) {
    CBTask t;
    t.out = base ? base + off[i] : nullptr;
    t.n = cs[i].dim * cs[i].dim;
    t.term0 = (int)P.terms.size();
    t.nterm = (int)cs[i].in.size();
    t.pad = 0;
    for (auto& pr : cs[i].in) {
      CBTerm ct;
      ct.in = block_ptr(h, pr.first, nullptr, off);
      ct.coef = pr.second;
      P.terms.push_back(ct);
    }
    P.maxn = std::max(P.maxn, t.n);
    P.tasks.push_back(t);
  }
}

void upload_comb(attn_handle* h, CBPlan& P) {
  P.d_tasks = upload(h, P.tasks);
  P.d_terms = upload(h, P.terms);
}

// slice geometry of a spectator leg for a (d0, d1, d2) tensor in layout [l][r][p]
// (or [p][l][r] for spectator p when transposed)
void slice_geom(int spect, const int* dm, int& ma, int& mb, int& ns, int64_t& sl, int64_t& row) {
  if (spect == 0) { ma = dm[1]; mb = dm[2]; ns = dm[0]; sl = (int64_t)dm[1] * dm[2]; row = dm[2]; }
  else if (spect == 1) { ma = dm[0]; mb = dm[2]; ns = dm[1]; sl = dm[2]; row = (int64_t)dm[1] * dm[2]; }
  else { ma = dm[0]; mb = dm[1]; ns = dm[2]; sl = (int64_t)dm[0] * dm[1]; row = dm[1]; }
}

bool sw_mfma(int ma, int mb) { return ma % 16 == 0 && mb % 16 == 0 && ma <= 128 && mb <= 128; }

void add_sw_task(SWGroup& g, SWTask t, int ns) {
  g.ma = t.ma;
  g.mb = t.mb;
  const int ti = (int)g.tasks.size();
  g.tasks.push_back(t);
  const double M = (double)ns * t.ma * t.mb;
  int i0 = t.item0, i1 = t.item0 + t.nitem;
  if (t.pad) {   // several outputs: their items are consecutive
    i0 = g.outs[t.item0].item0;
    i1 = g.outs[t.item0 + t.nitem - 1].item0 + g.outs[t.item0 + t.nitem - 1].nitem;
  }
  for (int i = i0; i < i1; i++)
    g.flops += 2.0 * M * ((g.items[i].A ? t.ma : 0) + (g.items[i].B ? t.mb : 0));
  if (sw_mfma(t.ma, t.mb)) {
    for (int s = 0; s < ns; s++)
      for (int st = 0; st < t.ma / 16; st += 4) g.wus.push_back(make_int4(ti, s, st, 0));
  } else {
    for (int s = 0; s < ns; s++)
      for (int e = 0; e < t.ma * t.mb; e += 256) g.wus.push_back(make_int4(ti, s, e, 0));
  }
}

SWGroup& group_for(std::vector<SWGroup>& gs, int ma, int mb) {
  for (auto& g : gs)
    if (g.ma == ma && g.mb == mb) return g;
  gs.emplace_back();
  gs.back().ma = ma;
  gs.back().mb = mb;
  return gs.back();
}

MPGroup& mgroup_for(std::vector<MPGroup>& gs, int mj, bool mf) {
  for (auto& g : gs)
    if (g.mj == mj && g.mfma == mf) return g;
  gs.emplace_back();
  gs.back().mj = mj;
  gs.back().mfma = mf;
  return gs.back();
}

void add_mp_task(MPGroup& g, MPTask t) {
  const int ti = (int)g.tasks.size();
  g.tasks.push_back(t);
  const int mj = t.j == 0 ? t.d0 : (t.j == 1 ? t.d1 : t.d2);
  const int64_t M = (int64_t)t.d0 * t.d1 * t.d2;
  if (g.mfma) {
    for (int64_t f = 0; f < M / mj / 64; f++) g.wus.push_back(make_int2(ti, (int)f));
  } else {
    for (int64_t e = 0; e < M; e += 256) g.wus.push_back(make_int2(ti, (int)e));
  }
}

// Workgroups are handed to the eight XCDs (each with its own L2) round robin by
// workgroup index.  Order the work units so that all units of one task (one
// group of operator blocks) land on the same XCD: tasks are assigned to XCDs
// greedily by unit count, and position i of the launch takes the next unit of
// XCD i mod 8 (or of any XCD with units left once that one is drained).
template <typename U>
void xcd_order(std::vector<U>& wus) {
  constexpr int kXcd = 8;
  if (wus.size() < 2 * kXcd) return;
  int ntask = 0;
  for (const U& u : wus) ntask = std::max(ntask, u.x + 1);
  std::vector<int64_t> cnt(ntask, 0);
  for (const U& u : wus) cnt[u.x]++;
  std::vector<int> order(ntask);
  for (int t = 0; t < ntask; t++) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
  std::vector<int> xcd_of(ntask, 0);
  int64_t load[kXcd] = {0};
  for (int t : order) {
    int best = 0;
    for (int x = 1; x < kXcd; x++)
      if (load[x] < load[best]) best = x;
    xcd_of[t] = best;
    load[best] += cnt[t];
  }
  std::vector<std::vector<U>> q(kXcd);
  for (const U& u : wus) q[xcd_of[u.x]].push_back(u);
  size_t pos[kXcd] = {0};
  std::vector<U> out;
  out.reserve(wus.size());
  for (size_t i = 0; i < wus.size(); i++) {
    int x = (int)(i % kXcd);
    if (pos[x] == q[x].size())
      for (int y = 0; y < kXcd; y++)
        if (pos[y] < q[y].size()) { x = y; break; }
    out.push_back(q[x][pos[x]++]);
  }
  wus.swap(out);
}

void upload_sw(attn_handle* h, std::vector<SWGroup>& gs, bool by_xcd = false) {
  for (auto& g : gs) {
    if (by_xcd) xcd_order(g.wus);
    g.d_tasks = upload(h, g.tasks);
    g.d_outs = upload(h, g.outs);
    g.d_items = upload(h, g.items);
    g.d_wus = upload(h, g.wus);
  }
}

// the register-direct mode kernel applies when every task contracts leg 0 or 1
// of a tensor whose last leg is a multiple of 16 (m_j <= 64)
bool mode_nt_ok(const std::vector<MPTask>& ts, bool mfma) {
  if (!mfma || ts.empty()) return false;
  for (const MPTask& t : ts) {
    const int mj = t.j == 0 ? t.d0 : (t.j == 1 ? t.d1 : t.d2);
    if (t.j > 1 || mj > 64 || t.d2 % 16) return false;
  }
  return true;
}

void upload_mp(attn_handle* h, std::vector<MPGroup>& gs) {
  for (auto& g : gs) {
    g.nt = mode_nt_ok(g.tasks, g.mfma);
    g.d_tasks = upload(h, g.tasks);
    g.d_jobs = upload(h, g.jobs);
    g.d_wus = upload(h, g.wus);
  }
}


void mv_chunks(const MatvecPlan& P, const int* dm, const int64_t target[3], int out[3]) {
  int64_t nit[3] = {0, 0, 0}, units[3] = {1, 1, 1};
  int ma[3], mb[3];
  for (const Item2& it : P.items) nit[it.spect]++;
  for (int sp = 0; sp < 3; sp++) {
    int ns;
    int64_t sl, row;
    slice_geom(sp, dm, ma[sp], mb[sp], ns, sl, row);
    units[sp] = sw_mfma(ma[sp], mb[sp]) ? (int64_t)ns * ((ma[sp] / 16 + 3) / 4)
                                        : (int64_t)ns * ((ma[sp] * mb[sp] + 255) / 256);
  }
  mv_chunk_counts(nit, ma, mb, units, (int64_t)dm[0] * dm[1] * dm[2], target, out);
}

// ------------------------------------------------------------------ plan construction
void build_mv_dev(attn_handle* h, int n, std::vector<int64_t>& comb_off_out) {
  const Model& M = h->M;
  const MatvecPlan& P = M.mv[n];
  MVDev& D = h->mv[n];
  const Node& nd = M.tree.nodes[n];
  const int dm[3] = {nd.dims[0], nd.dims[1], nd.dims[2]};
  std::copy(dm, dm + 3, D.dims);
  const int64_t Msz = (int64_t)dm[0] * dm[1] * dm[2];
  std::vector<int64_t> off;
  int64_t total = 0;
  build_comb(h, P.combines, h->d_mvcomb, D.comb, off, total);
  comb_off_out = off;
  h->comb_blocks[n].clear();
  for (size_t i = 0; i < P.combines.size(); i++) h->comb_blocks[n].push_back({off[i], P.combines[i].dim});
  int64_t part_used = 0;
  int nchs[3];
  const int64_t target[3] = {kMvTarget, kMvTarget, kMvTarget};
  mv_chunks(P, dm, target, nchs);
  // two-leg items and local operators, grouped by spectator
  for (int sp = 0; sp < 3; sp++) {
    std::vector<const Item2*> its;
    for (const Item2& it : P.items)
      if (it.spect == sp) its.push_back(&it);
    if (its.empty()) continue;
    int ma, mb, ns;
    int64_t sl, row;
    slice_geom(sp, dm, ma, mb, ns, sl, row);
    const int nch = nchs[sp];
    SWGroup& g = group_for(D.sw, ma, mb);
    for (int c = 0; c < nch; c++) {
      const size_t i0 = its.size() * c / nch, i1 = its.size() * (c + 1) / nch;
      if (i1 == i0) continue;
      SWTask t;
      std::memset(&t, 0, sizeof(t));
      const bool trans = sp == 2 && dm[2] > 1;   // [p][l][r] == [l][r][p] when m_p = 1
      t.x = trans ? (const void*)h->d_xt : nullptr;
      t.y = h->d_part + part_used;
      t.xs_slice = sl; t.xs_row = row; t.ys_slice = sl; t.ys_row = row;
      t.ma = ma; t.mb = mb;
      t.item0 = (int)g.items.size();
      for (size_t i = i0; i < i1; i++) {
        SWItem si;
        si.A = block_ptr(h, its[i]->A, h->d_mvcomb, off);
        si.B = block_ptr(h, its[i]->B, h->d_mvcomb, off);
        si.coef = its[i]->coef;
        g.items.push_back(si);
      }
      t.nitem = (int)(i1 - i0);
      t.accumulate = 0;
      add_sw_task(g, t, ns);
      D.srcs.push_back({h->d_part + part_used, trans ? 1 : 0, 0});
      part_used += Msz;
      if (trans) D.need_xt = true;
    }
  }
  // three-leg chains
  int64_t chain_used = 0;
  std::vector<std::vector<std::pair<const double*, const double*>>> stageC(3);   // per o1 leg: (op, V)
  for (const Chain& ch : P.chains) {
    const int t2 = (int)ch.O2.size(), t1 = (int)ch.O1.size();
    std::vector<double*> W(t2), Vv(t1);
    for (int c = 0; c < t2; c++) {
      W[c] = h->d_chain + chain_used;
      chain_used += Msz;
      MPGroup& g = mgroup_for(D.chainA, dm[ch.o2], mode_mfma_ok(dm[ch.o2], Msz));
      MPTask t{W[c], dm[0], dm[1], dm[2], ch.o2, (int)g.jobs.size(), 1, 0, 0};
      g.jobs.push_back({block_ptr(h, ch.O2[c], h->d_mvcomb, off), nullptr, 1.0});
      add_mp_task(g, t);
    }
    for (int a = 0; a < t1; a++) {
      MPGroup& g = mgroup_for(D.chainB, dm[ch.mid], mode_mfma_ok(dm[ch.mid], Msz));
      int j0 = (int)g.jobs.size();
      for (int c = 0; c < t2; c++) {
        const BRef& b = ch.Mid[(size_t)a * t2 + c];
        if (b.is_zero()) continue;
        g.jobs.push_back({block_ptr(h, b, h->d_mvcomb, off), W[c], 1.0});
      }
      if ((int)g.jobs.size() == j0) { Vv[a] = nullptr; continue; }
      Vv[a] = h->d_chain + chain_used;
      chain_used += Msz;
      MPTask t{Vv[a], dm[0], dm[1], dm[2], ch.mid, j0, (int)g.jobs.size() - j0, 0, 0};
      add_mp_task(g, t);
    }
    for (int a = 0; a < t1; a++)
      if (Vv[a]) stageC[ch.o1].push_back({block_ptr(h, ch.O1[a], h->d_mvcomb, off), Vv[a]});
  }
  for (int leg = 0; leg < 3; leg++) {
    if (stageC[leg].empty()) continue;
    double* out = h->d_chain + chain_used;
    chain_used += Msz;
    MPGroup& g = mgroup_for(D.chainC, dm[leg], mode_mfma_ok(dm[leg], Msz));
    MPTask t{out, dm[0], dm[1], dm[2], leg, (int)g.jobs.size(), (int)stageC[leg].size(), 0, 0};
    for (auto& pr : stageC[leg]) g.jobs.push_back({pr.first, pr.second, 1.0});
    add_mp_task(g, t);
    D.srcs.push_back({out, 0, 0});
  }
  if (part_used > h->part_cap || chain_used > h->chain_cap)
    throw StatusFail{ATTN_ERR_STATE, "internal: scratch sizing"};
  upload_comb(h, D.comb);
  upload_sw(h, D.sw, true);
  upload_mp(h, D.chainA);
  upload_mp(h, D.chainB);
  upload_mp(h, D.chainC);
  D.d_srcs = upload(h, D.srcs);
  // explicit item lists: the dense H_eff of tiny nodes (M <= 1024) and the
  // H_eff diagonal of every node
  {
    TinyPlan tp;
    std::memset(&tp, 0, sizeof(tp));
    std::vector<SWItem> titems;
    for (int sp = 0; sp < 3; sp++) {
      tp.item0[sp] = (int)titems.size();
      for (const Item2& it : P.items)
        if (it.spect == sp)
          titems.push_back({block_ptr(h, it.A, h->d_mvcomb, off), block_ptr(h, it.B, h->d_mvcomb, off), it.coef});
      tp.nitem[sp] = (int)titems.size() - tp.item0[sp];
    }
    tp.items = upload(h, titems);
    D.tiny_items = titems;
    for (int sp = 0; sp < 3; sp++) { D.tiny_item0[sp] = tp.item0[sp]; D.tiny_nitem[sp] = tp.nitem[sp]; }
    std::vector<Item3> it3;
    for (const Chain& ch : P.chains) {
      const int t2 = (int)ch.O2.size();
      for (size_t a = 0; a < ch.O1.size(); a++)
        for (int c = 0; c < t2; c++) {
          const BRef& mid = ch.Mid[a * t2 + c];
          if (mid.is_zero()) continue;
          Item3 q;
          q.op[ch.o1] = block_ptr(h, ch.O1[a], h->d_mvcomb, off);
          q.op[ch.mid] = block_ptr(h, mid, h->d_mvcomb, off);
          q.op[ch.o2] = block_ptr(h, ch.O2[c], h->d_mvcomb, off);
          q.coef = 1.0;
          it3.push_back(q);
        }
    }
    tp.items3 = upload(h, it3);
    D.tiny_items3 = it3;
    tp.n3 = (int)it3.size();
    tp.d0 = dm[0]; tp.d1 = dm[1]; tp.d2 = dm[2];
    D.d_plan = upload(h, std::vector<TinyPlan>{tp});
    if (Msz <= 1024) D.d_tiny = D.d_plan;
  }
}

// The register-direct gram kernel applies when every task contracts leg 0 or 1
// of a tensor whose last leg is a multiple of 16, over 16-aligned free ranges,
// with 32-byte aligned operands and m_j <= 64.
bool gram_nt_ok(const std::vector<GRTask>& ts, bool mfma) {
  if (!mfma || ts.empty()) return false;
  for (const GRTask& t : ts) {
    const int mj = t.j == 0 ? t.d0 : (t.j == 1 ? t.d1 : t.d2);
    if (t.j > 1 || mj > 64 || t.d2 % 16 || t.f0 % 16 || t.f1 % 16) return false;
    if ((uintptr_t)t.X % 32 || (uintptr_t)t.Z % 32) return false;
  }
  return true;
}

int64_t env_chunk_outputs(attn_handle* h, int64_t Msz) {
  const int64_t budget = (int64_t)2 << 30;   // bytes of Z scratch
  return std::max<int64_t>(1, std::min<int64_t>(4096, budget / (Msz * 8)));
}

// Geometry of an effective-operator update: tensor dims as contracted (leg 2
// is transposed to the front), contracted leg j, sandwich shape and slices.
struct EnvGeom {
  bool tr_in;
  int dm[3], j, mj, ma, mb, ns;
  int64_t Msz, sl, row;
};

EnvGeom env_geom(const Model& M, const EnvPlan& P) {
  const Node& nd = M.tree.nodes[P.node];
  int spect = P.leg;
  for (const EnvOut& o : P.outs)
    if (!o.items.empty()) { spect = o.items[0].spect; break; }
  EnvGeom g;
  g.tr_in = P.leg == 2;
  g.dm[0] = g.tr_in ? nd.dims[2] : nd.dims[0];
  g.dm[1] = g.tr_in ? nd.dims[0] : nd.dims[1];
  g.dm[2] = g.tr_in ? nd.dims[1] : nd.dims[2];
  g.Msz = (int64_t)g.dm[0] * g.dm[1] * g.dm[2];
  g.j = g.tr_in ? 0 : P.leg;
  g.mj = g.dm[g.j];
  slice_geom(g.tr_in ? 0 : spect, g.dm, g.ma, g.mb, g.ns, g.sl, g.row);
  return g;
}

// Workgroups an effective-operator update's sandwich launch aims at.
constexpr int64_t kEnvWorkgroups = 2048;

// Pieces per output: on the matrix cores an output whose item count exceeds
// the balanced share of one task is split into pieces (separate partial Z
// tensors, summed by the gram reduction) so that no task dominates the launch.
std::vector<int> env_pieces(const Model& M, const EnvPlan& P, int& cap_out) {
  const EnvGeom g = env_geom(M, P);
  std::vector<int> pc(P.outs.size(), 0);
  int64_t W = 0;
  for (size_t o = 0; o < P.outs.size(); o++) W += (int64_t)P.outs[o].items.size();
  const int64_t strips = std::max(1, (g.ma / 16 + 3) / 4);
  const int64_t ntask = std::max<int64_t>(1, (kEnvWorkgroups + g.ns * strips - 1) / (g.ns * strips));
  const int cap = sw_mfma(g.ma, g.mb) ? (int)std::max<int64_t>(4, (W + ntask - 1) / ntask) : 1 << 30;
  for (size_t o = 0; o < P.outs.size(); o++) {
    const int w = (int)P.outs[o].items.size();
    pc[o] = w == 0 ? 0 : (w + cap - 1) / cap;
  }
  cap_out = cap;
  return pc;
}

void build_env_dev(attn_handle* h, const EnvPlan& P, EnvDev& D) {
  if (P.node < 0) return;
  const Model& M = h->M;
  const Node& nd = M.tree.nodes[P.node];
  // toward the parent the tensor is first transposed to [p][l][r] so that the
  // (l, r) slices are contiguous; the contracted leg is then the first one.
  // At the root (m_p = 1) the items may use p as spectator: no transpose needed.
  const EnvGeom geo = env_geom(M, P);
  const bool tr_in = geo.tr_in;
  const int* dm = geo.dm;
  const int64_t Msz = geo.Msz;
  const int j = geo.j, mj = geo.mj, ma = geo.ma, mb = geo.mb, ns = geo.ns;
  const int64_t sl = geo.sl, row = geo.row;
  D.transpose = tr_in;
  std::copy(nd.dims, nd.dims + 3, D.dims);
  D.present = true;
  D.node = P.node; D.leg = P.leg; D.out_edge = P.out_edge; D.out_dir = P.out_dir;
  std::vector<int64_t> off;
  int64_t total = 0;
  build_comb(h, P.combines, h->d_envcomb, D.comb, off, total);
  upload_comb(h, D.comb);
  double* T = tr_in ? h->d_xt : h->d_T + h->T_off[P.node];
  double* base = h->store[P.out_dir][P.out_edge];
  const int64_t per = env_chunk_outputs(h, Msz);   // Z tensors per chunk
  const int64_t F = Msz / mj;
  const bool gmf = gram_mfma_ok(mj, Msz);
  int64_t fchunk = F;
  if (gmf) {
    // enough gram workgroups: ~8 chunks of the free index per output at most
    fchunk = std::max<int64_t>(64, ((F / 8) + 63) / 64 * 64);
    while (F % fchunk) fchunk += 64;
  }
  const int nfc = (int)(F / fchunk);
  int cap = 0;
  const std::vector<int> pieces = env_pieces(M, P, cap);
  const bool multi = sw_mfma(ma, mb);
  const int64_t strips = std::max(1, (ma / 16 + 3) / 4);
  size_t o0 = 0;
  while (o0 < P.outs.size()) {
    // chunk: consecutive outputs whose pieces fit the Z budget
    size_t o1 = o0;
    int64_t nz = 0;
    while (o1 < P.outs.size() && (nz + pieces[o1] <= per || o1 == o0)) { nz += pieces[o1]; o1++; }
    EnvChunk ch;
    ch.gr.mj = mj;
    ch.gr.mfma = gmf;
    // virtual outputs: (output, first item, item count, Z slot); partial grams
    // of all pieces of an output are consecutive and reduced together
    struct VOut { size_t o; int i0, ni; int64_t z; };
    std::vector<VOut> vouts;
    int64_t zslot = 0, pslot = 0;
    for (size_t o = o0; o < o1; o++) {
      const EnvOut& out = P.outs[o];
      double* blk = base + (int64_t)(out.slot + 1) * mj * mj;
      if (out.items.empty()) {
        ch.zero_blocks.push_back({blk, (int64_t)mj * mj});
        continue;
      }
      const int w = (int)out.items.size(), np = pieces[o];
      double* part = h->d_grpart + pslot * mj * mj;
      for (int k = 0; k < np; k++) {
        const int i0 = (int)((int64_t)w * k / np), i1 = (int)((int64_t)w * (k + 1) / np);
        vouts.push_back({o, i0, i1 - i0, zslot});
        double* Z = h->d_Z + zslot * Msz;
        for (int c = 0; c < nfc; c++) {
          GRTask gt;
          gt.X = T; gt.Z = Z; gt.partial = h->d_grpart + (pslot + (int64_t)k * nfc + c) * mj * mj;
          gt.d0 = dm[0]; gt.d1 = dm[1]; gt.d2 = dm[2]; gt.j = j;
          gt.f0 = (int)(c * fchunk); gt.f1 = (int)((c + 1) * fchunk);
          ch.gr.tasks.push_back(gt);
        }
        zslot++;
      }
      GRReduce rd;
      rd.partial = part; rd.out = blk; rd.m = mj; rd.npart = np * nfc;
      rd.coef = 1.0; rd.accumulate = 0; rd.pad = 0;
      ch.gr.reds.push_back(rd);
      pslot += (int64_t)np * nfc;
    }
    // tasks: on the matrix cores several virtual outputs share a task (one
    // staging of each slice of T serves all of them), packed longest first into
    // the least loaded task and issued heaviest first; otherwise one per task
    std::vector<std::vector<size_t>> packs;
    if (multi && !vouts.empty()) {
      const int64_t ntask = std::max<int64_t>(1, std::min<int64_t>((int64_t)vouts.size(),
                                                                   (kEnvWorkgroups + ns * strips - 1) / (ns * strips)));
      std::vector<size_t> byw(vouts.size());
      for (size_t v = 0; v < vouts.size(); v++) byw[v] = v;
      std::stable_sort(byw.begin(), byw.end(), [&](size_t a, size_t b) { return vouts[a].ni > vouts[b].ni; });
      std::vector<std::vector<size_t>> pk(ntask);
      std::vector<int64_t> load(ntask, 0);
      for (size_t v : byw) {
        int64_t best = 0;
        for (int64_t q = 1; q < ntask; q++)
          if (load[q] < load[best]) best = q;
        pk[best].push_back(v);
        load[best] += vouts[v].ni;
      }
      std::vector<int64_t> idx(ntask);
      for (int64_t q = 0; q < ntask; q++) idx[q] = q;
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return load[a] > load[b]; });
      for (int64_t q : idx)
        if (!pk[q].empty()) packs.push_back(pk[q]);
    } else {
      for (size_t v = 0; v < vouts.size(); v++) packs.push_back({v});
    }
    for (const std::vector<size_t>& pk : packs) {
      SWGroup& g = group_for(ch.sw, ma, mb);
      SWTask t;
      std::memset(&t, 0, sizeof(t));
      t.x = T; t.y = h->d_Z + vouts[pk[0]].z * Msz;
      t.xs_slice = sl; t.xs_row = row; t.ys_slice = sl; t.ys_row = row;
      t.ma = ma; t.mb = mb;
      if (multi) {
        t.pad = 1;
        t.item0 = (int)g.outs.size();
        t.nitem = (int)pk.size();
      } else {
        t.item0 = (int)g.items.size();
      }
      int nit = 0;
      for (size_t v : pk) {
        const VOut& vo = vouts[v];
        const EnvOut& out = P.outs[vo.o];
        if (multi) g.outs.push_back({h->d_Z + vo.z * Msz, (int)g.items.size(), vo.ni});
        for (int i = vo.i0; i < vo.i0 + vo.ni; i++) {
          const Item2& it = out.items[i];
          SWItem si;
          si.A = block_ptr(h, it.A, h->d_envcomb, off);
          si.B = block_ptr(h, it.B, h->d_envcomb, off);
          si.coef = it.coef;
          g.items.push_back(si);
          nit++;
        }
      }
      if (!multi) t.nitem = nit;
      add_sw_task(g, t, ns);
    }
    ch.gr.nt = gram_nt_ok(ch.gr.tasks, gmf);
    upload_sw(h, ch.sw);
    ch.gr.d_tasks = upload(h, ch.gr.tasks);
    ch.gr.d_reds = upload(h, ch.gr.reds);
    D.chunks.push_back(std::move(ch));
    o0 = o1;
  }
}

// ------------------------------------------------------------------ execution helpers
void run_comb(CBPlan& P, hipStream_t s) {
  if (!P.tasks.empty()) HIPCHK(launch_combine(P.d_tasks, P.d_terms, (int)P.tasks.size(), P.maxn, s));
}

void run_sw(std::vector<SWGroup>& gs, int dtype, const void* xbase, hipStream_t s) {
  for (auto& g : gs)
    HIPCHK(launch_sandwich(dtype, g.ma, g.mb, g.d_tasks, g.d_items, g.d_wus, (int)g.wus.size(), xbase, s,
                           g.d_outs));
}

hipEvent_t next_event(attn_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// matvec sandwich launches, bracketed by events when profiling
void run_sw_mv(attn_handle* h, std::vector<SWGroup>& gs, int dtype, const void* xbase, hipStream_t s) {
  for (auto& g : gs) {
    int a = -1, b = -1;
    if (h->prof && h->ev_used + 2 <= (size_t)1 << 20) {
      a = (int)h->ev_used;
      HIPCHK(hipEventRecord(next_event(h), s));
    }
    HIPCHK(launch_sandwich(g.fmt >= 2 ? g.fmt : dtype, g.ma, g.mb, g.d_tasks, g.d_items, g.d_wus, (int)g.wus.size(), xbase, s));
    if (a >= 0) {
      b = (int)h->ev_used;
      HIPCHK(hipEventRecord(next_event(h), s));
      h->prof_recs.push_back({a, b, g.flops, g.ma, g.mb, g.fmt >= 2 ? g.fmt : dtype});
    }
  }
}

void run_mp(std::vector<MPGroup>& gs, int dtype, const void* xbase, hipStream_t s) {
  for (auto& g : gs)
    HIPCHK(launch_mode(dtype, g.mj, g.mfma, g.d_tasks, g.d_jobs, g.d_wus, (int)g.wus.size(), xbase, s, g.nt));
}

// y <- H_eff(n) x (FP64), combines must be current.  With a Krylov job J
// (y = J's w), the partial dots of basis vectors [i0, i0 + nv) with y go to
// area pin in the same launch as the sum of the partial outputs.
void matvec_f64(attn_handle* h, int n, const double* x, double* y, hipStream_t s, const KJob* J = nullptr,
                int i0 = 0, int nv = 0, int pin = 0) {
  MVDev& D = h->mv[n];
  if (D.need_xt) HIPCHK(launch_transpose_plr(0, x, h->d_xt, D.dims[0], D.dims[1], D.dims[2], s));
  run_mp(D.chainA, 0, x, s);
  run_mp(D.chainB, 0, x, s);
  run_mp(D.chainC, 0, x, s);
  run_sw_mv(h, D.sw, 0, x, s);
  if (D.srcs.empty()) {
    HIPCHK(launch_zero(y, (int64_t)D.dims[0] * D.dims[1] * D.dims[2], s));
    if (J) HIPCHK(launch_kdots(J, 1, i0, nv, pin, s));
  } else if (J) {
    HIPCHK(launch_reduce_dots(D.d_srcs, (int)D.srcs.size(), J, D.dims[0], D.dims[1], D.dims[2], i0, nv, pin, s));
  } else {
    HIPCHK(launch_reduce_out(0, D.d_srcs, (int)D.srcs.size(), y, 0, D.dims[0], D.dims[1], D.dims[2], s));
  }
  h->n_matvec++;
  h->mv_flops += (double)h->M.mv[n].flops;
}

// ------------------------------------------------------------------ low-precision forms
// Mirror formats: 1 = FP32 (same layout as the FP64 blocks), 2 = split BF16
// (hi and lo planes, permuted row-major, for blocks whose dimension is a
// multiple of 32).  Both take 4 bytes per element, so a mirror element sits at
// half the byte offset of its FP64 original.
bool sw_bf16(int ma, int mb) { return ma % 32 == 0 && mb % 32 == 0 && ma <= 128 && mb <= 128; }

void* to_mirror(attn_handle* h, const void* p, int fmt) {
  if (!p) return nullptr;
  const uintptr_t a = (uintptr_t)p;
  const uintptr_t c0 = (uintptr_t)h->d_mvcomb;
  if (a >= c0 && a < c0 + (uintptr_t)h->mvcomb_elems * 8) return (char*)h->comb_lp[fmt - 1] + (a - c0) / 2;
  const Tree& tr = h->M.tree;
  for (int dir = 0; dir < 2; dir++)
    for (int e = 0; e < tr.n_edges(); e++) {
      const uintptr_t b = (uintptr_t)h->store[dir][e];
      if (b && a >= b && a < b + (uintptr_t)h->store_elems[dir][e] * 8) {
        void* m = h->mir[fmt - 1][dir][e];
        if (!m) throw StatusFail{ATTN_ERR_STATE, "internal: block without mirror"};
        return (char*)m + (a - b) / 2;
      }
    }
  throw StatusFail{ATTN_ERR_STATE, "internal: block outside every store"};
}

// The split-BF16 kernel at legs 64 x 64 keeps one workgroup of eight waves
// resident per CU (two waves per SIMD), so a launch takes ceil(W / 256)
// rounds of W workgroups.  Its tasks (copied from the FP64 plan, W = tasks x slices / 4)
// are re-cut into fewer, longer item ranges so that W is a multiple of 512:
// per class of tasks with the same slice geometry, the items are shared out
// over fewer tasks in proportion to the class's item count, each new task
// writing the partial output of one of the class's old tasks; the outputs
// left unwritten are added to `dropped`.
void rechunk_bf16(SWGroup& g, std::vector<int>& ns_of, std::vector<RDSrc>& srcs, std::vector<const void*>& dropped) {
  (void)srcs;
  const int nt = (int)g.tasks.size();
  if (nt == 0) return;
  for (const SWTask& t : g.tasks)
    if (t.pad) return;
  int64_t W = 0;
  for (int t = 0; t < nt; t++) W += (ns_of[t] + 3) / 4;
  const int64_t kRound = 512;   // two rounds; cutting to multiples of 256 measured slower (220 vs 241 TFLOP/s)
  if (W <= kRound || W % kRound == 0) return;
  const int64_t Wt = kRound * (W / kRound);
  // classes of tasks with one slice geometry (consecutive in task order)
  std::vector<std::vector<int>> cls;
  for (int t = 0; t < nt; t++) {
    const SWTask& a = g.tasks[t];
    bool found = false;
    for (auto& c : cls) {
      const SWTask& b = g.tasks[c[0]];
      if (a.x == b.x && a.xs_slice == b.xs_slice && a.xs_row == b.xs_row && a.ys_slice == b.ys_slice &&
          a.ys_row == b.ys_row && ns_of[t] == ns_of[c[0]] && a.accumulate == b.accumulate) {
        c.push_back(t);
        found = true;
        break;
      }
    }
    if (!found) cls.push_back({t});
  }
  const int nc = (int)cls.size();
  std::vector<int64_t> items(nc, 0), units(nc, 0);
  int64_t tot_items = 0;
  for (int c = 0; c < nc; c++) {
    for (int t : cls[c]) items[c] += g.tasks[t].nitem;
    units[c] = (ns_of[cls[c][0]] + 3) / 4;
    tot_items += items[c];
  }
  // tasks per class: the workgroup target in proportion to item counts
  std::vector<int> keep(nc, 1);
  int64_t used = 0;
  for (int c = 0; c < nc; c++) used += units[c];
  for (int c = 0; c < nc; c++) {
    const int64_t want = Wt * items[c] / std::max<int64_t>(1, tot_items) / units[c];
    keep[c] = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cls[c].size(), want));
  }
  int64_t w = 0;
  for (int c = 0; c < nc; c++) w += keep[c] * units[c];
  for (int guard = 0; w < Wt && guard < 4096; guard++) {   // top up the classes with the most items per task
    int best = -1;
    for (int c = 0; c < nc; c++)
      if (keep[c] < (int)cls[c].size() && w + units[c] <= Wt &&
          (best < 0 || items[c] * keep[best] > items[best] * keep[c]))
        best = c;
    if (best < 0) break;
    keep[best]++;
    w += units[best];
  }
  if (w % kRound != 0) return;   // no exact cut: keep the plan as it is
  std::vector<SWTask> tasks;
  std::vector<SWItem> its;
  std::vector<int> nns;
  for (int c = 0; c < nc; c++) {
    std::vector<SWItem> ci;
    for (int t : cls[c])
      for (int i = g.tasks[t].item0; i < g.tasks[t].item0 + g.tasks[t].nitem; i++) ci.push_back(g.items[i]);
    const int k = keep[c];
    for (int j = 0; j < k; j++) {
      SWTask t = g.tasks[cls[c][j]];
      const size_t i0 = ci.size() * j / k, i1 = ci.size() * (j + 1) / k;
      t.item0 = (int)its.size();
      t.nitem = (int)(i1 - i0);
      its.insert(its.end(), ci.begin() + i0, ci.begin() + i1);
      tasks.push_back(t);
      nns.push_back(ns_of[cls[c][j]]);
    }
    for (size_t j = k; j < cls[c].size(); j++) dropped.push_back(g.tasks[cls[c][j]].y);
  }
  g.tasks.swap(tasks);
  g.items.swap(its);
  ns_of.swap(nns);
}

// Build the mirrors and the work lists of precision form `dtype` (1 = FP32,
// 2 = split BF16; the latter runs its mode products and the sandwich groups
// whose legs are not multiples of 32 in FP32).
void ensure_lowp(attn_handle* h, int dtype) {
  if (h->lowp_ready[dtype - 1]) return;
  const Tree& tr = h->M.tree;
  for (int fmt = 1; fmt <= dtype; fmt++) {
    if (!h->mir[fmt - 1][0].empty()) continue;
    for (int dir = 0; dir < 2; dir++) {
      h->mir[fmt - 1][dir].assign(tr.n_edges(), nullptr);
      for (int e = 0; e < tr.n_edges(); e++)
        if (h->store[dir][e] && (fmt == 1 || tr.edge_dim(e) % 32 == 0))
          h->mir[fmt - 1][dir][e] = dev_alloc(h, h->store_elems[dir][e] * 4);
    }
    h->comb_lp[fmt - 1] = dev_alloc(h, std::max<int64_t>(h->mvcomb_elems, 1) * 4);
  }
  std::vector<MVDev>& LP = h->mvlp[dtype - 1];
  LP.assign(tr.nodes.size(), MVDev());
  for (size_t n = 0; n < tr.nodes.size(); n++) {
    const MVDev& D = h->mv[n];
    MVDev& L = LP[n];
    L.need_xt = D.need_xt;
    std::copy(D.dims, D.dims + 3, L.dims);
    L.sw = D.sw;
    L.srcs = D.srcs;
    std::vector<const void*> dropped;   // partial outputs no task of this form writes
    for (auto& g : L.sw) {
      bool bf = dtype == 2 && sw_bf16(g.ma, g.mb);
      if (bf)
        for (auto& it : g.items) {
          if ((uintptr_t)to_mirror(h, it.A, 2) % 16 || (uintptr_t)to_mirror(h, it.B, 2) % 16) bf = false;
        }
      g.fmt = bf ? 2 : 1;
      for (auto& it : g.items) { it.A = to_mirror(h, it.A, g.fmt); it.B = to_mirror(h, it.B, g.fmt); }
      if (bf && g.ma <= 64 && g.mb <= 64) {
        // one slice per wave: units of up to four consecutive slices of a task
        std::vector<int> ns_of(g.tasks.size(), 0);
        for (const int4& wu : g.wus) ns_of[wu.x] = std::max(ns_of[wu.x], wu.y + 1);
        rechunk_bf16(g, ns_of, L.srcs, dropped);
        std::vector<int4> w2;
        for (size_t ti = 0; ti < g.tasks.size(); ti++)
          for (int s0 = 0; s0 < ns_of[ti]; s0 += 4) w2.push_back(make_int4((int)ti, s0, 0, std::min(4, ns_of[ti] - s0)));
        g.wus.swap(w2);
        g.fmt = 3;
      }
      if (dtype == 1 && g.ma == 64 && g.mb == 64) {
        // FP32 at legs 64: two row strips per wave, units of up to two slices
        std::vector<int> ns_of(g.tasks.size(), 0);
        for (const int4& wu : g.wus) ns_of[wu.x] = std::max(ns_of[wu.x], wu.y + 1);
        std::vector<int4> w2;
        for (size_t ti = 0; ti < g.tasks.size(); ti++)
          for (int s0 = 0; s0 < ns_of[ti]; s0 += 2) w2.push_back(make_int4((int)ti, s0, 0, std::min(2, ns_of[ti] - s0)));
        g.wus.swap(w2);
        g.fmt = 4;
      }
    }
    const std::vector<MPGroup>* src[3] = {&D.chainA, &D.chainB, &D.chainC};
    std::vector<MPGroup>* dst[3] = {&L.chainA, &L.chainB, &L.chainC};
    for (int k = 0; k < 3; k++) {
      *dst[k] = *src[k];
      for (auto& g : *dst[k])
        for (auto& jb : g.jobs) jb.A = to_mirror(h, jb.A, 1);
    }
    if (!dropped.empty()) {
      std::vector<RDSrc> keep;
      for (const RDSrc& r : L.srcs)
        if (std::find(dropped.begin(), dropped.end(), r.p) == dropped.end()) keep.push_back(r);
      L.srcs.swap(keep);
    }
    upload_sw(h, L.sw, true);
    upload_mp(h, L.chainA);
    upload_mp(h, L.chainB);
    upload_mp(h, L.chainC);
    L.d_srcs = upload(h, L.srcs);
  }
  h->lowp_ready[dtype - 1] = true;
}

// Conversion list that refreshes the mirrors read by node n's matvec in form
// `dtype`: its three incoming stores and its combined blocks.
std::vector<CVTask> lowp_conversions(attn_handle* h, int n, int dtype) {
  const Tree& tr = h->M.tree;
  std::vector<CVTask> cv;
  auto add = [&](const double* src, void* dst, int64_t elems, int dim, int fmt) {
    if (dst) cv.push_back({src, dst, elems, dim, fmt});
  };
  auto add_store = [&](int dir, int e) {
    if (e < 0 || !h->store[dir][e]) return;
    const int dim = tr.edge_dim(e);
    for (int fmt = 1; fmt <= dtype; fmt++)
      add(h->store[dir][e], h->mir[fmt - 1][dir][e], h->store_elems[dir][e], dim, fmt);
  };
  add_store(0, tr.edge_of_child(n, 0));
  add_store(0, tr.edge_of_child(n, 1));
  if (n != tr.root) add_store(1, tr.edge_of_node(n));
  for (auto& cb : h->comb_blocks[n]) {
    const int64_t el = (int64_t)cb.second * cb.second;
    for (int fmt = 1; fmt <= dtype; fmt++)
      if (fmt == 1 || cb.second % 32 == 0)
        add(h->d_mvcomb + cb.first, (char*)h->comb_lp[fmt - 1] + cb.first * 4, el, cb.second, fmt);
  }
  return cv;
}

void prepare_lowp(attn_handle* h, int n, int dtype, hipStream_t s) {
  std::vector<CVTask> cv = lowp_conversions(h, n, dtype);
  int64_t maxn = 0;
  for (auto& c : cv) maxn = std::max(maxn, c.n);
  if (cv.size() > (size_t)h->cv_cap) throw StatusFail{ATTN_ERR_STATE, "internal: conversion list too long"};
  HIPCHK(hipMemcpyAsync(h->d_cvtasks, cv.data(), cv.size() * sizeof(CVTask), hipMemcpyHostToDevice, s));
  HIPCHK(launch_convert(dtype, (const CVTask*)h->d_cvtasks, (int)cv.size(), maxn, s));
  // the host list must outlive the asynchronous copy
  HIPCHK(hipStreamSynchronize(s));
}

// y <- H_eff(n) x in form `dtype` (mirrors current); x is FP32, y FP64
// (out_dtype 0) or FP32 (out_dtype 1).
void matvec_lowp(attn_handle* h, int n, int dtype, const float* x, void* y, int out_dtype, hipStream_t s) {
  MVDev& D = h->mvlp[dtype - 1][n];
  if (D.need_xt) HIPCHK(launch_transpose_plr(1, x, h->d_xt, D.dims[0], D.dims[1], D.dims[2], s));
  run_mp(D.chainA, 1, x, s);
  run_mp(D.chainB, 1, x, s);
  run_mp(D.chainC, 1, x, s);
  run_sw_mv(h, D.sw, 1, x, s);
  const int64_t M = (int64_t)D.dims[0] * D.dims[1] * D.dims[2];
  if (D.srcs.empty()) {
    HIPCHK(hipMemsetAsync(y, 0, (size_t)M * (out_dtype == 0 ? 8 : 4), s));
  } else {
    HIPCHK(launch_reduce_out(1, D.d_srcs, (int)D.srcs.size(), y, out_dtype, D.dims[0], D.dims[1], D.dims[2], s));
  }
  h->n_matvec++;
  h->mv_flops += (double)h->M.mv[n].flops;
}

int leg_toward(const Tree& tr, int a, int b) {
  if (tr.nodes[a].parent == b) return 2;
  if (tr.nodes[a].child[0] == b) return 0;
  if (tr.nodes[a].child[1] == b) return 1;
  return -1;
}

// Mark stale every store whose source side contains node n.
void invalidate_from(attn_handle* h, int n) {
  const Tree& tr = h->M.tree;
  const Node& nd = tr.nodes[n];
  for (int c = 0; c < (int)tr.nodes.size(); c++) {
    if (c == tr.root) continue;
    const Node& cn = tr.nodes[c];
    const int e = tr.edge_of_node(c);
    const bool below = nd.lo >= cn.lo && nd.hi <= cn.hi;   // n inside subtree(c)
    if (below) h->valid[0][e] = 0;
    else h->valid[1][e] = 0;
  }
}

bool incoming_valid(attn_handle* h, int n) {
  const Tree& tr = h->M.tree;
  for (int sd = 0; sd < 2; sd++) {
    const int e = tr.edge_of_child(n, sd);
    if (!tr.edge_is_site(e) && !h->valid[0][e]) return false;
  }
  if (n != tr.root && !h->valid[1][tr.edge_of_node(n)]) return false;
  return true;
}

void run_env(attn_handle* h, EnvDev& D, hipStream_t s) {
  run_comb(D.comb, s);
  if (D.transpose)
    HIPCHK(launch_transpose_plr(0, h->d_T + h->T_off[D.node], h->d_xt, D.dims[0], D.dims[1], D.dims[2], s));
  for (auto& ch : D.chunks) {
    for (auto& zb : ch.zero_blocks) HIPCHK(launch_zero(zb.first, zb.second, s));
    run_sw(ch.sw, 0, nullptr, s);
    HIPCHK(launch_gram(ch.gr.mj, ch.gr.mfma, ch.gr.d_tasks, (int)ch.gr.tasks.size(), s, ch.gr.nt));
    HIPCHK(launch_gram_reduce(ch.gr.d_reds, (int)ch.gr.reds.size(), ch.gr.mj, s));
  }
  h->n_env++;
}

void build_qr_dev(attn_handle* h, int n, int leg, QRDev& Q) {
  const Node& nd = h->M.tree.nodes[n];
  const int dm[3] = {nd.dims[0], nd.dims[1], nd.dims[2]};
  const int mj = dm[leg];
  const int64_t Msz = (int64_t)dm[0] * dm[1] * dm[2];
  const int64_t rows = Msz / mj;
  const int64_t nn = (int64_t)h->mmax * h->mmax;
  double* T = h->d_T + h->T_off[n];
  double* G = h->d_qrmat;
  double* Rinv = G + 4 * nn;
  Q.present = true;
  Q.mj = mj; Q.rows = rows; Q.Msz = Msz;
  Q.gmf = gram_mfma_ok(mj, Msz);
  int64_t fchunk = rows;
  if (Q.gmf) {
    fchunk = std::max<int64_t>(64, ((rows / 32) + 63) / 64 * 64);
    while (rows % fchunk) fchunk += 64;
  }
  Q.nfc = (int)(rows / fchunk);
  GRReduce gr;
  gr.partial = h->d_grpart; gr.out = G; gr.m = mj; gr.npart = Q.nfc; gr.coef = 1.0; gr.accumulate = 0; gr.pad = 0;
  Q.d_gr = upload(h, std::vector<GRReduce>{gr});
  Q.h_gr = {gr};
  Q.mmf = mode_mfma_ok(mj, Msz);
  std::vector<int2> wus;
  if (Q.mmf) for (int64_t f = 0; f < rows / 64; f++) wus.push_back(make_int2(0, (int)f));
  else for (int64_t e = 0; e < Msz; e += 256) wus.push_back(make_int2(0, (int)e));
  Q.nwus = (int)wus.size();
  Q.d_wus = upload(h, wus);
  // the passes rotate through T -> tmp -> tmp2 -> T, so Q lands in T
  double* const bufs[4] = {T, h->d_tmp, h->d_tmp2, T};
  for (int pass = 0; pass < 3; pass++) {
    double* src = bufs[pass];
    double* dst = bufs[pass + 1];
    std::vector<GRTask> gt(Q.nfc);
    for (int c = 0; c < Q.nfc; c++) {
      gt[c].X = src; gt[c].Z = src; gt[c].partial = h->d_grpart + (int64_t)c * mj * mj;
      gt[c].d0 = dm[0]; gt[c].d1 = dm[1]; gt[c].d2 = dm[2]; gt[c].j = leg;
      gt[c].f0 = (int)(c * fchunk); gt[c].f1 = (int)((c + 1) * fchunk);
    }
    Q.gnt = gram_nt_ok(gt, Q.gmf) && (pass == 0 || Q.gnt);
    Q.d_gt[pass] = upload(h, gt);
    Q.h_gt[pass] = gt;
    MPTask mt{dst, dm[0], dm[1], dm[2], leg, 0, 1, 0, 0};
    Q.d_mt[pass] = upload(h, std::vector<MPTask>{mt});
    MPJob mjb{Rinv, src, 1.0};
    Q.d_mj[pass] = upload(h, std::vector<MPJob>{mjb});
    Q.h_mp[pass].mj = mj;
    Q.h_mp[pass].mfma = Q.mmf;
    Q.mnt = mode_nt_ok({mt}, Q.mmf);
    Q.h_mp[pass].tasks = {mt};
    Q.h_mp[pass].jobs = {mjb};
    Q.h_mp[pass].wus = wus;
  }
}

void build_ab_dev(attn_handle* h, int q, int leg, ABDev& A) {
  const Node& nd = h->M.tree.nodes[q];
  const int dm[3] = {nd.dims[0], nd.dims[1], nd.dims[2]};
  const int mj = dm[leg];
  const int64_t Msz = (int64_t)dm[0] * dm[1] * dm[2];
  double* T = h->d_T + h->T_off[q];
  A.present = true;
  A.mj = mj; A.Msz = Msz;
  A.mmf = mode_mfma_ok(mj, Msz);
  std::vector<int2> wus;
  if (A.mmf) for (int64_t f = 0; f < Msz / mj / 64; f++) wus.push_back(make_int2(0, (int)f));
  else for (int64_t e = 0; e < Msz; e += 256) wus.push_back(make_int2(0, (int)e));
  A.nwus = (int)wus.size();
  A.d_wus = upload(h, wus);
  MPTask mt{h->d_tmp2, dm[0], dm[1], dm[2], leg, 0, 1, 0, 0};
  A.d_mt = upload(h, std::vector<MPTask>{mt});
  MPJob mjb{h->d_qrR, T, 1.0};
  A.d_mj = upload(h, std::vector<MPJob>{mjb});
  A.h_mp.mj = mj;
  A.h_mp.mfma = A.mmf;
  A.mnt = mode_nt_ok({mt}, A.mmf);
  A.h_mp.tasks = {mt};
  A.h_mp.jobs = {mjb};
  A.h_mp.wus = wus;
}

// QR of T_n with leg `leg` as the column index (shifted CholeskyQR followed by
// two CholeskyQR passes): T_n <- Q in place, R (column-major) into d_qrR.
bool qr_small_ok(const int* dm, int leg) {
  const int64_t M = (int64_t)dm[0] * dm[1] * dm[2];
  return dm[leg] <= 64 && M <= 4096;
}

void qr_node(attn_handle* h, int n, int leg, hipStream_t s) {
  QRDev& Q = h->qr[leg][n];
  if (!Q.present) throw StatusFail{ATTN_ERR_STATE, "internal: no QR plan for this leg"};
  const Node& nd = h->M.tree.nodes[n];
  if (qr_small_ok(nd.dims, leg)) {
    HIPCHK(launch_qr_small(h->d_T + h->T_off[n], nd.dims[0], nd.dims[1], nd.dims[2], leg, h->d_qrR,
                           h->d_st, s));
    h->n_qr++;
    return;
  }
  const int mj = Q.mj;
  const int64_t nn = (int64_t)h->mmax * h->mmax;
  double* G = h->d_qrmat;
  double* R[3] = {G + nn, G + 2 * nn, G + 3 * nn};
  double* Rinv = G + 4 * nn;
  double* Rt = G + 5 * nn;
  double* ws = G + 6 * nn;   // Cholesky workspace for links wider than 128
  // the passes rotate T -> tmp -> tmp2 -> T (plans built that way): Q ends in T
  for (int pass = 0; pass < 3; pass++) {
    HIPCHK(launch_gram(mj, Q.gmf, Q.d_gt[pass], Q.nfc, s, Q.gnt));
    HIPCHK(launch_gram_reduce(Q.d_gr, 1, mj, s));
    HIPCHK(launch_chol_inv(G, mj, R[pass], Rinv, pass == 0 ? 1 : 0, Q.rows, h->d_st, ws, s));
    HIPCHK(launch_mode(0, mj, Q.mmf, Q.d_mt[pass], Q.d_mj[pass], Q.d_wus, Q.nwus, nullptr, s, Q.mnt));
  }
  HIPCHK(launch_small_matmul(R[1], R[0], Rt, mj, s));
  HIPCHK(launch_small_matmul(R[2], Rt, h->d_qrR, mj, s));
  h->n_qr++;
}

// T_q <- R x_leg T_q with R in d_qrR
void absorb(attn_handle* h, int q, int leg, hipStream_t s) {
  ABDev& A = h->ab[leg][q];
  if (!A.present) throw StatusFail{ATTN_ERR_STATE, "internal: no absorb plan for this leg"};
  HIPCHK(launch_mode(0, A.mj, A.mmf, A.d_mt, A.d_mj, A.d_wus, A.nwus, nullptr, s, A.mnt));
  HIPCHK(launch_copy(h->d_T + h->T_off[q], h->d_tmp2, A.Msz, s));
}

attn_status guard(attn_handle* h, const std::function<attn_status()>& f) {
  if (!h) return ATTN_ERR_ARG;
  if (h->dead) { h->err = "handle unusable after an earlier HIP or numeric error"; return ATTN_ERR_STATE; }
  try {
    h->err.clear();
    return f();
  } catch (const HipFail& e) {
    h->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    h->dead = true;
    return ATTN_ERR_HIP;
  } catch (const StatusFail& e) {
    h->err = e.msg;
    if (e.st == ATTN_ERR_NUMERIC) h->dead = true;
    return e.st;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return ATTN_ERR_OOM;
  }
}

void check_state(attn_handle* h, hipStream_t s, const char* where) {
  KrylovState st;
  HIPCHK(hipMemcpyAsync(&st, h->d_st, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st.status != 0)
    throw StatusFail{ATTN_ERR_NUMERIC, std::string(where) + (st.status == 2 ? ": QR factorisation broke down" : ": non-finite value")};
}

void reset_state(attn_handle* h, int kmax, hipStream_t s) {
  HIPCHK(launch_kinit(h->d_kjobs64 + h->M.tree.root, 1, kmax, s));
}

attn_status need_device(attn_handle* h) {
  if (h->host_only) { h->err = "handle was built with ATTN_HOST_ONLY"; return ATTN_ERR_STATE; }
  if (h->dryrun) { h->err = "handle was built with ATTN_DRYRUN"; return ATTN_ERR_STATE; }
  return ATTN_OK;
}

// ------------------------------------------------------------------ eigensolver
double lanczos(attn_handle* h, int n, int kreq, int precision, int* nmv, hipStream_t s) {
  MVDev& D = h->mv[n];
  const int64_t Msz = (int64_t)D.dims[0] * D.dims[1] * D.dims[2];
  const int kk = std::min(kreq, h->kcap - 1);
  const int k = (int)std::min<int64_t>(kk, Msz);
  run_comb(D.comb, s);
  // tiny nodes (dense H_eff, negligible work) stay in FP64 for every form
  if (D.d_tiny) {
    HIPCHK(launch_tiny(h->d_tjobs + n, 1, (int)Msz, (int)Msz, kk, s));
    h->n_matvec += k;
    h->mv_flops += (double)k * h->M.mv[n].flops;
    if (h->defer_status) {
      if (nmv) *nmv = k;
      return std::nan("");
    }
    KrylovState st;
    HIPCHK(hipMemcpyAsync(&st, h->d_st, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st.status != 0 || !std::isfinite(st.scal[0])) throw StatusFail{ATTN_ERR_NUMERIC, "non-finite value in the eigensolver"};
    if (nmv) *nmv = k;
    return st.scal[0];
  }
  if (precision != ATTN_F64) {
    ensure_lowp(h, precision);
    prepare_lowp(h, n, precision, s);
  }
  // the low-precision job also writes an FP32 copy of each new basis vector
  const KJob* J = (precision == ATTN_F64 ? h->d_kjobs64 : h->d_kjobs32) + n;
  double* V = h->d_V;
  HIPCHK(launch_kinit(J, 1, k, s));
  HIPCHK(launch_knorm(J, 1, s));
  HIPCHK(launch_kscale(J, 1, Msz, 0, s));
  for (int j = 0; j < k; j++) {
    // dots after the product: V[0..j] . w into P1, or at the last step only
    // v_j . w (alpha_j) into P0
    const bool last = j == k - 1;
    const int i0 = last ? j : 0, nv = last ? 1 : j + 1, pin = last ? 0 : 1;
    if (precision == ATTN_F64) {
      matvec_f64(h, n, V + (int64_t)j * Msz, h->d_w, s, J, i0, nv, pin);
    } else {
      matvec_lowp(h, n, precision, h->d_x32, h->d_w, 0, s);
      HIPCHK(launch_kdots(J, 1, i0, nv, pin, s));
    }
    if (last) {
      HIPCHK(launch_kalpha(J, 1, j, s));
      break;
    }
    HIPCHK(launch_kortho(J, 1, j, 1, 0, 1, s));
    HIPCHK(launch_kortho(J, 1, j, 2, 1, 0, s));
    HIPCHK(launch_kbeta(J, 1, j, Msz, s));
  }
  HIPCHK(launch_ktridiag(J, 1, s));
  HIPCHK(launch_kritz(J, 1, s));
  HIPCHK(launch_kscale(J, 1, Msz, 1, s));
  if (h->defer_status) {
    if (nmv) *nmv = k;
    return std::nan("");
  }
  KrylovState st;
  HIPCHK(hipMemcpyAsync(&st, h->d_st, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st.status != 0 || !std::isfinite(st.scal[0])) throw StatusFail{ATTN_ERR_NUMERIC, "non-finite value in the eigensolver"};
  if (nmv) *nmv = k;
  return st.scal[0];
}


// ------------------------------------------------------------------ Davidson form
void ensure_davidson(attn_handle* h) {
  if (h->d_djobs) return;
  const Tree& tr = h->M.tree;
  const int nn = (int)tr.nodes.size();
  const int64_t Mx = h->Mmax;
  auto alloc = [&](int64_t n_doubles) { return (double*)dev_alloc(h, std::max<int64_t>(n_doubles, 1) * 8); };
  double* W = alloc((int64_t)kDavMax * Mx);
  double* Vt = alloc((int64_t)2 * kDavMax * Mx);
  double* u = alloc(Mx);
  double* r = alloc(Mx);
  double* t = alloc(Mx);
  double* dg = alloc(Mx);
  double* red = alloc((int64_t)8 * kDavMax * kRedBlocks);
  h->d_dav = (DavState*)dev_alloc(h, sizeof(DavState));
  if (!h->d_mlp) h->d_mlp = dev_alloc(h, kMlpParams * 2);
  h->h_djobs.resize(nn);
  for (int n = 0; n < nn; n++)
    h->h_djobs[n] = DJob{h->d_V, W, Vt, u, r, t, dg, h->d_T + h->T_off[n], red, h->d_dav, h->d_mlp, h->T_len[n]};
  h->d_djobs = upload(h, h->h_djobs);
}

// Davidson eigensolve at node n (the centre).  precond: ATTN_PRECOND_JACOBI or
// ATTN_PRECOND_LEARNED (falls back to Jacobi when the model's correction is
// not finite, or when its residual reduction is worse than the running Jacobi
// rate for two consecutive iterations).
double davidson(attn_handle* h, int n, const attn_solver_opts& o, int* nmv_out, hipStream_t s) {
  ensure_davidson(h);
  MVDev& D = h->mv[n];
  const int64_t Msz = h->T_len[n];
  const int restart = std::max(1, std::min(o.restart > 0 ? o.restart : 8, kDavMax / 2));
  const int maxsub = std::max(restart + 2, std::min(o.krylov_k, kDavMax));
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const double tol = o.tol > 0 ? o.tol : 1e-7;
  const DJob* J = h->d_djobs + n;
  const DJob& Jh = h->h_djobs[n];
  bool learned = o.precond == ATTN_PRECOND_LEARNED;
  run_comb(D.comb, s);
  if (o.precision != ATTN_F64) {
    ensure_lowp(h, o.precision);
    prepare_lowp(h, n, o.precision, s);
  }
  HIPCHK(launch_dav(0, J, 0, 0, tol, s));
  HIPCHK(launch_heff_diag(D.d_plan, J, Msz, s));
  HIPCHK(launch_dav(1, J, 0, 0, tol, s));
  HIPCHK(launch_dav(1, J, 0, 1, tol, s));
  int k = 1, nmv = 0, bad = 0;
  double prev = -1.0, rate_sum = 0;
  int rate_n = 0;
  DavState st;
  for (int it = 0; it < max_iter; it++) {
    double* v = Jh.V + (int64_t)(k - 1) * Msz;
    double* w = Jh.W + (int64_t)(k - 1) * Msz;
    if (o.precision == ATTN_F64) {
      matvec_f64(h, n, v, w, s);
    } else {
      HIPCHK(launch_cast(v, 0, h->d_x32, 1, Msz, s));
      matvec_lowp(h, n, o.precision, h->d_x32, w, 0, s);
    }
    nmv++;
    HIPCHK(launch_dav(2, J, k, 0, tol, s));
    HIPCHK(launch_dav(3, J, k, 0, tol, s));
    HIPCHK(launch_dav(4, J, k, 0, tol, s));
    HIPCHK(launch_dav(learned ? 6 : 5, J, k, 0, tol, s));
    HIPCHK(launch_dav(7, J, k, 0, tol, s));
    HIPCHK(hipMemcpyAsync(&st, h->d_dav, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->n_dav_iter++;
    if (st.status == 1) throw StatusFail{ATTN_ERR_NUMERIC, "non-finite value in the Davidson eigensolver"};
    if (st.converged) break;
    if (learned && st.tbad) {   // model output not finite: Jacobi for the rest of the solve
      learned = false;
      h->n_fallback++;
      HIPCHK(launch_dav(5, J, k, 0, tol, s));
    } else if (learned && prev > 0) {
      bad = st.rnorm / prev > h->jacobi_rate ? bad + 1 : 0;
      if (bad >= 2) { learned = false; h->n_fallback++; }
    }
    if (!learned && prev > 0) { rate_sum += st.rnorm / prev; rate_n++; }
    prev = st.rnorm;
    HIPCHK(launch_dav(8, J, k, 5, tol, s));
    HIPCHK(launch_dav(9, J, k, 6, tol, s));
    if (k == maxsub) {
      HIPCHK(launch_dav(11, J, k, restart, tol, s));
      HIPCHK(hipMemcpyAsync(Jh.V, Jh.Vt, (size_t)restart * Msz * 8, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(Jh.W, Jh.Vt + (int64_t)restart * Msz, (size_t)restart * Msz * 8,
                            hipMemcpyDeviceToDevice, s));
      k = restart;
    }
    HIPCHK(launch_dav(10, J, k, k, tol, s));
    HIPCHK(hipMemcpyAsync(&st, h->d_dav, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st.status == 2 && learned) {
      // the model's correction adds nothing to the basis: Jacobi from here on
      // (r is unchanged; the Jacobi prologue clears the status)
      learned = false;
      h->n_fallback++;
      HIPCHK(launch_dav(5, J, k, 0, tol, s));
      HIPCHK(launch_dav(8, J, k, 5, tol, s));
      HIPCHK(launch_dav(9, J, k, 6, tol, s));
      HIPCHK(launch_dav(10, J, k, k, tol, s));
      HIPCHK(hipMemcpyAsync(&st, h->d_dav, sizeof(st), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    if (st.status == 2) break;   // the correction lies in the basis: nothing left to add
    k++;
  }
  if (rate_n > 0) h->jacobi_rate = 0.5 * h->jacobi_rate + 0.5 * (rate_sum / rate_n);
  HIPCHK(launch_dav(12, J, k, 0, tol, s));
  HIPCHK(hipMemcpyAsync(&st, h->d_dav, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st.status == 1 || !std::isfinite(st.theta)) throw StatusFail{ATTN_ERR_NUMERIC, "non-finite value in the Davidson eigensolver"};
  h->last_rnorm = st.rnorm;
  h->n_matvec += nmv;
  if (nmv_out) *nmv_out = nmv;
  return st.theta;
}
}  // namespace rt

// ====================================================================== C interface
extern "C" {

attn_status attn_build_tpo(const attn_problem* p, attn_handle** out) {
  if (!out) { g_build_error = "out is NULL"; return ATTN_ERR_ARG; }
  *out = nullptr;
  attn_handle* h = new (std::nothrow) attn_handle();
  if (!h) { g_build_error = "host allocation failed"; return ATTN_ERR_OOM; }
  std::string err;
  attn_status st;
  try {
    st = build_model(p, h->M, err);
  } catch (const std::bad_alloc&) {
    st = ATTN_ERR_OOM;
    err = "host allocation failed";
  }
  if (st != ATTN_OK) {
    g_build_error = err;
    delete h;
    return st;
  }
  try {
    h->prob.assign(p);
  } catch (const std::bad_alloc&) {
    g_build_error = "host allocation failed";
    delete h;
    return ATTN_ERR_OOM;
  }
  h->problem_hash = h->prob.hash();
  h->host_only = (p->flags & ATTN_HOST_ONLY) != 0;
  h->dryrun = (p->flags & ATTN_DRYRUN) != 0;
  h->device = p->device;
  const Tree& tr = h->M.tree;
  const int nn = (int)tr.nodes.size();
  h->iso.assign(nn, 2);
  h->iso[tr.root] = -1;
  h->center = tr.root;
  h->valid[0].assign(tr.n_edges(), 0);
  h->valid[1].assign(tr.n_edges(), 0);
  for (int s = 0; s < tr.N; s++) h->valid[0][s] = 1;
  if (h->host_only) {
    *out = h;
    return ATTN_OK;
  }
  try {
    if (!h->dryrun) {
      HIPCHK(hipSetDevice(h->device));
      HIPCHK(prepare_kernel_attributes());
    }
    // tensors
    int64_t tot = 0;
    for (int n = 0; n < nn; n++) {
      const Node& nd = tr.nodes[n];
      const int64_t Msz = (int64_t)nd.dims[0] * nd.dims[1] * nd.dims[2];
      h->T_off.push_back(tot);
      h->T_len.push_back(Msz);
      tot += Msz;
      h->Mmax = std::max(h->Mmax, Msz);
    }
    h->d_T = (double*)dev_alloc(h, tot * sizeof(double));
    // effective-operator stores
    h->store[0].assign(tr.n_edges(), nullptr);
    h->store[1].assign(tr.n_edges(), nullptr);
    h->store_elems[0].assign(tr.n_edges(), 0);
    h->store_elems[1].assign(tr.n_edges(), 0);
    for (int e = 0; e < tr.n_edges(); e++) {
      const int dim = tr.edge_dim(e);
      const int64_t sz = (int64_t)(1 + h->M.n_slots[e]) * dim * dim;
      if (tr.edge_is_site(e)) {
        h->store[0][e] = upload(h, h->M.site_blocks[e]);
        h->store_elems[0][e] = (int64_t)h->M.site_blocks[e].size();
        continue;
      }
      for (int dir = 0; dir < 2; dir++) {
        h->store_elems[dir][e] = sz;
        void* q = dev_alloc(h, sz * sizeof(double));
        if (!h->dryrun) HIPCHK(hipMemset(q, 0, sz * sizeof(double)));
        h->store[dir][e] = (double*)q;
      }
    }
    // scratch sizing
    int64_t part_need = 0, chain_need = 0, mvcomb_need = 0, envcomb_need = 0, z_need = 0, grp_need = 0;
    for (int n = 0; n < nn; n++) {
      const Node& nd = tr.nodes[n];
      const int dm[3] = {nd.dims[0], nd.dims[1], nd.dims[2]};
      const int64_t Msz = (int64_t)dm[0] * dm[1] * dm[2];
      const MatvecPlan& P = h->M.mv[n];
      int nparts = 0, nchs[3];
      const int64_t target[3] = {kMvTarget, kMvTarget, kMvTarget};
      mv_chunks(P, dm, target, nchs);
      for (int sp = 0; sp < 3; sp++) nparts += nchs[sp];
      part_need = std::max(part_need, nparts * Msz);
      int64_t cn = 0;
      for (auto& ch : P.chains) cn += (int64_t)(ch.O1.size() + ch.O2.size());
      cn += 3;
      chain_need = std::max(chain_need, cn * Msz);
      int64_t cb = 0;
      for (auto& c : P.combines) cb += (int64_t)c.dim * c.dim;
      mvcomb_need = std::max(mvcomb_need, cb);
      const EnvPlan* eps[3] = {&h->M.env_up[n], &h->M.env_down[0][n], &h->M.env_down[1][n]};
      for (const EnvPlan* ep : eps) {
        if (ep->node < 0) continue;
        int64_t c2 = 0;
        for (auto& c : ep->combines) c2 += (int64_t)c.dim * c.dim;
        envcomb_need = std::max(envcomb_need, c2);
        const int64_t per = env_chunk_outputs(h, Msz);
        int cap = 0;
        const std::vector<int> pcs = env_pieces(h->M, *ep, cap);
        int64_t nz = 0;
        for (int pc : pcs) nz += pc;
        // a chunk holds at most `per` pieces, or one output with more
        int64_t maxp = 0;
        for (int pc : pcs) maxp = std::max<int64_t>(maxp, pc);
        const int64_t nout = std::max<int64_t>(1, std::max(std::min<int64_t>(per, nz), maxp));
        z_need = std::max(z_need, nout * Msz);
        const int mj = dm[ep->leg];
        grp_need = std::max(grp_need, nout * 8 * (int64_t)mj * mj + (int64_t)mj * mj);
      }
      for (int leg = 0; leg < 3; leg++) grp_need = std::max(grp_need, (int64_t)64 * dm[leg] * dm[leg]);
    }
    auto alloc = [&](int64_t n_doubles) -> double* {
      return (double*)dev_alloc(h, std::max<int64_t>(n_doubles, 1) * sizeof(double));
    };
    h->d_V = alloc((int64_t)h->kcap * h->Mmax);
    h->d_w = alloc(h->Mmax);
    h->d_xt = alloc(h->Mmax);
    h->d_tmp = alloc(h->Mmax);
    h->d_tmp2 = alloc(std::max<int64_t>(h->Mmax, (int64_t)1024 * 1024));
    h->d_x32 = (float*)alloc(h->Mmax);
    h->d_y32 = (float*)alloc(h->Mmax);
    h->part_cap = std::max<int64_t>(part_need, 1);
    h->d_part = alloc(h->part_cap);
    h->chain_cap = std::max<int64_t>(chain_need, 1);
    h->d_chain = alloc(h->chain_cap);
    h->d_mvcomb = alloc(mvcomb_need);
    h->mvcomb_elems = mvcomb_need;
    h->d_envcomb = alloc(envcomb_need);
    h->d_Z = alloc(z_need);
    h->d_grpart = alloc(grp_need);
    h->d_red = alloc((int64_t)4 * 64 * kRedBlocks);
    for (int n = 0; n < nn; n++)
      for (int l = 0; l < 3; l++) h->mmax = std::max(h->mmax, tr.nodes[n].dims[l]);
    h->d_qrmat = alloc(qrmat_doubles(h->mmax));
    h->d_qrR = alloc((int64_t)h->mmax * h->mmax);
    h->cv_cap = 6 + 2 * (int)std::max<size_t>(1, [&] { size_t mx = 0; for (int n = 0; n < nn; n++) mx = std::max(mx, h->M.mv[n].combines.size()); return mx; }());
    h->d_cvtasks = dev_alloc(h, (size_t)h->cv_cap * sizeof(CVTask));
    h->d_st = (KrylovState*)dev_alloc(h, sizeof(KrylovState));
    // device plans
    h->mv.assign(nn, MVDev());
    h->comb_blocks.assign(nn, {});
    h->env_up.assign(nn, EnvDev());
    h->env_down[0].assign(nn, EnvDev());
    h->env_down[1].assign(nn, EnvDev());
    for (int l = 0; l < 3; l++) {
      h->qr[l].assign(nn, QRDev());
      h->ab[l].assign(nn, ABDev());
    }
    for (int n = 0; n < nn; n++) {
      std::vector<int64_t> off;
      build_mv_dev(h, n, off);
      const Node& nd = tr.nodes[n];
      if (n != tr.root) {
        build_qr_dev(h, n, 2, h->qr[2][n]);
        build_ab_dev(h, n, 2, h->ab[2][n]);   // R from a parent moving down
      }
      for (int sd = 0; sd < 2; sd++)
        if (nd.child[sd] >= 0) {
          build_qr_dev(h, n, sd, h->qr[sd][n]);
          build_ab_dev(h, n, sd, h->ab[sd][n]);   // R from a child moving up
        }
      if (n != tr.root) build_env_dev(h, h->M.env_up[n], h->env_up[n]);
      for (int sd = 0; sd < 2; sd++) build_env_dev(h, h->M.env_down[sd][n], h->env_down[sd][n]);
    }
    // eigensolver job descriptors, one per node (the FP32 one also keeps an
    // FP32 copy of the newest basis vector for the low-precision matvec)
    std::vector<KJob> kj64(nn), kj32(nn);
    std::vector<TJob> tj(nn);
    for (int n = 0; n < nn; n++) {
      const int64_t Msz = h->T_len[n];
      double* T = h->d_T + h->T_off[n];
      kj64[n] = KJob{h->d_V, h->d_w, T, h->d_red, h->d_st, nullptr, nullptr, Msz};
      kj32[n] = kj64[n];
      kj32[n].x32 = h->d_x32;
      tj[n] = TJob{h->mv[n].d_tiny, h->d_tmp2, T, h->d_V, h->d_w, h->d_st, (int32_t)Msz, 0};
    }
    h->h_kjobs = kj64;
    h->h_tjobs = tj;
    h->d_kjobs64 = upload(h, kj64);
    h->d_kjobs32 = upload(h, kj32);
    h->d_tjobs = upload(h, tj);
    if (!h->dryrun) HIPCHK(hipDeviceSynchronize());
  } catch (const HipFail& e) {
    g_build_error = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    attn_destroy(h);
    return e.e == hipErrorOutOfMemory ? ATTN_ERR_OOM : ATTN_ERR_HIP;
  } catch (const StatusFail& e) {
    g_build_error = e.msg;
    attn_destroy(h);
    return e.st;
  }
  *out = h;
  return ATTN_OK;
}

attn_status attn_destroy(attn_handle* h) {
  if (!h) return ATTN_OK;
  if (!h->host_only && !h->dryrun) {
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (void* p : h->owned) (void)hipFree(p);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (auto& g : h->sgraphs) (void)hipGraphExecDestroy(g.exec);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
  }
  delete h;
  return ATTN_OK;
}

const char* attn_last_error(const attn_handle* h) {
  if (!h) return g_build_error.c_str();
  return h->err.c_str();
}

attn_status attn_node_info(const attn_handle* h, int32_t node, int32_t dims[3], int32_t* n_cross,
                           double* flops) {
  if (!h) return ATTN_ERR_ARG;
  const Tree& tr = h->M.tree;
  if (node < 0 || node >= (int)tr.nodes.size()) return ATTN_ERR_ARG;
  if (dims) for (int i = 0; i < 3; i++) dims[i] = tr.nodes[node].dims[i];
  if (n_cross) *n_cross = h->M.mv[node].n_cross;
  if (flops) *flops = (double)h->M.mv[node].flops;
  return ATTN_OK;
}

attn_status attn_tree_info(const attn_handle* h, int32_t* n_nodes, int32_t* root, int64_t* env_bytes) {
  if (!h) return ATTN_ERR_ARG;
  const Tree& tr = h->M.tree;
  if (n_nodes) *n_nodes = (int)tr.nodes.size();
  if (root) *root = tr.root;
  if (env_bytes) {
    int64_t b = 0;
    for (int e = 0; e < tr.n_edges(); e++) {
      const int dim = tr.edge_dim(e);
      b += (int64_t)(1 + h->M.n_slots[e]) * dim * dim * 8 * (tr.edge_is_site(e) ? 1 : 2);
    }
    *env_bytes = b;
  }
  return ATTN_OK;
}

attn_status attn_get_center(const attn_handle* h, int32_t* node) {
  if (!h || !node) return ATTN_ERR_ARG;
  *node = h->center;
  return ATTN_OK;
}

attn_status attn_counters(const attn_handle* h, int64_t* n_matvec, int64_t* n_env, int64_t* n_qr,
                          double* matvec_flops) {
  if (!h) return ATTN_ERR_ARG;
  if (n_matvec) *n_matvec = h->n_matvec;
  if (n_env) *n_env = h->n_env;
  if (n_qr) *n_qr = h->n_qr;
  if (matvec_flops) *matvec_flops = h->mv_flops;
  return ATTN_OK;
}

attn_status attn_profile(attn_handle* h, int32_t enable, int32_t min_dim, double* ms, double* flops,
                         int64_t* launches) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    HIPCHK(hipSetDevice(h->device));
    if (enable) {
      h->prof = true;
      h->ev_used = 0;
      h->prof_recs.clear();
      return ATTN_OK;
    }
    HIPCHK(hipDeviceSynchronize());
    double tms = 0, tfl = 0;
    int64_t nl = 0;
    for (auto& r : h->prof_recs) {
      if (std::min(r.ma, r.mb) < min_dim) continue;
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, h->ev_pool[r.a], h->ev_pool[r.b]));
      tms += e;
      tfl += r.flops;
      nl++;
    }
    if (ms) *ms = tms;
    if (flops) *flops = tfl;
    if (launches) *launches = nl;
    h->prof = false;
    h->ev_used = 0;
    h->prof_recs.clear();
    return ATTN_OK;
  });
}

attn_status attn_set_tensor(attn_handle* h, int32_t node, const double* host, int64_t len) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (node < 0 || node >= (int)h->M.tree.nodes.size() || !host) { h->err = "bad node or NULL"; return ATTN_ERR_ARG; }
    if (len != h->T_len[node]) { h->err = "length does not match the tensor size"; return ATTN_ERR_SHAPE; }
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpy(h->d_T + h->T_off[node], host, len * sizeof(double), hipMemcpyHostToDevice));
    invalidate_from(h, node);
    return ATTN_OK;
  });
}

attn_status attn_get_tensor(attn_handle* h, int32_t node, double* host, int64_t len) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (node < 0 || node >= (int)h->M.tree.nodes.size() || !host) { h->err = "bad node or NULL"; return ATTN_ERR_ARG; }
    if (len != h->T_len[node]) { h->err = "length does not match the tensor size"; return ATTN_ERR_SHAPE; }
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host, h->d_T + h->T_off[node], len * sizeof(double), hipMemcpyDeviceToHost));
    return ATTN_OK;
  });
}

attn_status attn_update_env(attn_handle* h, int32_t node, int32_t leg, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    const Tree& tr = h->M.tree;
    if (node < 0 || node >= (int)tr.nodes.size() || leg < 0 || leg > 2) { h->err = "bad node or leg"; return ATTN_ERR_ARG; }
    if (leg == 2 && node == tr.root) { h->err = "the root has no parent link"; return ATTN_ERR_ARG; }
    if (leg < 2 && tr.nodes[node].child[leg] < 0) { h->err = "leg leads to a site"; return ATTN_ERR_ARG; }
    if (h->iso[node] != leg) { h->err = "node is not isometric toward the leg"; return ATTN_ERR_STATE; }
    // inputs: the two other incoming stores
    for (int l2 = 0; l2 < 3; l2++) {
      if (l2 == leg) continue;
      if (l2 == 2) {
        if (node != tr.root && !h->valid[1][tr.edge_of_node(node)]) { h->err = "stale effective operator (parent link)"; return ATTN_ERR_STATE; }
      } else {
        const int e = tr.edge_of_child(node, l2);
        if (!tr.edge_is_site(e) && !h->valid[0][e]) { h->err = "stale effective operator (child link)"; return ATTN_ERR_STATE; }
      }
    }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    EnvDev& D = leg == 2 ? h->env_up[node] : h->env_down[leg][node];
    run_env(h, D, s);
    const int e = leg == 2 ? tr.edge_of_node(node) : tr.edge_of_child(node, leg);
    h->valid[leg == 2 ? 0 : 1][e] = 1;
    return ATTN_OK;
  });
}

attn_status attn_heff_apply(attn_handle* h, int32_t node, int32_t dtype, const void* x, void* y,
                            void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (node < 0 || node >= (int)h->M.tree.nodes.size() || !x || !y) { h->err = "bad node or NULL pointer"; return ATTN_ERR_ARG; }
    if (node != h->center) { h->err = "node is not the isometry centre"; return ATTN_ERR_STATE; }
    if (!incoming_valid(h, node)) { h->err = "stale effective operators at the node"; return ATTN_ERR_STATE; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    MVDev& D = h->mv[node];
    if (dtype == ATTN_F64) {
      run_comb(D.comb, s);
      matvec_f64(h, node, (const double*)x, (double*)y, s);
      return ATTN_OK;
    }
    if (dtype == ATTN_F32 || dtype == ATTN_BF16X2) {
      ensure_lowp(h, dtype);
      run_comb(D.comb, s);
      prepare_lowp(h, node, dtype, s);
      matvec_lowp(h, node, dtype, (const float*)x, y, 1, s);
      return ATTN_OK;
    }
    h->err = "unknown dtype";
    return ATTN_ERR_ARG;
  });
}

attn_status attn_isometrize(attn_handle* h, int32_t from, int32_t to, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    const Tree& tr = h->M.tree;
    if (from < 0 || to < 0 || from >= (int)tr.nodes.size() || to >= (int)tr.nodes.size()) { h->err = "bad node"; return ATTN_ERR_ARG; }
    const int leg = leg_toward(tr, from, to);
    if (leg < 0) { h->err = "nodes are not adjacent"; return ATTN_ERR_ARG; }
    if (from != h->center) { h->err = "from is not the isometry centre"; return ATTN_ERR_STATE; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    qr_node(h, from, leg, s);
    absorb(h, to, leg_toward(tr, to, from), s);
    h->iso[from] = leg;
    h->iso[to] = -1;
    h->center = to;
    invalidate_from(h, from);
    invalidate_from(h, to);
    return ATTN_OK;
  });
}

attn_status attn_eigsolve_node(attn_handle* h, int32_t node, const attn_solver_opts* opts,
                               double* theta, int32_t* n_matvec, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (node < 0 || node >= (int)h->M.tree.nodes.size()) { h->err = "bad node"; return ATTN_ERR_ARG; }
    if (node != h->center) { h->err = "node is not the isometry centre"; return ATTN_ERR_STATE; }
    if (!incoming_valid(h, node)) { h->err = "stale effective operators at the node"; return ATTN_ERR_STATE; }
    attn_solver_opts o;
    if (opts) o = *opts;
    else { std::memset(&o, 0, sizeof(o)); o.krylov_k = 20; }
    if (o.krylov_k < 1) { h->err = "krylov_k must be >= 1"; return ATTN_ERR_ARG; }
    if (o.solver != ATTN_SOLVER_LANCZOS && o.solver != ATTN_SOLVER_DAVIDSON) { h->err = "unknown solver"; return ATTN_ERR_ARG; }
    if (o.solver == ATTN_SOLVER_DAVIDSON && o.precond == ATTN_PRECOND_LEARNED && !h->mlp_ready) {
      h->err = "learned preconditioner requested before attn_precond_set_weights";
      return ATTN_ERR_STATE;
    }
    if (o.precision < ATTN_F64 || o.precision > ATTN_BF16X2) { h->err = "unknown precision"; return ATTN_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    int nmv = 0;
    const double th = o.solver == ATTN_SOLVER_DAVIDSON ? davidson(h, node, o, &nmv, s)
                                                       : lanczos(h, node, o.krylov_k, o.precision, &nmv, s);
    invalidate_from(h, node);
    if (theta) *theta = th;
    if (n_matvec) *n_matvec = nmv;
    return ATTN_OK;
  });
}

attn_status attn_init_state(attn_handle* h, const double* raw, int64_t len, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    const Tree& tr = h->M.tree;
    int64_t tot = 0;
    for (int64_t l : h->T_len) tot += l;
    if (!raw) { h->err = "raw is NULL"; return ATTN_ERR_ARG; }
    if (len != tot) { h->err = "raw length does not match the tree"; return ATTN_ERR_SHAPE; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipMemcpyAsync(h->d_T, raw, tot * sizeof(double), hipMemcpyHostToDevice, s));
    reset_state(h, 0, s);
    const int nn = (int)tr.nodes.size();
    for (int n = 0; n < nn; n++) {
      if (n == tr.root) continue;
      qr_node(h, n, 2, s);   // Q replaces the block, R is discarded
    }
    HIPCHK(launch_knorm(h->d_kjobs64 + tr.root, 1, s));
    HIPCHK(launch_kscale(h->d_kjobs64 + tr.root, 1, h->T_len[tr.root], 1, s));
    for (int n = 0; n < nn; n++) h->iso[n] = 2;
    h->iso[tr.root] = -1;
    h->center = tr.root;
    for (int e = tr.N; e < tr.n_edges(); e++) { h->valid[0][e] = 0; h->valid[1][e] = 0; }
    for (int n = 0; n < nn; n++) {
      if (n == tr.root) continue;
      run_env(h, h->env_up[n], s);
      h->valid[0][tr.edge_of_node(n)] = 1;
    }
    check_state(h, s, "attn_init_state");
    h->state_ready = true;
    return ATTN_OK;
  });
}

attn_status attn_precond_set_weights(attn_handle* h, const float* params, int64_t n) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (!params || n != kMlpParams) { h->err = "expected " + std::to_string(kMlpParams) + " parameters"; return ATTN_ERR_SHAPE; }
    HIPCHK(hipSetDevice(h->device));
    if (!h->d_mlp) h->d_mlp = dev_alloc(h, kMlpParams * 2);
    float* tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, kMlpParams * sizeof(float)));
    hipError_t e1 = hipMemcpy(tmp, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    hipError_t e2 = e1 == hipSuccess ? launch_to_half(tmp, h->d_mlp, kMlpParams, nullptr) : e1;
    hipError_t e3 = e2 == hipSuccess ? hipDeviceSynchronize() : e2;
    (void)hipFree(tmp);
    HIPCHK(e3);
    h->mlp_ready = true;
    return ATTN_OK;
  });
}

attn_status attn_solver_stats(const attn_handle* h, int64_t* dav_iters, int64_t* fallbacks, double* last_rnorm,
                              double* jacobi_rate) {
  if (!h) return ATTN_ERR_ARG;
  if (dav_iters) *dav_iters = h->n_dav_iter;
  if (fallbacks) *fallbacks = h->n_fallback;
  if (last_rnorm) *last_rnorm = h->last_rnorm;
  if (jacobi_rate) *jacobi_rate = h->jacobi_rate;
  return ATTN_OK;
}

attn_status attn_heff_diagonal(attn_handle* h, int32_t node, double* diag, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (node < 0 || node >= (int)h->M.tree.nodes.size() || !diag) { h->err = "bad node or NULL pointer"; return ATTN_ERR_ARG; }
    if (node != h->center) { h->err = "node is not the isometry centre"; return ATTN_ERR_STATE; }
    if (!incoming_valid(h, node)) { h->err = "stale effective operators at the node"; return ATTN_ERR_STATE; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    ensure_davidson(h);
    run_comb(h->mv[node].comb, s);
    HIPCHK(launch_heff_diag(h->mv[node].d_plan, h->d_djobs + node, h->T_len[node], s));
    HIPCHK(hipMemcpyAsync(diag, h->h_djobs[node].diag, h->T_len[node] * sizeof(double), hipMemcpyDeviceToDevice, s));
    return ATTN_OK;
  });
}

attn_status attn_precond_harvest(attn_handle* h, int32_t node, int32_t n_pairs, double cg_tol, int32_t cg_max,
                                 float* feats, float* targets, double* cg_res, void* stream) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    const Tree& tr = h->M.tree;
    if (node < 0 || node >= (int)tr.nodes.size() || n_pairs < 1 || !feats || !targets || cg_max < 1) {
      h->err = "bad arguments";
      return ATTN_ERR_ARG;
    }
    if (node != h->center) { h->err = "node is not the isometry centre"; return ATTN_ERR_STATE; }
    if (!incoming_valid(h, node)) { h->err = "stale effective operators at the node"; return ATTN_ERR_STATE; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->device));
    ensure_davidson(h);
    const int64_t M = h->T_len[node];
    const DJob* J = h->d_djobs + node;
    const DJob& Jh = h->h_djobs[node];
    // MINRES work vectors and partial sums
    double* vec[9];
    for (int i = 0; i < 9; i++) vec[i] = (double*)dev_alloc(h, M * 8);
    double* part = (double*)dev_alloc(h, kRedBlocks * 8);
    std::vector<double> hp(kRedBlocks);
    auto dot = [&](const double* a, const double* b) {
      HIPCHK(launch_vdot(a, b, M, part, s));
      HIPCHK(hipMemcpyAsync(hp.data(), part, kRedBlocks * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double acc = 0;
      for (double v : hp) acc += v;
      return acc;
    };
    MVDev& D = h->mv[node];
    run_comb(D.comb, s);
    // keep T_n: the Davidson iterations below only generate residuals
    double* Tsave = (double*)dev_alloc(h, M * 8);
    HIPCHK(hipMemcpyAsync(Tsave, Jh.T, M * 8, hipMemcpyDeviceToDevice, s));
    const double tol = 0.0;
    HIPCHK(launch_dav(0, J, 0, 0, tol, s));
    HIPCHK(launch_heff_diag(D.d_plan, J, M, s));
    HIPCHK(launch_dav(1, J, 0, 0, tol, s));
    HIPCHK(launch_dav(1, J, 0, 1, tol, s));
    int k = 1;
    DavState st;
    for (int pair = 0; pair < n_pairs; pair++) {
      matvec_f64(h, node, Jh.V + (int64_t)(k - 1) * M, Jh.W + (int64_t)(k - 1) * M, s);
      HIPCHK(launch_dav(2, J, k, 0, tol, s));
      HIPCHK(launch_dav(3, J, k, 0, tol, s));
      HIPCHK(launch_dav(4, J, k, 0, tol, s));
      HIPCHK(launch_dav(5, J, k, 0, tol, s));   // Jacobi correction (continues the iteration)
      HIPCHK(launch_dav(7, J, k, 0, tol, s));
      HIPCHK(hipMemcpyAsync(&st, h->d_dav, sizeof(st), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (st.status) throw StatusFail{ATTN_ERR_NUMERIC, "non-finite value while harvesting"};
      const double theta = st.theta;
      // u normalised in place
      const double un = std::sqrt(dot(Jh.u, Jh.u));
      HIPCHK(launch_axpby(0.0, Jh.u, 1.0 / un, Jh.u, M, s));
      // MINRES (C. C. Paige, M. A. Saunders, SIAM J. Numer. Anal. 12 (1975)) on the
      // symmetric, in general indefinite system (1 - u u^T)(H - theta)(1 - u u^T) x = -r
      // restricted to the complement of u (-r is orthogonal to u)
      double *x = vec[0], *r1 = vec[1], *r2 = vec[2], *y = vec[3], *v = vec[4], *wo = vec[5], *wn = vec[6];
      HIPCHK(launch_zero(x, M, s));
      HIPCHK(launch_zero(wo, M, s));
      HIPCHK(launch_zero(wn, M, s));
      HIPCHK(launch_axpby(-1.0, Jh.r, 0.0, r1, M, s));
      const double ur = dot(Jh.u, r1);
      HIPCHK(launch_axpby(-ur, Jh.u, 1.0, r1, M, s));
      HIPCHK(launch_axpby(1.0, r1, 0.0, r2, M, s));
      HIPCHK(launch_axpby(1.0, r1, 0.0, y, M, s));
      const double beta1 = std::sqrt(dot(r1, r1));
      double beta = beta1, oldb = 0, dbar = 0, epsln = 0, phibar = beta1, cs = -1, sn = 0;
      int it = 0;
      for (; it < cg_max && phibar > cg_tol * beta1 && beta > 0; it++) {
        HIPCHK(launch_axpby(1.0 / beta, y, 0.0, v, M, s));
        matvec_f64(h, node, v, y, s);
        HIPCHK(launch_axpby(-theta, v, 1.0, y, M, s));
        const double uy = dot(Jh.u, y);
        HIPCHK(launch_axpby(-uy, Jh.u, 1.0, y, M, s));
        if (it > 0) HIPCHK(launch_axpby(-beta / oldb, r1, 1.0, y, M, s));
        const double alfa = dot(v, y);
        HIPCHK(launch_axpby(-alfa / beta, r2, 1.0, y, M, s));
        std::swap(r1, r2);      // r1 <- r2
        std::swap(r2, y);       // r2 <- y (y now holds the free buffer)
        oldb = beta;
        beta = std::sqrt(dot(r2, r2));
        const double oldeps = epsln;
        const double delta = cs * dbar + sn * alfa;
        const double gbar = sn * dbar - cs * alfa;
        epsln = sn * beta;
        dbar = -cs * beta;
        const double gamma = std::max(std::sqrt(gbar * gbar + beta * beta), 1e-300);
        cs = gbar / gamma;
        sn = beta / gamma;
        const double phi = cs * phibar;
        phibar = sn * phibar;
        // w_new = (v - oldeps w_older - delta w_newer) / gamma, written over w_older
        HIPCHK(launch_axpby(-delta / gamma, wn, -oldeps / gamma, wo, M, s));
        HIPCHK(launch_axpby(1.0 / gamma, v, 1.0, wo, M, s));
        std::swap(wo, wn);
        HIPCHK(launch_axpby(phi, wn, 1.0, x, M, s));
        HIPCHK(launch_axpby(1.0, r2, 0.0, y, M, s));   // next Lanczos vector (unnormalised)
      }
      // true residual of the projected system
      matvec_f64(h, node, x, y, s);
      HIPCHK(launch_axpby(-theta, x, 1.0, y, M, s));
      const double ux = dot(Jh.u, y);
      HIPCHK(launch_axpby(-ux, Jh.u, 1.0, y, M, s));
      HIPCHK(launch_axpby(1.0, Jh.r, 1.0, y, M, s));
      const double ru = dot(Jh.u, Jh.r);
      HIPCHK(launch_axpby(-ru, Jh.u, 1.0, y, M, s));
      const double rr = dot(y, y);
      const double bn = beta1;
      if (cg_res) cg_res[pair] = std::sqrt(rr) / bn;
      HIPCHK(launch_harvest_write(Jh.diag, Jh.r, vec[0], theta, st.dinf, st.rinf, feats + (int64_t)pair * M * 3,
                                  targets + (int64_t)pair * M, M, s));
      // continue the Davidson iteration with the Jacobi correction
      HIPCHK(launch_dav(8, J, k, 5, tol, s));
      HIPCHK(launch_dav(9, J, k, 6, tol, s));
      if (k == kDavMax) {
        HIPCHK(launch_dav(11, J, k, 8, tol, s));
        HIPCHK(hipMemcpyAsync(Jh.V, Jh.Vt, (size_t)8 * M * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(Jh.W, Jh.Vt + 8 * M, (size_t)8 * M * 8, hipMemcpyDeviceToDevice, s));
        k = 8;
      }
      HIPCHK(launch_dav(10, J, k, k, tol, s));
      k++;
    }
    HIPCHK(hipMemcpyAsync(Jh.T, Tsave, M * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    // scratch of this call is released with the handle (dev_alloc); drop it now
    std::vector<void*> tmp(vec, vec + 9);
    tmp.push_back(part);
    tmp.push_back(Tsave);
    for (void* ptr : tmp) {
      auto it2 = std::find(h->owned.begin(), h->owned.end(), ptr);
      if (it2 != h->owned.end()) { h->owned.erase(it2); (void)hipFree(ptr); }
      for (size_t a = 0; a < h->allocs.size(); a++)
        if (h->allocs[a].first == (uintptr_t)ptr) { h->allocs.erase(h->allocs.begin() + a); break; }
    }
    return ATTN_OK;
  });
}

attn_status attn_mlp_train(const float* feats, const float* targets, int64_t n, int32_t steps, int32_t batch,
                           float lr, float* params, float* loss, void* stream) {
  if (!feats || !targets || !params || steps < 1 || batch < 64 || batch % 64 || n < batch) return ATTN_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *gpart = nullptr, *dl = nullptr;
  hipError_t e = prepare_kernel_attributes();
  auto al = [&](float** p, size_t cnt) { if (e == hipSuccess) e = hipMalloc(p, cnt * sizeof(float)); };
  al(&w, kMlpParams);
  al(&m, kMlpParams);
  al(&v, kMlpParams);
  al(&grad, kMlpParams + 1);
  al(&gpart, (size_t)(batch / 64) * (kMlpParams + 1));
  al(&dl, steps);
  if (e == hipSuccess) e = hipMemcpy(w, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m, 0, kMlpParams * sizeof(float));
  if (e == hipSuccess) e = hipMemset(v, 0, kMlpParams * sizeof(float));
  const int64_t nb = n / batch;
  for (int st = 1; st <= steps && e == hipSuccess; st++) {
    const int64_t off = ((st - 1) % nb) * batch;
    e = launch_mlp_train_step(w, feats, targets, off, batch, gpart, grad, m, v, st, lr, dl, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(params, w, kMlpParams * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && loss) e = hipMemcpy(loss, dl, steps * sizeof(float), hipMemcpyDeviceToHost);
  for (float* p : {w, m, v, grad, gpart, dl})
    if (p) (void)hipFree(p);
  return e == hipSuccess ? ATTN_OK : ATTN_ERR_HIP;
}

attn_status attn_mlp_eval(const float* params, const float* feats, float* out, int64_t n, void* stream) {
  if (!params || !feats || !out || n < 0) return ATTN_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  float* tmp = nullptr;
  void* w16 = nullptr;
  hipError_t e = hipMalloc(&tmp, kMlpParams * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&w16, kMlpParams * 2);
  if (e == hipSuccess) e = hipMemcpy(tmp, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_to_half(tmp, w16, kMlpParams, s);
  if (e == hipSuccess && n > 0) e = launch_mlp_eval(w16, feats, out, n, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (tmp) (void)hipFree(tmp);
  if (w16) (void)hipFree(w16);
  return e == hipSuccess ? ATTN_OK : ATTN_ERR_HIP;
}

attn_status attn_move_center(attn_handle* h, int32_t target, void* stream) {
  if (!h) return ATTN_ERR_ARG;
  const Tree& tr = h->M.tree;
  if (target < 0 || target >= (int)tr.nodes.size()) { h->err = "bad node"; return ATTN_ERR_ARG; }
  if (h->center < 0) { h->err = "no isometry centre (state not initialised)"; return ATTN_ERR_STATE; }
  int a = h->center, b = target;
  auto depth = [&](int x) { int dd = 0; while (tr.nodes[x].parent >= 0) { x = tr.nodes[x].parent; dd++; } return dd; };
  int da = depth(a), db = depth(b);
  std::vector<int> pa{a}, pb{b};
  while (da > db) { a = tr.nodes[a].parent; pa.push_back(a); da--; }
  while (db > da) { b = tr.nodes[b].parent; pb.push_back(b); db--; }
  while (a != b) { a = tr.nodes[a].parent; pa.push_back(a); b = tr.nodes[b].parent; pb.push_back(b); }
  pb.pop_back();
  std::vector<int> path = pa;
  for (int i = (int)pb.size() - 1; i >= 0; i--) path.push_back(pb[i]);
  for (size_t i = 0; i + 1 < path.size(); i++) {
    attn_status st = attn_isometrize(h, path[i], path[i + 1], stream);
    if (st) return st;
    st = attn_update_env(h, path[i], leg_toward(tr, path[i], path[i + 1]), stream);
    if (st) return st;
  }
  return ATTN_OK;
}

attn_status attn_sweep(attn_handle* h, int32_t n_sweeps, const attn_sweep_opts* opts,
                       double* energies, double* seconds) {
  if (!h) return ATTN_ERR_ARG;
  if (n_sweeps < 0) { h->err = "n_sweeps < 0"; return ATTN_ERR_ARG; }
  const Tree& tr = h->M.tree;
  attn_solver_opts so;
  if (opts) so = opts->solver;
  else { std::memset(&so, 0, sizeof(so)); so.krylov_k = 20; }
  // Lanczos sweeps check the per-node status on the device and read it (with
  // the last eigenvalue) once per sweep, so the host never waits inside a
  // sweep; the Davidson form steers its restarts from the host and keeps its
  // own synchronisation.
  const bool defer = so.solver == ATTN_SOLVER_LANCZOS && !h->dead && h->d_st;
  // with use_graphs, FP64 Lanczos sweeps run from HIP graphs on a stream of
  // the handle (not while the matvec launches are being timed)
  const bool graphs = defer && opts && opts->use_graphs && so.precision == ATTN_F64 && so.krylov_k >= 1 &&
                      !h->host_only && !h->dryrun;
  auto state = [&]() {
    attn_handle::SweepState st;
    st.center = h->center;
    st.iso = h->iso;
    st.valid0 = h->valid[0];
    st.valid1 = h->valid[1];
    return st;
  };
  double th = 0;   // energy of the sweep: the last node's eigenvalue
  auto node_loop = [&](void* stream) -> attn_status {
    for (int n = 0; n < (int)tr.nodes.size(); n++) {
      attn_status st = attn_move_center(h, n, stream);
      if (st == ATTN_OK) st = attn_eigsolve_node(h, n, &so, &th, nullptr, stream);
      if (st) return st;
    }
    return ATTN_OK;
  };
  for (int sw = 0; sw < n_sweeps; sw++) {
    auto t0 = std::chrono::steady_clock::now();
    th = 0;
    const bool use_graph = graphs && !h->prof;
    if (use_graph && !h->gstream) {
      if (hipSetDevice(h->device) != hipSuccess || hipStreamCreate(&h->gstream) != hipSuccess) {
        h->err = "stream creation failed";
        return ATTN_ERR_HIP;
      }
    }
    hipStream_t s = use_graph ? h->gstream : nullptr;
    if (defer) {
      if (hipSetDevice(h->device) != hipSuccess || launch_zero_int(&h->d_st->sticky, 1, s) != hipSuccess) {
        h->err = "status reset failed";
        return ATTN_ERR_HIP;
      }
      h->defer_status = true;
    }
    if (use_graph) {
      const attn_handle::SweepState pre = state();
      attn_handle::SweepGraph* G = nullptr;
      for (auto& g : h->sgraphs)
        if (g.krylov_k == so.krylov_k && g.pre == pre) G = &g;
      if (!G) {
        // capture this sweep's launches (nothing runs yet), then launch them
        attn_handle::SweepGraph ng;
        ng.krylov_k = so.krylov_k;
        ng.pre = pre;
        const int64_t m0 = h->n_matvec, e0 = h->n_env, q0 = h->n_qr;
        const double f0 = h->mv_flops;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          h->defer_status = false;
          h->err = "graph capture failed to start";
          return ATTN_ERR_HIP;
        }
        const attn_status st = node_loop((void*)s);
        const hipError_t ec = hipStreamEndCapture(s, &g);
        h->defer_status = false;
        if (st || ec != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          if (!st) { h->err = "graph capture failed"; h->dead = true; }
          return st ? st : ATTN_ERR_HIP;
        }
        const hipError_t ei = hipGraphInstantiate(&ng.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) { h->err = "graph instantiation failed"; h->dead = true; return ATTN_ERR_HIP; }
        ng.post = state();
        ng.d_matvec = h->n_matvec - m0; ng.d_env = h->n_env - e0; ng.d_qr = h->n_qr - q0;
        ng.d_flops = h->mv_flops - f0;
        if (h->sgraphs.size() >= 2) {
          (void)hipGraphExecDestroy(h->sgraphs.front().exec);
          h->sgraphs.erase(h->sgraphs.begin());
        }
        h->sgraphs.push_back(ng);
        G = &h->sgraphs.back();
        if (hipGraphLaunch(G->exec, s) != hipSuccess) { h->err = "graph launch failed"; h->dead = true; return ATTN_ERR_HIP; }
      } else {
        if (hipGraphLaunch(G->exec, s) != hipSuccess) { h->err = "graph launch failed"; h->dead = true; return ATTN_ERR_HIP; }
        // the host bookkeeping of the replayed sweep
        h->center = G->post.center;
        h->iso = G->post.iso;
        h->valid[0] = G->post.valid0;
        h->valid[1] = G->post.valid1;
        h->n_matvec += G->d_matvec; h->n_env += G->d_env; h->n_qr += G->d_qr;
        h->mv_flops += G->d_flops;
      }
    } else {
      const attn_status st = node_loop(nullptr);
      if (st) { h->defer_status = false; return st; }
    }
    h->defer_status = false;
    if ((s ? hipStreamSynchronize(s) : hipDeviceSynchronize()) != hipSuccess) {
      h->err = "device synchronisation failed";
      h->dead = true;
      return ATTN_ERR_HIP;
    }
    if (defer) {
      KrylovState st;
      if (hipMemcpy(&st, h->d_st, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) {
        h->err = "status read failed";
        h->dead = true;
        return ATTN_ERR_HIP;
      }
      if (st.sticky != 0) {
        h->err = (st.sticky & 2) ? "sweep: QR factorisation broke down" : "sweep: non-finite value in the eigensolver";
        h->dead = true;
        return ATTN_ERR_NUMERIC;
      }
      th = st.scal[0];
    }
    auto t1 = std::chrono::steady_clock::now();
    h->sweep_energies.push_back(th);
    if (energies) energies[sw] = th;
    if (seconds) seconds[sw] = std::chrono::duration<double>(t1 - t0).count();
  }
  return ATTN_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ work-list validation
// Checks, on the host, that every work unit of every device plan reads and
// writes only inside the buffers it was built for.
namespace {
struct Checker {
  const attn_handle* h;
  std::string err;
  bool ok = true;
  void fail(const std::string& m) { if (ok) err = m; ok = false; }
  // [p, p + bytes) inside one allocation
  void span(const void* p, int64_t bytes, const char* what) {
    if (!ok) return;
    if (!p) { fail(std::string(what) + ": null pointer"); return; }
    uintptr_t a = (uintptr_t)p;
    for (auto& al : h->allocs)
      if (a >= al.first && a + (uint64_t)bytes <= al.first + al.second) return;
    fail(std::string(what) + ": out of bounds");
  }
  void sw(const SWGroup& g, int64_t xbase_len, int esz) {
    for (const int4& wu : g.wus) {
      if (wu.x < 0 || wu.x >= (int)g.tasks.size()) { fail("sandwich: task index"); return; }
      const SWTask& t = g.tasks[wu.x];
      if (t.ma != g.ma || t.mb != g.mb) { fail("sandwich: group dims"); return; }
      const bool mf = sw_mfma(t.ma, t.mb);
      int64_t rows_hi;
      if (mf) {
        if (wu.z % 4 || wu.z * 16 >= t.ma) { fail("sandwich: strip"); return; }
        rows_hi = t.ma;   // the WG stages all rows of the slice
      } else {
        if (wu.z < 0 || wu.z >= t.ma * t.mb) { fail("sandwich: element"); return; }
        rows_hi = t.ma;
      }
      const int64_t xext = wu.y * t.xs_slice + (rows_hi - 1) * t.xs_row + t.mb;
      if (t.x) span(t.x, xext * esz, "sandwich x");
      else if (xext > xbase_len) fail("sandwich: x beyond the input vector");
      span(t.y, (wu.y * t.ys_slice + (t.ma - 1) * t.ys_row + t.mb) * esz, "sandwich y");
      std::vector<std::pair<int, int>> ranges;
      if (t.pad) {
        if (!mf) { fail("sandwich: several outputs on the generic kernel"); return; }
        if (t.item0 < 0 || t.item0 + t.nitem > (int)g.outs.size()) { fail("sandwich: output range"); return; }
        for (int o = t.item0; o < t.item0 + t.nitem; o++) {
          span(g.outs[o].y, (wu.y * t.ys_slice + (t.ma - 1) * t.ys_row + t.mb) * esz, "sandwich y (output)");
          ranges.push_back({g.outs[o].item0, g.outs[o].nitem});
        }
      } else {
        ranges.push_back({t.item0, t.nitem});
      }
      for (auto& rg : ranges) {
        if (rg.first < 0 || rg.first + rg.second > (int)g.items.size()) { fail("sandwich: item range"); return; }
        for (int i = rg.first; i < rg.first + rg.second; i++) {
          if (g.items[i].A) span(g.items[i].A, (int64_t)t.ma * t.ma * esz, "sandwich A");
          if (g.items[i].B) span(g.items[i].B, (int64_t)t.mb * t.mb * esz, "sandwich B");
        }
      }
      if (!ok) return;
    }
  }
  void mp(const MPGroup& g, int64_t xbase_len, int esz) {
    for (const int2& wu : g.wus) {
      if (wu.x < 0 || wu.x >= (int)g.tasks.size()) { fail("mode: task index"); return; }
      const MPTask& t = g.tasks[wu.x];
      const int mj = t.j == 0 ? t.d0 : (t.j == 1 ? t.d1 : t.d2);
      if (mj != g.mj) { fail("mode: group dims"); return; }
      const int64_t M = (int64_t)t.d0 * t.d1 * t.d2;
      if (g.mfma) { if ((int64_t)(wu.y + 1) * 64 * mj > M) { fail("mode: tile"); return; } }
      else if (wu.y < 0 || wu.y >= M) { fail("mode: element"); return; }
      span(t.out, M * esz, "mode out");
      if (t.job0 < 0 || t.job0 + t.njob > (int)g.jobs.size()) { fail("mode: job range"); return; }
      for (int k = t.job0; k < t.job0 + t.njob; k++) {
        span(g.jobs[k].A, (int64_t)mj * mj * esz, "mode A");
        if (g.jobs[k].in) span(g.jobs[k].in, M * esz, "mode in");
        else if (M > xbase_len) fail("mode: in beyond the input vector");
      }
      if (!ok) return;
    }
  }
  void gr(const std::vector<GRTask>& ts, bool mfma) {
    for (const GRTask& t : ts) {
      const int mj = t.j == 0 ? t.d0 : (t.j == 1 ? t.d1 : t.d2);
      const int64_t M = (int64_t)t.d0 * t.d1 * t.d2;
      if (t.f0 < 0 || t.f1 > M / mj || t.f0 >= t.f1) { fail("gram: f range"); return; }
      if (mfma && ((t.f1 - t.f0) % 64 || t.f0 % 64)) { fail("gram: f range not tiled"); return; }
      span(t.X, M * 8, "gram X");
      span(t.Z, M * 8, "gram Z");
      span(t.partial, (int64_t)mj * mj * 8, "gram partial");
    }
  }
  void red(const std::vector<GRReduce>& rs) {
    for (const GRReduce& r : rs) {
      span(r.partial, (int64_t)r.npart * r.m * r.m * 8, "reduce partial");
      span(r.out, (int64_t)r.m * r.m * 8, "reduce out");
    }
  }
  void cb(const CBPlan& P) {
    for (const CBTask& t : P.tasks) {
      span(t.out, (int64_t)t.n * 8, "combine out");
      for (int k = t.term0; k < t.term0 + t.nterm; k++) span(P.terms[k].in, (int64_t)t.n * 8, "combine in");
    }
  }
};
}  // namespace

extern "C" attn_status attn_validate(const attn_handle* h) {
  if (!h) return ATTN_ERR_ARG;
  if (h->host_only) return ATTN_ERR_STATE;
  Checker c{h, "", true};
  const Tree& tr = h->M.tree;
  for (int n = 0; n < (int)tr.nodes.size() && c.ok; n++) {
    const MVDev& D = h->mv[n];
    const int64_t M = (int64_t)D.dims[0] * D.dims[1] * D.dims[2];
    c.cb(D.comb);
    for (auto& g : D.sw) c.sw(g, M, 8);
    for (auto& g : D.chainA) c.mp(g, M, 8);
    for (auto& g : D.chainB) c.mp(g, M, 8);
    for (auto& g : D.chainC) c.mp(g, M, 8);
    for (auto& sr : D.srcs) c.span(sr.p, M * 8, "reduce source");
    {
      if (D.d_tiny && M > 1024) c.fail("tiny node too large");
      for (int sp = 0; sp < 3; sp++) {
        const int64_t ma = sp == 0 ? D.dims[1] : D.dims[0], mb = sp == 2 ? D.dims[1] : D.dims[2];
        for (int i = D.tiny_item0[sp]; i < D.tiny_item0[sp] + D.tiny_nitem[sp]; i++) {
          if (D.tiny_items[i].A) c.span(D.tiny_items[i].A, ma * ma * 8, "tiny A");
          if (D.tiny_items[i].B) c.span(D.tiny_items[i].B, mb * mb * 8, "tiny B");
        }
      }
      for (auto& q : D.tiny_items3)
        for (int l = 0; l < 3; l++) c.span(q.op[l], (int64_t)D.dims[l] * D.dims[l] * 8, "tiny op3");
      if (D.d_tiny) c.span(h->d_tmp2, M * M * 8, "dense H_eff");
    }
    if (D.need_xt) c.span(h->d_xt, M * 8, "transposed input");
    {
      const KJob& J = h->h_kjobs[n];
      if (J.n != M) c.fail("eigensolve job size");
      c.span(J.T, M * 8, "job tensor");
      c.span(J.V, (int64_t)h->kcap * M * 8, "job basis");
      c.span(J.w, M * 8, "job residual");
      c.span(h->d_x32, M * 4, "job FP32 copy");
      c.span(J.red, (int64_t)4 * 64 * kRedBlocks * 8, "job partial sums");
      c.span(J.st, sizeof(KrylovState), "job state");
      if (D.d_tiny) {
        const TJob& tj = h->h_tjobs[n];
        if (tj.M != M || tj.plan != D.d_tiny) c.fail("tiny job");
        c.span(tj.H, M * M * 8, "tiny H");
      }
    }
    const EnvDev* eds[3] = {&h->env_up[n], &h->env_down[0][n], &h->env_down[1][n]};
    for (const EnvDev* E : eds) {
      if (!E->present) continue;
      c.cb(E->comb);
      for (auto& ch : E->chunks) {
        for (auto& g : ch.sw) c.sw(g, 0, 8);
        c.gr(ch.gr.tasks, ch.gr.mfma);
        c.red(ch.gr.reds);
        for (auto& zb : ch.zero_blocks) c.span(zb.first, zb.second * 8, "zero block");
      }
    }
    for (int l = 0; l < 3; l++) {
      const QRDev& Q = h->qr[l][n];
      if (Q.present) {
        for (int pass = 0; pass < 3; pass++) {
          c.gr(Q.h_gt[pass], Q.gmf);
          c.mp(Q.h_mp[pass], 0, 8);
        }
        c.red(Q.h_gr);
        c.span(h->d_qrmat, qrmat_doubles(h->mmax) * 8, "qr matrices");
      }
      const ABDev& A = h->ab[l][n];
      if (A.present) c.mp(A.h_mp, 0, 8);
    }
  }
  // low-precision forms: a dry-run handle builds them here; a device handle
  // checks the ones it has built
  attn_handle* hm = const_cast<attn_handle*>(h);
  for (int dt = 1; dt <= 2 && c.ok; dt++) {
    if (h->dryrun) {
      try { ensure_lowp(hm, dt); } catch (const StatusFail& f) { c.fail(f.msg); break; }
    }
    if (!h->lowp_ready[dt - 1]) continue;
    for (int n = 0; n < (int)tr.nodes.size() && c.ok; n++) {
      const MVDev& D = h->mvlp[dt - 1][n];
      const int64_t M = (int64_t)D.dims[0] * D.dims[1] * D.dims[2];
      for (auto& g : D.sw) {
        c.sw(g, M, 4);
        if (g.fmt == 3 || g.fmt == 4)
          for (const int4& wu : g.wus) {
            const SWTask& t = g.tasks[wu.x];
            if (wu.w < 1 || wu.w > (g.fmt == 3 ? 4 : 2)) c.fail("several-slice unit: slice count");
            // the last slice of the unit, whole (ma x mb) slab
            const int64_t last = (int64_t)(wu.y + wu.w - 1);
            if (t.x) c.span(t.x, (last * t.xs_slice + (t.ma - 1) * t.xs_row + t.mb) * 4, "several-slice unit x");
            else if (last * t.xs_slice + (t.ma - 1) * t.xs_row + t.mb > M) c.fail("several-slice unit: x beyond the input");
            c.span(t.y, (last * t.ys_slice + (t.ma - 1) * t.ys_row + t.mb) * 4, "several-slice unit y");
            if (g.fmt == 4 && (t.ma != 64 || t.mb != 64 || t.pad)) c.fail("two-strip unit: legs or outputs");
          }
        if (g.fmt == 2 || g.fmt == 3) {
          if (!sw_bf16(g.ma, g.mb)) c.fail("split-BF16 group with legs not multiples of 32");
          for (auto& it : g.items)
            if ((uintptr_t)it.A % 16 || (uintptr_t)it.B % 16) c.fail("split-BF16 block not 16-byte aligned");
        }
      }
      for (auto& g : D.chainA) c.mp(g, M, 4);
      for (auto& g : D.chainB) c.mp(g, M, 4);
      for (auto& g : D.chainC) c.mp(g, M, 4);
      for (auto& sr : D.srcs) c.span(sr.p, M * 4, "reduce source");
      if (D.need_xt) c.span(h->d_xt, M * 4, "transposed input");
      const std::vector<CVTask> cv = lowp_conversions(hm, n, dt);
      if (cv.size() > (size_t)h->cv_cap) c.fail("conversion list too long");
      for (auto& t : cv) {
        c.span(t.src, t.n * 8, "conversion source");
        c.span(t.dst, t.n * 4, "conversion destination");
        if (t.fmt == 2 && (t.m % 32 || t.n % ((int64_t)t.m * t.m))) c.fail("split-BF16 conversion shape");
      }
    }
  }
  if (!c.ok) { const_cast<attn_handle*>(h)->err = c.err; return ATTN_ERR_STATE; }
  return ATTN_OK;
}
