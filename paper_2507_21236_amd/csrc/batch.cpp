// Batched form: many independent problem instances (each its own handle, of
// any size) swept in lock step.  Step t moves every instance's isometry centre
// to its node t (post-order) and solves that node; the eigensolver work of all
// instances in a step is merged into mixed-shape launches over one work list
// (or, in the persistent form, each matvec of the step into one launch over an
// ordered work list), and each step is captured once as a HIP graph and
// replayed in later sweeps.
#include "runtime.hpp"

struct attn_batch {
  std::vector<attn_handle*> hs;
  std::string err;
  int device = 0;
  int precision = ATTN_F32;
  int krylov_k = 20;
  bool use_graphs = true;
  int persistent = 0;         // 0 staged launches, 1 persistent launch, 2 per step the faster of the two
  bool dead = false;
  int n_cu = 0;
  int32_t* d_pm = nullptr;   // [0] abort word, then (one line further) the counters of the persistent matvec
  std::vector<void*> owned;
  std::vector<double*> x64;   // FP64 form: per-instance copy of the newest basis vector
  hipStream_t s[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> evs;
  // autotuned per leg shape (ma, mb): target workgroups per sandwich launch
  // group, and the tile of a wave (1: one 16-row strip; 2: two strips, FP32
  // legs 64 in the staged launches only, as a launch of its own)
  struct Tune {
    int ma, mb, target, tile;
  };
  std::vector<Tune> tuned;
  int default_target = (int)kMvTarget;   // the single-handle split

  struct Merged {
    std::vector<SWTask> sw_tasks;
    std::vector<SWItem> sw_items;
    std::vector<int4> sw_wus;
    size_t sw_lds = 0;
    std::vector<MPTask> mp_tasks[3];
    std::vector<MPJob> mp_jobs[3];
    std::vector<int2> mp_wus[3];
    size_t mp_lds[3] = {0, 0, 0};
    std::vector<TRTask> tr;
    int64_t tr_max = 0;
    std::vector<RDSrc> rd_srcs;
    std::vector<RDTask> rd;
    int64_t rd_max = 0;
    std::vector<int4> sw_wus2;   // two-strip units (task, first slice, 0, slices)
    int4* d_sw_wus2 = nullptr;
    // instance of every task (persistent form)
    std::vector<int> sw_inst, mp_inst[3], tr_inst, rd_inst;
    std::vector<PUnit> pu;
    std::vector<int32_t> tickets;
    int pm_grid = 0;
    size_t pm_lds = 0;
    PMArgs pm;
    bool use_pm = false;   // this step's matvec runs as the persistent launch
    // device copies
    SWTask* d_sw_tasks = nullptr;
    SWItem* d_sw_items = nullptr;
    int4* d_sw_wus = nullptr;
    MPTask* d_mp_tasks[3] = {nullptr, nullptr, nullptr};
    MPJob* d_mp_jobs[3] = {nullptr, nullptr, nullptr};
    int2* d_mp_wus[3] = {nullptr, nullptr, nullptr};
    TRTask* d_tr = nullptr;
    RDSrc* d_rd_srcs = nullptr;
    RDTask* d_rd = nullptr;
    PUnit* d_pu = nullptr;
    int32_t* d_tickets = nullptr;
  };

  struct Step {
    std::vector<std::vector<std::pair<int, int>>> moves;   // per instance: links (from, to)
    std::vector<CBTask> cb_tasks;
    std::vector<CBTerm> cb_terms;
    int cb_maxn = 0;
    std::vector<CVTask> cv;
    int64_t cv_max = 0;
    std::vector<TJob> tj;
    int tj_minM = 1 << 30, tj_maxM = 0;
    std::vector<KJob> kj;
    int64_t kj_max = 0;
    std::vector<int> kj_inst;   // instance of each eigensolve job
    Merged mv;
    double flops = 0;           // algorithmic matvec flops of one matvec of every instance
    CBTask* d_cb_tasks = nullptr;
    CBTerm* d_cb_terms = nullptr;
    CVTask* d_cv = nullptr;
    TJob* d_tj = nullptr;
    KJob* d_kj = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Step> steps;
};

namespace {

struct BatchFail {
  attn_status st;
  std::string msg;
};

void* balloc(attn_batch* b, size_t bytes) {
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, std::max<size_t>(bytes, 8)));
  b->owned.push_back(p);
  return p;
}

template <typename T>
T* bupload(attn_batch* b, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  T* p = (T*)balloc(b, v.size() * sizeof(T));
  HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

int target_for(const attn_batch* b, int ma, int mb) {
  for (auto& t : b->tuned)
    if (t.ma == ma && t.mb == mb) return t.target;
  return b->default_target;
}

int tile_for(const attn_batch* b, int ma, int mb) {
  for (auto& t : b->tuned)
    if (t.ma == ma && t.mb == mb) return t.tile;
  return 1;
}

// two-strip tiles apply to FP32 legs 64 x 64 in the staged launches
bool w2_allowed(const attn_batch* b, int ma, int mb) {
  return b->precision == ATTN_F32 && ma == 64 && mb == 64 && b->persistent == 0;
}

// Link-by-link centre path from a to c (up to the common ancestor, then down).
std::vector<int> tree_path(const Tree& tr, int a, int c) {
  auto depth = [&](int x) { int dd = 0; while (tr.nodes[x].parent >= 0) { x = tr.nodes[x].parent; dd++; } return dd; };
  int da = depth(a), dc = depth(c);
  std::vector<int> pa{a}, pc{c};
  while (da > dc) { a = tr.nodes[a].parent; pa.push_back(a); da--; }
  while (dc > da) { c = tr.nodes[c].parent; pc.push_back(c); dc--; }
  while (a != c) { a = tr.nodes[a].parent; pa.push_back(a); c = tr.nodes[c].parent; pc.push_back(c); }
  pc.pop_back();
  for (int i = (int)pc.size() - 1; i >= 0; i--) pa.push_back(pc[i]);
  return pa;
}

// Sandwich units of node n of handle h, appended to the merged list.  x is the
// instance's fixed input buffer; `shape` restricts to one (ma, mb) (autotuning).
void add_sandwich(attn_batch* b, attn_handle* h, int n, const void* x, attn_batch::Merged& m,
                  std::vector<RDSrc>& srcs, const std::pair<int, int>* shape, bool* fits) {
  const Model& M = h->M;
  const MatvecPlan& P = M.mv[n];
  const Node& nd = M.tree.nodes[n];
  const int dm[3] = {nd.dims[0], nd.dims[1], nd.dims[2]};
  const int64_t Msz = (int64_t)dm[0] * dm[1] * dm[2];
  const int fmt = b->precision == ATTN_F64 ? 0 : 1;
  const size_t esz = fmt ? 4 : 8;
  std::vector<int64_t> off;   // combined-block offsets of the node
  {
    int64_t tot = 0;
    for (const Combine& c : P.combines) { off.push_back(tot); tot += (int64_t)c.dim * c.dim; }
  }
  int64_t part_used = 0;
  int nchs[3];
  {
    int64_t target[3];
    for (int sp = 0; sp < 3; sp++) {
      int ma, mb, ns;
      int64_t sl, row;
      slice_geom(sp, dm, ma, mb, ns, sl, row);
      target[sp] = target_for(b, ma, mb);
    }
    mv_chunks(P, dm, target, nchs);
  }
  for (int sp = 0; sp < 3; sp++) {
    std::vector<const Item2*> its;
    for (const Item2& it : P.items)
      if (it.spect == sp) its.push_back(&it);
    if (its.empty()) continue;
    int ma, mb, ns;
    int64_t sl, row;
    slice_geom(sp, dm, ma, mb, ns, sl, row);
    if (shape && (shape->first != ma || shape->second != mb)) continue;
    const bool mf = sw_mfma(ma, mb) && mb <= 64;
    const int nch = nchs[sp];
    for (int ci = 0; ci < nch; ci++) {
      const size_t i0 = its.size() * ci / nch, i1 = its.size() * (ci + 1) / nch;
      if (i1 == i0) continue;
      if (part_used + Msz > h->part_cap) { *fits = false; return; }
      SWTask t;
      std::memset(&t, 0, sizeof(t));
      const bool trans = sp == 2 && dm[2] > 1;
      t.x = trans ? (const void*)h->d_xt : x;
      t.y = h->d_part + part_used;
      t.xs_slice = sl; t.xs_row = row; t.ys_slice = sl; t.ys_row = row;
      t.ma = ma; t.mb = mb;
      t.item0 = (int)m.sw_items.size();
      t.nitem = (int)(i1 - i0);
      for (size_t i = i0; i < i1; i++) {
        SWItem si;
        si.A = block_ptr(h, its[i]->A, h->d_mvcomb, off);
        si.B = block_ptr(h, its[i]->B, h->d_mvcomb, off);
        if (fmt) { si.A = to_mirror(h, si.A, 1); si.B = to_mirror(h, si.B, 1); }
        si.coef = its[i]->coef;
        m.sw_items.push_back(si);
      }
      const int ti = (int)m.sw_tasks.size();
      m.sw_tasks.push_back(t);
      if (mf && w2_allowed(b, ma, mb) && tile_for(b, ma, mb) == 2) {
        for (int s = 0; s < ns; s += 2) m.sw_wus2.push_back(make_int4(ti, s, 0, std::min(2, ns - s)));
      } else if (mf) {
        for (int s = 0; s < ns; s++)
          for (int st = 0; st < ma / 16; st += 4) m.sw_wus.push_back(make_int4(ti, s, st, mb / 16));
        m.sw_lds = std::max(m.sw_lds, (size_t)ma * (mb + 2) * esz);
      } else {
        for (int s = 0; s < ns; s++)
          for (int e = 0; e < ma * mb; e += 256) m.sw_wus.push_back(make_int4(ti, s, e, 0));
        m.sw_lds = std::max(m.sw_lds, gen_slice_lds(ma, mb, esz));
      }
      srcs.push_back({h->d_part + part_used, trans ? 1 : 0, 0});
      part_used += Msz;
    }
  }
}

// Chain (three-leg term) stages of node n, copied from the handle's plan with
// explicit input pointers; the chain outputs are appended to srcs.
void add_chains(attn_batch* b, attn_handle* h, int n, const void* x, attn_batch::Merged& m,
                std::vector<RDSrc>& srcs) {
  const MVDev& D = b->precision == ATTN_F64 ? h->mv[n] : h->mvlp[0][n];
  const size_t esz = b->precision == ATTN_F64 ? 8 : 4;
  const std::vector<MPGroup>* st[3] = {&D.chainA, &D.chainB, &D.chainC};
  for (int k = 0; k < 3; k++)
    for (const MPGroup& g : *st[k]) {
      const int t0 = (int)m.mp_tasks[k].size();
      const int j0 = (int)m.mp_jobs[k].size();
      const bool mf = g.mfma && g.mj <= 64;
      if (g.mfma && !mf) throw BatchFail{ATTN_ERR_UNSUPPORTED, "batched form: legs above 64"};
      for (MPTask t : g.tasks) {
        t.job0 += j0;
        t.pad = mf ? g.mj / 16 : 0;
        m.mp_tasks[k].push_back(t);
      }
      for (MPJob jb : g.jobs) {
        if (!jb.in) jb.in = x;
        m.mp_jobs[k].push_back(jb);
      }
      for (int2 wu : g.wus) m.mp_wus[k].push_back(make_int2(wu.x + t0, wu.y));
      if (mf) m.mp_lds[k] = std::max(m.mp_lds[k], (size_t)g.mj * 66 * esz);
    }
  const uintptr_t c0 = (uintptr_t)h->d_chain, c1 = c0 + (uintptr_t)h->chain_cap * 8;
  for (const RDSrc& r : D.srcs)
    if ((uintptr_t)r.p >= c0 && (uintptr_t)r.p < c1) srcs.push_back(r);
}

void upload_merged(attn_batch* b, attn_batch::Merged& m) {
  m.d_sw_tasks = bupload(b, m.sw_tasks);
  m.d_sw_items = bupload(b, m.sw_items);
  m.d_sw_wus = bupload(b, m.sw_wus);
  m.d_sw_wus2 = bupload(b, m.sw_wus2);
  for (int k = 0; k < 3; k++) {
    m.d_mp_tasks[k] = bupload(b, m.mp_tasks[k]);
    m.d_mp_jobs[k] = bupload(b, m.mp_jobs[k]);
    m.d_mp_wus[k] = bupload(b, m.mp_wus[k]);
  }
  m.d_tr = bupload(b, m.tr);
  m.d_rd_srcs = bupload(b, m.rd_srcs);
  for (RDTask& t : m.rd) t.srcs = m.d_rd_srcs + (size_t)(uintptr_t)t.srcs;   // offsets -> pointers
  m.d_rd = bupload(b, m.rd);
  m.d_pu = bupload(b, m.pu);
  m.d_tickets = bupload(b, m.tickets);
  std::memset(&m.pm, 0, sizeof(m.pm));
  m.pm.units = m.d_pu;
  m.pm.tickets = m.d_tickets;
  m.pm.n_tickets = m.tickets.empty() ? 0 : (int32_t)m.tickets.size() - 1;
  m.pm.n_units = (int32_t)m.pu.size();
  m.pm.n_cnt = kPmFirst + 4 * (int32_t)b->hs.size();
  m.pm.cnt = b->d_pm ? b->d_pm + kPmStride : nullptr;
  m.pm.abort = b->d_pm;
  m.pm.sw_tasks = m.d_sw_tasks;
  m.pm.sw_items = m.d_sw_items;
  for (int k = 0; k < 3; k++) {
    m.pm.mp_tasks[k] = m.d_mp_tasks[k];
    m.pm.mp_jobs[k] = m.d_mp_jobs[k];
  }
  m.pm.tr = m.d_tr;
  m.pm.rd = m.d_rd;
}

// Ordered work list of the persistent matvec.  Counters per instance i:
// kPmFirst + 4 i + {0: transposes, 1: chain stage 1, 2: chain stage 2,
// 3: partial and chain outputs}.  Order: transposes, chain stage 1, the first
// third of the sandwich tiles, stage 2, the second third, stage 3, the last
// third, reductions.  Every wait points at units earlier in the list, and the
// sandwich thirds give the chain stages independent work to overlap with, so
// the chain's three dependent stages do not end up behind all of the tiles.
void build_units(attn_batch* b, attn_batch::Merged& m) {
  const int ni = (int)b->hs.size();
  auto ctr = [](int i, int k) { return kPmFirst + 4 * i + k; };
  std::vector<int> n(4 * ni, 0);
  m.pu.clear();
  auto push = [&](int kind, int a, int bb, int c, int d, int wait, int sig) {
    PUnit u;
    u.kind = kind; u.a = a; u.b = bb; u.c = c; u.d = d;
    u.wait = wait;
    u.need = wait >= 0 ? n[wait - kPmFirst] : 0;
    u.signal = sig;
    m.pu.push_back(u);
    if (sig >= 0) n[sig - kPmFirst]++;
  };
  std::vector<char> has_tr(ni, 0);
  for (size_t r = 0; r < m.tr.size(); r++) {
    const int i = m.tr_inst[r];
    const int64_t M = (int64_t)m.tr[r].ml * m.tr[r].mr * m.tr[r].mp;
    for (int64_t e = 0; e < M; e += kPmTileT) push(PU_TRANSPOSE, (int)r, (int)e, 0, 0, -1, ctr(i, 0));
    has_tr[i] = 1;
  }
  for (const int2& wu : m.mp_wus[0]) push(PU_MODE, 0, wu.x, wu.y, 0, -1, ctr(m.mp_inst[0][wu.x], 1));
  const bool chains = !m.mp_wus[1].empty() || !m.mp_wus[2].empty();
  const size_t nsw = m.sw_wus.size();
  auto sandwiches = [&](size_t w0, size_t w1) {
    for (size_t w = w0; w < w1; w++) {
      const int4& wu = m.sw_wus[w];
      const int i = m.sw_inst[wu.x];
      const bool tr = m.sw_tasks[wu.x].x == (const void*)b->hs[i]->d_xt;
      if (tr && !has_tr[i]) throw BatchFail{ATTN_ERR_STATE, "internal: transposed input without its transpose"};
      push(PU_SANDWICH, wu.x, wu.y, wu.z, wu.w, tr ? ctr(i, 0) : -1, ctr(i, 3));
    }
  };
  sandwiches(0, chains ? nsw / 3 : nsw);
  for (const int2& wu : m.mp_wus[1]) {
    const int i = m.mp_inst[1][wu.x];
    push(PU_MODE, 1, wu.x, wu.y, 0, ctr(i, 1), ctr(i, 2));
  }
  if (chains) sandwiches(nsw / 3, 2 * nsw / 3);
  for (const int2& wu : m.mp_wus[2]) {
    const int i = m.mp_inst[2][wu.x];
    push(PU_MODE, 2, wu.x, wu.y, 0, ctr(i, 2), ctr(i, 3));
  }
  if (chains) sandwiches(2 * nsw / 3, nsw);
  for (size_t r = 0; r < m.rd.size(); r++) {
    const int i = m.rd_inst[r];
    const int64_t M = (int64_t)m.rd[r].ml * m.rd[r].mr * m.rd[r].mp;
    for (int64_t e = 0; e < M; e += kPmTileR) push(PU_REDUCE, (int)r, (int)e, 0, 0, ctr(i, 3), -1);
  }
  // counters nobody waits on are not signalled (each signal costs a release)
  std::vector<char> waited(4 * ni, 0);
  for (const PUnit& u : m.pu)
    if (u.wait >= 0) waited[u.wait - kPmFirst] = 1;
  for (PUnit& u : m.pu)
    if (u.signal >= 0 && !waited[u.signal - kPmFirst]) u.signal = -1;
  m.pm_lds = m.sw_lds;
  for (int k = 0; k < 3; k++) m.pm_lds = std::max(m.pm_lds, m.mp_lds[k]);
  if (m.pm_lds > (size_t)kPmMaxLds) throw BatchFail{ATTN_ERR_UNSUPPORTED, "persistent matvec: LDS above its limit"};
  int per_cu = 0;
  HIPCHK(batch_matvec_occupancy(b->precision == ATTN_F64 ? 0 : 1, m.pm_lds, &per_cu));
  if (per_cu < 1) throw BatchFail{ATTN_ERR_UNSUPPORTED, "persistent matvec does not fit a CU"};
  const int64_t slots = (int64_t)per_cu * b->n_cu;
  // tickets: runs of up to K consecutive units with the same kind, wait and
  // signal.  Chain-stage, transpose and reduction units go one per ticket:
  // the chain stages are on the dependency path, and the reductions end the
  // launch, so neither may pile up in one workgroup.  Sandwich tiles are many
  // and alike; they go in runs sized for about eight tickets per workgroup.
  const int64_t Ks = std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)nsw / (8 * slots)));
  m.tickets.clear();
  for (size_t u = 0; u < m.pu.size(); u++) {
    const PUnit& q = m.pu[u];
    const int64_t K = q.kind == PU_SANDWICH ? Ks : 1;
    const bool start = m.tickets.empty() || (int64_t)(u - m.tickets.back()) >= K ||
                       m.pu[m.tickets.back()].kind != q.kind || m.pu[m.tickets.back()].wait != q.wait ||
                       m.pu[m.tickets.back()].need != q.need || m.pu[m.tickets.back()].signal != q.signal;
    if (start) m.tickets.push_back((int32_t)u);
  }
  const int64_t nt = (int64_t)m.tickets.size();
  m.tickets.push_back((int32_t)m.pu.size());
  m.pm_grid = (int)std::max<int64_t>(kPmQueues, std::min<int64_t>(slots, nt));   // a workgroup per queue
}

void build_step(attn_batch* b, int t) {
  attn_batch::Step& S = b->steps[t];
  const int ni = (int)b->hs.size();
  S.moves.assign(ni, {});
  const int fmt = b->precision == ATTN_F64 ? 0 : 1;
  for (int i = 0; i < ni; i++) {
    attn_handle* h = b->hs[i];
    const Tree& tr = h->M.tree;
    const int nn = (int)tr.nodes.size();
    if (t >= nn) continue;
    const int n = t;
    const int prev = t == 0 ? tr.root : t - 1;
    const std::vector<int> path = tree_path(tr, prev, n);
    for (size_t k = 0; k + 1 < path.size(); k++) S.moves[i].push_back({path[k], path[k + 1]});
    const MVDev& D = h->mv[n];
    // combined blocks of the node (FP64)
    const int base = (int)S.cb_terms.size();
    for (CBTask c : D.comb.tasks) {
      c.term0 += base;
      S.cb_tasks.push_back(c);
      S.cb_maxn = std::max(S.cb_maxn, c.n);
    }
    for (const CBTerm& c : D.comb.terms) S.cb_terms.push_back(c);
    const int64_t Msz = h->T_len[n];
    S.flops += (double)h->M.mv[n].flops;
    if (D.d_tiny) {
      S.tj.push_back(h->h_tjobs[n]);
      S.tj_minM = std::min(S.tj_minM, (int)Msz);
      S.tj_maxM = std::max(S.tj_maxM, (int)Msz);
      continue;
    }
    if (fmt) {
      for (const CVTask& c : lowp_conversions(h, n, 1)) {
        S.cv.push_back(c);
        S.cv_max = std::max(S.cv_max, c.n);
      }
    }
    KJob J = h->h_kjobs[n];
    const void* x;
    if (fmt) { J.x32 = h->d_x32; x = h->d_x32; }
    else { J.x64 = b->x64[i]; x = b->x64[i]; }
    S.kj.push_back(J);
    S.kj_inst.push_back(i);
    S.kj_max = std::max(S.kj_max, Msz);
    // matvec work of the node
    std::vector<RDSrc> srcs;
    bool fits = true;
    add_sandwich(b, h, n, x, S.mv, srcs, nullptr, &fits);
    if (!fits) throw BatchFail{ATTN_ERR_STATE, "batched form: partial-output scratch too small"};
    add_chains(b, h, n, x, S.mv, srcs);
    if (D.need_xt) {
      S.mv.tr.push_back({x, h->d_xt, D.dims[0], D.dims[1], D.dims[2], 0});
      S.mv.tr_max = std::max(S.mv.tr_max, Msz);
    }
    S.mv.sw_inst.resize(S.mv.sw_tasks.size(), i);
    for (int k = 0; k < 3; k++) S.mv.mp_inst[k].resize(S.mv.mp_tasks[k].size(), i);
    S.mv.tr_inst.resize(S.mv.tr.size(), i);
    S.mv.rd_inst.push_back(i);
    RDTask rt;
    rt.srcs = (const RDSrc*)(uintptr_t)S.mv.rd_srcs.size();   // offset, made a pointer at upload
    rt.y = h->d_w;
    rt.nsrc = (int)srcs.size();
    rt.ml = D.dims[0]; rt.mr = D.dims[1]; rt.mp = D.dims[2];
    for (auto& r : srcs) S.mv.rd_srcs.push_back(r);
    S.mv.rd.push_back(rt);
    S.mv.rd_max = std::max(S.mv.rd_max, Msz);
  }
  S.d_cb_tasks = bupload(b, S.cb_tasks);
  S.d_cb_terms = bupload(b, S.cb_terms);
  S.d_cv = bupload(b, S.cv);
  S.d_tj = bupload(b, S.tj);
  S.d_kj = bupload(b, S.kj);
  if (b->persistent && !S.kj.empty()) {
    build_units(b, S.mv);
    S.mv.use_pm = true;
  }
  upload_merged(b, S.mv);
}

void run_matvec(attn_batch* b, attn_batch::Merged& m, hipStream_t s) {
  const int dt = b->precision == ATTN_F64 ? 0 : 1;
  if (m.use_pm) {
    HIPCHK(launch_batch_matvec(dt, m.pm, m.pm_grid, m.pm_lds, s));
    return;
  }
  HIPCHK(launch_transpose_list(dt, m.d_tr, (int)m.tr.size(), m.tr_max, s));
  for (int k = 0; k < 3; k++)
    HIPCHK(launch_batch_mode(dt, m.d_mp_tasks[k], m.d_mp_jobs[k], m.d_mp_wus[k], (int)m.mp_wus[k].size(),
                             m.mp_lds[k], s));
  HIPCHK(launch_batch_sandwich(dt, m.d_sw_tasks, m.d_sw_items, m.d_sw_wus, (int)m.sw_wus.size(), m.sw_lds, s));
  if (!m.sw_wus2.empty())
    HIPCHK(launch_sandwich(4, 64, 64, m.d_sw_tasks, m.d_sw_items, m.d_sw_wus2, (int)m.sw_wus2.size(), nullptr, s,
                           nullptr));
  HIPCHK(launch_reduce_list(dt, m.d_rd, (int)m.rd.size(), m.rd_max, s));
}

// Enqueue step t on stream s0; the centre moves of the instances are spread
// over the four streams and joined before the eigensolves.
void enqueue_step(attn_batch* b, int t, hipStream_t s0) {
  attn_batch::Step& S = b->steps[t];
  const int ni = (int)b->hs.size();
  HIPCHK(hipEventRecord(b->evs[0], s0));
  for (int q = 1; q < 4; q++) HIPCHK(hipStreamWaitEvent(b->s[q], b->evs[0], 0));
  for (int i = 0; i < ni; i++) {
    attn_handle* h = b->hs[i];
    const Tree& tr = h->M.tree;
    hipStream_t s = i % 4 == 0 ? s0 : b->s[i % 4];
    for (auto& mv : S.moves[i]) {
      const int from = mv.first, to = mv.second;
      const int leg = leg_toward(tr, from, to);
      qr_node(h, from, leg, s);
      absorb(h, to, leg_toward(tr, to, from), s);
      EnvDev& D = leg == 2 ? h->env_up[from] : h->env_down[leg][from];
      run_env(h, D, s);
    }
  }
  for (int q = 1; q < 4; q++) {
    HIPCHK(hipEventRecord(b->evs[q], b->s[q]));
    HIPCHK(hipStreamWaitEvent(s0, b->evs[q], 0));
  }
  if (!S.cb_tasks.empty())
    HIPCHK(launch_combine(S.d_cb_tasks, S.d_cb_terms, (int)S.cb_tasks.size(), S.cb_maxn, s0));
  if (!S.cv.empty()) HIPCHK(launch_convert(1, S.d_cv, (int)S.cv.size(), S.cv_max, s0));
  const int kk = std::min(b->krylov_k, 64);
  if (!S.tj.empty()) HIPCHK(launch_tiny(S.d_tj, (int)S.tj.size(), S.tj_minM, S.tj_maxM, kk, s0));
  if (S.kj.empty()) return;
  const int nj = (int)S.kj.size();
  const KJob* J = S.d_kj;
  HIPCHK(launch_kinit(J, nj, kk, s0));
  HIPCHK(launch_knorm(J, nj, s0));
  HIPCHK(launch_kscale(J, nj, S.kj_max, 0, s0));
  for (int j = 0; j < kk; j++) {
    run_matvec(b, S.mv, s0);
    if (j == kk - 1) {   // last step: only alpha_j
      HIPCHK(launch_kdots(J, nj, j, 1, 0, s0));
      HIPCHK(launch_kalpha(J, nj, j, s0));
      break;
    }
    HIPCHK(launch_kdots(J, nj, 0, j + 1, 1, s0));
    HIPCHK(launch_kortho(J, nj, j, 1, 0, 1, s0));
    HIPCHK(launch_kortho(J, nj, j, 2, 1, 0, s0));
    HIPCHK(launch_kbeta(J, nj, j, S.kj_max, s0));
  }
  HIPCHK(launch_ktridiag(J, nj, s0));
  HIPCHK(launch_kritz(J, nj, s0));
  HIPCHK(launch_kscale(J, nj, S.kj_max, 1, s0));
}

// Per step, time the step's matvec as staged launches and as the persistent
// launch (one warm-up, then three of each; the inputs are whatever the
// buffers hold, which does not change the time of the contractions) and keep
// the faster.  Both forms give the same results bit for bit.
void choose_forms(attn_batch* b) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipStream_t s = b->s[0];
  for (auto& S : b->steps) {
    if (S.kj.empty()) continue;
    float t[2] = {0, 0};
    for (int f = 0; f < 2; f++) {
      S.mv.use_pm = f == 1;
      run_matvec(b, S.mv, s);
      HIPCHK(hipEventRecord(e0, s));
      for (int r = 0; r < 3; r++) run_matvec(b, S.mv, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&t[f], e0, e1));
    }
    S.mv.use_pm = t[1] < t[0];
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
}

// Handles must sit in the state a sweep starts from (and ends in): centre at
// the root, every other node isometric toward its parent, upward effective
// operators current.
bool canonical(attn_handle* h) {
  const Tree& tr = h->M.tree;
  if (!h->state_ready || h->center != tr.root) return false;
  for (int n = 0; n < (int)tr.nodes.size(); n++) {
    if (n == tr.root) continue;
    if (h->iso[n] != 2 || !h->valid[0][tr.edge_of_node(n)]) return false;
  }
  return true;
}

// Time the merged sandwich launch of one leg shape over every step with each
// candidate work split and keep the fastest.
void autotune(attn_batch* b) {
  std::vector<std::pair<int, int>> shapes;
  for (attn_handle* h : b->hs) {
    const Tree& tr = h->M.tree;
    for (int n = 0; n < (int)tr.nodes.size(); n++) {
      if (h->mv[n].d_tiny) continue;
      const Node& nd = tr.nodes[n];
      for (const Item2& it : h->M.mv[n].items) {
        int ma, mb, ns;
        int64_t sl, row;
        slice_geom(it.spect, nd.dims, ma, mb, ns, sl, row);
        if (std::find(shapes.begin(), shapes.end(), std::make_pair(ma, mb)) == shapes.end())
          shapes.push_back({ma, mb});
      }
    }
  }
  const int cands[4] = {64, 256, (int)kMvTarget, 4096};   // the single-handle split among them
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int nsteps = (int)b->steps.size();
  for (auto& sh : shapes) {
    float best = 1e30f;
    int best_c = b->default_target, best_tile = 1;
    const int ntile = w2_allowed(b, sh.first, sh.second) ? 2 : 1;
    for (int tile = 1; tile <= ntile; tile++)
      for (int c : cands) {
        b->tuned.push_back({sh.first, sh.second, c, tile});
        std::vector<attn_batch::Merged> ms(nsteps);
        bool fits = true;
        for (int t = 0; t < nsteps && fits; t++) {
          for (int i = 0; i < (int)b->hs.size() && fits; i++) {
            attn_handle* h = b->hs[i];
            if (t >= (int)h->M.tree.nodes.size() || h->mv[t].d_tiny) continue;
            std::vector<RDSrc> srcs;
            const void* x = b->precision == ATTN_F64 ? (const void*)b->x64[i] : (const void*)h->d_x32;
            add_sandwich(b, h, t, x, ms[t], srcs, &sh, &fits);
          }
        }
        b->tuned.pop_back();
        if (!fits) continue;
        std::vector<void*> mark(b->owned);
        for (auto& m : ms) upload_merged(b, m);
        const int dt = b->precision == ATTN_F64 ? 0 : 1;
        float ms_tot = 0;
        for (int rep = 0; rep < 2; rep++) {   // first pass warms up
          HIPCHK(hipEventRecord(e0, b->s[0]));
          for (auto& m : ms) {
            HIPCHK(launch_batch_sandwich(dt, m.d_sw_tasks, m.d_sw_items, m.d_sw_wus, (int)m.sw_wus.size(),
                                         m.sw_lds, b->s[0]));
            if (!m.sw_wus2.empty())
              HIPCHK(launch_sandwich(4, 64, 64, m.d_sw_tasks, m.d_sw_items, m.d_sw_wus2, (int)m.sw_wus2.size(),
                                     nullptr, b->s[0], nullptr));
          }
          HIPCHK(hipEventRecord(e1, b->s[0]));
          HIPCHK(hipEventSynchronize(e1));
          HIPCHK(hipEventElapsedTime(&ms_tot, e0, e1));
        }
        // free the trial lists
        for (size_t k = mark.size(); k < b->owned.size(); k++) HIPCHK(hipFree(b->owned[k]));
        b->owned.resize(mark.size());
        if (ms_tot < best) { best = ms_tot; best_c = c; best_tile = tile; }
      }
    b->tuned.push_back({sh.first, sh.second, best_c, best_tile});
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
}

void destroy_batch(attn_batch* b) {
  for (auto& S : b->steps)
    if (S.exec) (void)hipGraphExecDestroy(S.exec);
  for (hipEvent_t e : b->evs) (void)hipEventDestroy(e);
  for (int q = 0; q < 4; q++)
    if (b->s[q]) (void)hipStreamDestroy(b->s[q]);
  for (void* p : b->owned) (void)hipFree(p);
  delete b;
}

thread_local std::string g_batch_error;

}  // namespace

extern "C" {

attn_status attn_batch_create(attn_handle* const* hs, int32_t n, const attn_batch_opts* opts,
                              attn_batch** out) {
  if (!out) return ATTN_ERR_ARG;
  *out = nullptr;
  if (!hs || n < 1) { g_batch_error = "need at least one handle"; return ATTN_ERR_ARG; }
  attn_batch_opts o;
  if (opts) o = *opts;
  else { std::memset(&o, 0, sizeof(o)); o.krylov_k = 20; o.precision = ATTN_F32; o.use_graphs = 1; }
  if (o.krylov_k < 1) { g_batch_error = "krylov_k must be >= 1"; return ATTN_ERR_ARG; }
  if (o.precision != ATTN_F64 && o.precision != ATTN_F32) {
    g_batch_error = "batched form runs FP64 or FP32 contractions";
    return ATTN_ERR_UNSUPPORTED;
  }
  for (int i = 0; i < n; i++) {
    attn_handle* h = hs[i];
    if (!h) { g_batch_error = "NULL handle"; return ATTN_ERR_ARG; }
    if (h->host_only || h->dryrun || h->dead) { g_batch_error = "handle cannot run on the device"; return ATTN_ERR_STATE; }
    if (h->device != hs[0]->device) { g_batch_error = "handles on different devices"; return ATTN_ERR_UNSUPPORTED; }
    if (h->M.tree.d != hs[0]->M.tree.d) { g_batch_error = "mixed local dimensions"; return ATTN_ERR_UNSUPPORTED; }
    if (h->mmax > 64) { g_batch_error = "batched form: bond dimensions above 64"; return ATTN_ERR_UNSUPPORTED; }
    for (int k = 0; k < i; k++)
      if (hs[k] == h) { g_batch_error = "a handle appears twice"; return ATTN_ERR_ARG; }
  }
  attn_batch* b = new attn_batch();
  b->hs.assign(hs, hs + n);
  b->device = hs[0]->device;
  b->precision = o.precision;
  b->krylov_k = o.krylov_k;
  b->use_graphs = o.use_graphs != 0;
  if (o.persistent < 0 || o.persistent > 2) {
    g_batch_error = "persistent must be 0, 1 or 2";
    delete b;
    return ATTN_ERR_ARG;
  }
  b->persistent = o.persistent;
  try {
    HIPCHK(hipSetDevice(b->device));
    HIPCHK(prepare_kernel_attributes());
    HIPCHK(hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device));
    if (b->persistent) {
      const size_t bytes = (size_t)(1 + kPmFirst + 4 * n) * kPmStride * sizeof(int32_t);
      b->d_pm = (int32_t*)balloc(b, bytes);
      HIPCHK(hipMemset(b->d_pm, 0, bytes));
    }
    for (int q = 0; q < 4; q++) HIPCHK(hipStreamCreate(&b->s[q]));
    b->evs.resize(4);
    for (auto& e : b->evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int maxn = 0;
    for (attn_handle* h : b->hs) {
      if (o.precision == ATTN_F32) ensure_lowp(h, 1);
      maxn = std::max(maxn, (int)h->M.tree.nodes.size());
      b->x64.push_back(o.precision == ATTN_F64 ? (double*)balloc(b, h->Mmax * sizeof(double)) : nullptr);
    }
    b->steps.resize(maxn);
    if (o.autotune) autotune(b);
    for (int t = 0; t < maxn; t++) build_step(b, t);
    if (b->persistent == 2) choose_forms(b);
    HIPCHK(hipDeviceSynchronize());
  } catch (const HipFail& e) {
    g_batch_error = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    destroy_batch(b);
    return ATTN_ERR_HIP;
  } catch (const BatchFail& e) {
    g_batch_error = e.msg;
    destroy_batch(b);
    return e.st;
  } catch (const StatusFail& e) {
    g_batch_error = e.msg;
    destroy_batch(b);
    return e.st;
  }
  *out = b;
  return ATTN_OK;
}

attn_status attn_batch_sweep(attn_batch* b, int32_t n_sweeps, double* energies, double* seconds) {
  if (!b) return ATTN_ERR_ARG;
  if (b->dead) { b->err = "batch unusable after an earlier HIP or numeric error"; return ATTN_ERR_STATE; }
  if (n_sweeps < 0) { b->err = "n_sweeps < 0"; return ATTN_ERR_ARG; }
  const int ni = (int)b->hs.size();
  for (int i = 0; i < ni; i++)
    if (!canonical(b->hs[i])) {
      b->err = "handle " + std::to_string(i) + " is not in the sweep start state (run attn_init_state or full sweeps)";
      return ATTN_ERR_STATE;
    }
  try {
    HIPCHK(hipSetDevice(b->device));
    hipStream_t s0 = b->s[0];
    for (int sw = 0; sw < n_sweeps; sw++) {
      HIPCHK(hipDeviceSynchronize());
      auto t0 = std::chrono::steady_clock::now();
      for (int t = 0; t < (int)b->steps.size(); t++) {
        attn_batch::Step& S = b->steps[t];
        if (!b->use_graphs) { enqueue_step(b, t, s0); continue; }
        if (!S.exec) {
          hipGraph_t g;
          HIPCHK(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
          try {
            enqueue_step(b, t, s0);
          } catch (...) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(s0, &dummy);
            throw;
          }
          HIPCHK(hipStreamEndCapture(s0, &g));
          HIPCHK(hipGraphInstantiate(&S.exec, g, nullptr, nullptr, 0));
          HIPCHK(hipGraphDestroy(g));
        }
        HIPCHK(hipGraphLaunch(S.exec, s0));
      }
      HIPCHK(hipStreamSynchronize(s0));
      auto t1 = std::chrono::steady_clock::now();
      if (b->persistent) {
        int32_t ab = 0;
        HIPCHK(hipMemcpy(&ab, b->d_pm, sizeof(ab), hipMemcpyDeviceToHost));
        if (ab) {
          b->dead = true;
          b->err = "persistent matvec: a wait for earlier units exceeded its limit";
          return ATTN_ERR_HIP;
        }
      }
      for (int i = 0; i < ni; i++) {
        attn_handle* h = b->hs[i];
        KrylovState st;
        HIPCHK(hipMemcpy(&st, h->d_st, sizeof(st), hipMemcpyDeviceToHost));
        if (st.status != 0 || !std::isfinite(st.scal[0])) {
          b->dead = true;
          b->err = "non-finite value or factorisation breakdown in instance " + std::to_string(i);
          return ATTN_ERR_NUMERIC;
        }
        if (energies) energies[(int64_t)i * n_sweeps + sw] = st.scal[0];
        // host bookkeeping: the sweep ends where it started; counters
        const Tree& tr = h->M.tree;
        for (int e = tr.N; e < tr.n_edges(); e++) h->valid[1][e] = 0;
        for (int nd = 0; nd < (int)tr.nodes.size(); nd++) {
          h->n_matvec += std::min<int64_t>(std::min(b->krylov_k, 64), h->T_len[nd]);
          h->mv_flops += (double)std::min<int64_t>(std::min(b->krylov_k, 64), h->T_len[nd]) * h->M.mv[nd].flops;
        }
      }
      for (auto& S : b->steps)
        for (int i = 0; i < ni; i++) {
          b->hs[i]->n_qr += (int64_t)S.moves[i].size();
          b->hs[i]->n_env += (int64_t)S.moves[i].size();
        }
      if (seconds) seconds[sw] = std::chrono::duration<double>(t1 - t0).count();
    }
  } catch (const HipFail& e) {
    b->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    b->dead = true;
    return ATTN_ERR_HIP;
  } catch (const BatchFail& e) {
    b->err = e.msg;
    return e.st;
  } catch (const StatusFail& e) {
    b->err = e.msg;
    return e.st;
  }
  return ATTN_OK;
}

attn_status attn_batch_info(const attn_batch* b, int32_t* n_steps, int64_t* n_launch_units,
                            int32_t* n_tuned, int32_t* tuned /* [n][4] = ma, mb, target, rows per wave */,
                            int32_t cap) {
  if (!b) return ATTN_ERR_ARG;
  if (n_steps) *n_steps = (int32_t)b->steps.size();
  if (n_launch_units) {
    int64_t u = 0;
    for (auto& S : b->steps) u += (int64_t)(S.mv.sw_wus.size() + S.mv.sw_wus2.size());
    *n_launch_units = u;
  }
  if (n_tuned) *n_tuned = (int32_t)b->tuned.size();
  if (tuned)
    for (int k = 0; k < (int)b->tuned.size() && k < cap; k++) {
      tuned[4 * k] = b->tuned[k].ma;
      tuned[4 * k + 1] = b->tuned[k].mb;
      tuned[4 * k + 2] = b->tuned[k].target;
      tuned[4 * k + 3] = 16 * b->tuned[k].tile;
    }
  return ATTN_OK;
}

attn_status attn_batch_forms(const attn_batch* b, int32_t* n_matvec_steps, int32_t* n_persistent_steps) {
  if (!b) return ATTN_ERR_ARG;
  int32_t nm = 0, np = 0;
  for (auto& S : b->steps) {
    if (S.kj.empty()) continue;
    nm++;
    np += S.mv.use_pm ? 1 : 0;
  }
  if (n_matvec_steps) *n_matvec_steps = nm;
  if (n_persistent_steps) *n_persistent_steps = np;
  return ATTN_OK;
}

const char* attn_batch_last_error(const attn_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}

attn_status attn_batch_destroy(attn_batch* b) {
  if (!b) return ATTN_ERR_ARG;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  destroy_batch(b);
  return ATTN_OK;
}

}  // extern "C"
