// State persistence of a handle: the problem copy and its hash, rebuilding the
// effective operators toward the centre, and checkpoint / restore files.
#include <cstdio>

#include "runtime.hpp"

using namespace attn;
using namespace rt;

// ------------------------------------------------------------------ problem copy
void ProblemCopy::assign(const attn_problem* p) {
  n_sites = p->n_sites;
  d = p->d;
  m = p->m;
  flags = p->flags;
  device = p->device;
  leaf_order.assign(p->leaf_order, p->leaf_order + p->n_sites);
  term_nsites.assign(p->term_nsites, p->term_nsites + p->n_terms);
  int64_t ns = 0;
  for (int t = 0; t < p->n_terms; t++) ns += p->term_nsites[t];
  term_sites.assign(p->term_sites, p->term_sites + ns);
  term_ops.assign(p->term_ops, p->term_ops + ns * p->d * p->d);
  term_coef.assign(p->term_coef, p->term_coef + p->n_terms);
  de_sites.assign(p->de_sites, p->de_sites + 2 * (int64_t)p->n_de);
  const int64_t d4 = (int64_t)p->d * p->d * p->d * p->d;
  de_u.assign(p->de_u, p->de_u + d4 * p->n_de);
}

attn_problem ProblemCopy::view() const {
  attn_problem p;
  std::memset(&p, 0, sizeof(p));
  p.n_sites = n_sites;
  p.d = d;
  p.m = m;
  p.leaf_order = leaf_order.data();
  p.n_terms = (int32_t)term_nsites.size();
  p.term_nsites = term_nsites.data();
  p.term_sites = term_sites.data();
  p.term_ops = term_ops.data();
  p.term_coef = term_coef.data();
  p.n_de = (int32_t)(de_sites.size() / 2);
  p.de_sites = de_sites.data();
  p.de_u = de_u.data();
  p.flags = flags;
  p.device = device;
  return p;
}

namespace {
struct Fnv {
  uint64_t v = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) {
      v ^= c[i];
      v *= 1099511628211ull;
    }
  }
  template <typename T>
  void pod(const T& x) { bytes(&x, sizeof(T)); }
  template <typename T>
  void vec(const std::vector<T>& x) {
    pod((uint64_t)x.size());
    if (!x.empty()) bytes(x.data(), x.size() * sizeof(T));
  }
};
}  // namespace

uint64_t ProblemCopy::hash() const {
  Fnv f;
  f.pod(n_sites);
  f.pod(d);
  f.pod(m);
  f.vec(leaf_order);
  f.vec(term_nsites);
  f.vec(term_sites);
  f.vec(term_ops);
  f.vec(term_coef);
  f.vec(de_sites);
  f.pod((uint32_t)(flags & ATTN_DE_STRICT));
  return f.v;
}

// ------------------------------------------------------------------ effective operators toward the centre
namespace rt {
void rebuild_envs(attn_handle* h, hipStream_t s) {
  const Tree& tr = h->M.tree;
  const int nn = (int)tr.nodes.size();
  const int c = h->center;
  for (int e = tr.N; e < tr.n_edges(); e++) { h->valid[0][e] = 0; h->valid[1][e] = 0; }
  std::vector<char> on_path(nn, 0);
  std::vector<int> path;   // centre up to the root
  for (int x = c; x >= 0; x = tr.nodes[x].parent) { on_path[x] = 1; path.push_back(x); }
  // stores from below on every link whose subtree does not hold the centre
  // (node ids are a post-order: children come before their parent)
  for (int n = 0; n < nn; n++) {
    if (on_path[n]) continue;
    run_env(h, h->env_up[n], s);
    h->valid[0][tr.edge_of_node(n)] = 1;
  }
  // stores from above down the path, from the root to the centre
  for (int i = (int)path.size() - 1; i >= 1; i--) {
    const int q = path[i], x = path[i - 1];
    const int side = tr.nodes[x].side;
    run_env(h, h->env_down[side][q], s);
    h->valid[1][tr.edge_of_node(x)] = 1;
  }
}
}  // namespace rt

// ------------------------------------------------------------------ checkpoint files
//
// Layout (host byte order, checked by a marker):
//   char[8] "ATTNCKPT", uint32 version (1), uint32 0x01020304,
//   uint64 problem hash, int32 n_sites, d, m, n_nodes,
//   int32 n_de, double de_u[n_de * d^4],
//   int32 centre, int32 iso[n_nodes],
//   int64 n_sweeps, double energies[n_sweeps],
//   int64 n_values, double tensors[n_values] (T_0, T_1, ... in node order),
//   uint64 FNV-1a of every byte before it.
namespace {
const char kMagic[8] = {'A', 'T', 'T', 'N', 'C', 'K', 'P', 'T'};
const uint32_t kVersion = 1, kOrder = 0x01020304u;

struct Writer {
  FILE* f = nullptr;
  Fnv sum;
  bool ok = true;
  void put(const void* p, size_t n) {
    if (!ok || n == 0) return;
    if (fwrite(p, 1, n, f) != n) ok = false;
    sum.bytes(p, n);
  }
  template <typename T>
  void pod(const T& x) { put(&x, sizeof(T)); }
};

struct Reader {
  std::vector<unsigned char> buf;
  size_t pos = 0;
  bool ok = true;
  void get(void* p, size_t n) {
    if (!ok) return;
    if (pos + n > buf.size()) { ok = false; return; }
    std::memcpy(p, buf.data() + pos, n);
    pos += n;
  }
  template <typename T>
  T pod() { T x{}; get(&x, sizeof(T)); return x; }
};

struct Ckpt {
  uint64_t hash = 0;
  int32_t n_sites = 0, d = 0, m = 0, n_nodes = 0, n_de = 0, center = -1;
  std::vector<double> de_u, energies, T;
  std::vector<int32_t> iso;
};

// Reads and checks a checkpoint file; returns ATTN_OK or ATTN_ERR_IO with a message.
attn_status read_ckpt(const char* path, Ckpt& c, std::string& err) {
  FILE* f = fopen(path, "rb");
  if (!f) { err = std::string("cannot open ") + path; return ATTN_ERR_IO; }
  Reader r;
  unsigned char tmp[1 << 16];
  size_t n;
  while ((n = fread(tmp, 1, sizeof(tmp), f)) > 0) r.buf.insert(r.buf.end(), tmp, tmp + n);
  const bool rerr = ferror(f) != 0;
  fclose(f);
  if (rerr) { err = "read error"; return ATTN_ERR_IO; }
  if (r.buf.size() < 8 + 8) { err = "file too short for a checkpoint"; return ATTN_ERR_IO; }
  Fnv sum;
  sum.bytes(r.buf.data(), r.buf.size() - 8);
  uint64_t stored;
  std::memcpy(&stored, r.buf.data() + r.buf.size() - 8, 8);
  char magic[8];
  r.get(magic, 8);
  if (std::memcmp(magic, kMagic, 8) != 0) { err = "not a checkpoint file"; return ATTN_ERR_IO; }
  if (stored != sum.v) { err = "checksum mismatch (truncated or corrupt file)"; return ATTN_ERR_IO; }
  const uint32_t ver = r.pod<uint32_t>(), order = r.pod<uint32_t>();
  if (ver != kVersion || order != kOrder) { err = "unsupported checkpoint version or byte order"; return ATTN_ERR_IO; }
  c.hash = r.pod<uint64_t>();
  c.n_sites = r.pod<int32_t>();
  c.d = r.pod<int32_t>();
  c.m = r.pod<int32_t>();
  c.n_nodes = r.pod<int32_t>();
  c.n_de = r.pod<int32_t>();
  const int64_t d4 = (int64_t)c.d * c.d * c.d * c.d;
  if (!r.ok || c.n_nodes < 1 || c.n_de < 0 || c.d < 2 || d4 * c.n_de > (int64_t)r.buf.size()) {
    err = "malformed checkpoint header";
    return ATTN_ERR_IO;
  }
  c.de_u.resize(d4 * c.n_de);
  r.get(c.de_u.data(), c.de_u.size() * sizeof(double));
  c.center = r.pod<int32_t>();
  c.iso.resize(c.n_nodes);
  r.get(c.iso.data(), c.iso.size() * sizeof(int32_t));
  const int64_t ns = r.pod<int64_t>();
  if (!r.ok || ns < 0 || ns * 8 > (int64_t)r.buf.size()) { err = "malformed sweep record"; return ATTN_ERR_IO; }
  c.energies.resize(ns);
  r.get(c.energies.data(), ns * sizeof(double));
  const int64_t nv = r.pod<int64_t>();
  if (!r.ok || nv < 0 || nv * 8 > (int64_t)r.buf.size()) { err = "malformed tensor record"; return ATTN_ERR_IO; }
  c.T.resize(nv);
  r.get(c.T.data(), nv * sizeof(double));
  if (!r.ok || r.pos + 8 != r.buf.size()) { err = "malformed checkpoint body"; return ATTN_ERR_IO; }
  return ATTN_OK;
}

// Isometry direction of node n when the centre is c: the leg toward the next
// node on the tree path from n to c (-1 at the centre).
int iso_toward(const Tree& tr, int n, int c) {
  if (n == c) return -1;
  const Node& nd = tr.nodes[n];
  const Node& cn = tr.nodes[c];
  const bool c_below = cn.lo >= nd.lo && cn.hi <= nd.hi;
  if (!c_below) return 2;
  const int l = nd.child[0];
  if (l >= 0) {
    const Node& ln = tr.nodes[l];
    if (cn.lo >= ln.lo && cn.hi <= ln.hi) return 0;
  }
  return 1;
}
}  // namespace

extern "C" {

attn_status attn_problem_hash(const attn_handle* h, uint64_t* hash) {
  if (!h || !hash) return ATTN_ERR_ARG;
  *hash = h->problem_hash;
  return ATTN_OK;
}

attn_status attn_sweep_history(const attn_handle* h, int64_t* n_sweeps, double* energies, int64_t cap) {
  if (!h) return ATTN_ERR_ARG;
  if (n_sweeps) *n_sweeps = (int64_t)h->sweep_energies.size();
  if (energies)
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)h->sweep_energies.size()); i++)
      energies[i] = h->sweep_energies[i];
  return ATTN_OK;
}

attn_status attn_checkpoint_info(const char* path, uint64_t* hash, int32_t* n_nodes, int32_t* center,
                                 int64_t* n_sweeps) {
  if (!path) return ATTN_ERR_ARG;
  Ckpt c;
  std::string err;
  if (attn_status st = read_ckpt(path, c, err)) return st;
  if (hash) *hash = c.hash;
  if (n_nodes) *n_nodes = c.n_nodes;
  if (center) *center = c.center;
  if (n_sweeps) *n_sweeps = (int64_t)c.energies.size();
  return ATTN_OK;
}

attn_status attn_checkpoint(attn_handle* h, const char* path) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (!path) { h->err = "path is NULL"; return ATTN_ERR_ARG; }
    if (!h->state_ready) { h->err = "no state to save (attn_init_state not called)"; return ATTN_ERR_STATE; }
    const Tree& tr = h->M.tree;
    const int nn = (int)tr.nodes.size();
    int64_t tot = 0;
    for (int64_t l : h->T_len) tot += l;
    std::vector<double> T(tot);
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(T.data(), h->d_T, tot * sizeof(double), hipMemcpyDeviceToHost));
    const std::string tmp = std::string(path) + ".tmp";
    Writer w;
    w.f = fopen(tmp.c_str(), "wb");
    if (!w.f) { h->err = "cannot create " + tmp; return ATTN_ERR_IO; }
    w.put(kMagic, 8);
    w.pod(kVersion);
    w.pod(kOrder);
    w.pod(h->problem_hash);
    w.pod((int32_t)tr.N);
    w.pod((int32_t)tr.d);
    w.pod((int32_t)tr.m);
    w.pod((int32_t)nn);
    w.pod((int32_t)(h->prob.de_sites.size() / 2));
    w.put(h->prob.de_u.data(), h->prob.de_u.size() * sizeof(double));
    w.pod((int32_t)h->center);
    for (int n = 0; n < nn; n++) w.pod((int32_t)h->iso[n]);
    w.pod((int64_t)h->sweep_energies.size());
    w.put(h->sweep_energies.data(), h->sweep_energies.size() * sizeof(double));
    w.pod(tot);
    w.put(T.data(), T.size() * sizeof(double));
    const uint64_t sum = w.sum.v;
    if (w.ok && fwrite(&sum, 1, 8, w.f) != 8) w.ok = false;
    if (fclose(w.f) != 0) w.ok = false;
    if (!w.ok) { std::remove(tmp.c_str()); h->err = "write error on " + tmp; return ATTN_ERR_IO; }
    if (std::rename(tmp.c_str(), path) != 0) { std::remove(tmp.c_str()); h->err = std::string("cannot rename to ") + path; return ATTN_ERR_IO; }
    return ATTN_OK;
  });
}

attn_status attn_restore(attn_handle* h, const char* path) {
  return guard(h, [&]() -> attn_status {
    if (attn_status e = need_device(h)) return e;
    if (!path) { h->err = "path is NULL"; return ATTN_ERR_ARG; }
    Ckpt c;
    std::string err;
    if (attn_status st = read_ckpt(path, c, err)) { h->err = err; return st; }
    const Tree& tr = h->M.tree;
    const int nn = (int)tr.nodes.size();
    if (c.hash != h->problem_hash || c.n_nodes != nn || c.n_sites != tr.N || c.d != tr.d || c.m != tr.m) {
      h->err = "checkpoint belongs to another problem";
      return ATTN_ERR_MISMATCH;
    }
    if (c.de_u != h->prob.de_u) {
      h->err = "checkpoint holds other disentanglers than the handle";
      return ATTN_ERR_MISMATCH;
    }
    int64_t tot = 0;
    for (int64_t l : h->T_len) tot += l;
    if ((int64_t)c.T.size() != tot) { h->err = "tensor record does not match the tree"; return ATTN_ERR_IO; }
    if (c.center < 0 || c.center >= nn) { h->err = "centre out of range"; return ATTN_ERR_IO; }
    for (int n = 0; n < nn; n++)
      if (c.iso[n] != iso_toward(tr, n, c.center)) { h->err = "isometry directions do not point to the centre"; return ATTN_ERR_IO; }
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = nullptr;
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(h->d_T, c.T.data(), tot * sizeof(double), hipMemcpyHostToDevice));
    reset_state(h, 0, s);
    for (int n = 0; n < nn; n++) h->iso[n] = c.iso[n];
    h->center = c.center;
    rebuild_envs(h, s);
    check_state(h, s, "attn_restore");
    h->sweep_energies = c.energies;
    h->state_ready = true;
    return ATTN_OK;
  });
}

}  // extern "C"
