// C ABI, graph loader, per-GFD planner and launch driver.
//
// Path per GFD (FastGFDs paper, Section IV-B, on one GPU):
//   plan (host, microseconds): 2-core of the pattern skeleton, root, BFS
//     spanning tree, core-first matching order, per-step probes;
//   CPI build (device): label/degree candidate filter, one top-down and one
//     bottom-up marking pass, CPI adjacency lists per spanning-tree edge;
//   enumeration (device): level-synchronous extension over the CPI, the
//     X -> Y check fused into the last level, first-K selection.
// All launches of a call are queued without host round trips; one
// synchronisation per call reads the status words.  A GFD whose frontier or
// violation staging overflowed its share of the budget is re-run on the
// chunked path, which bounds every level by the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "gfd.h"
#include "gfd_internal.h"

using namespace gfd;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

static int32_t set_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

struct GfdError {
  int32_t code;
  std::string msg;
};

#define HIPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (void)hipGetLastError();                                                          \
      throw GfdError{e_ == hipErrorOutOfMemory ? GFD_ENOMEM : GFD_EDEVICE,              \
                     std::string(#call) + ": " + hipGetErrorString(e_)};                 \
    }                                                                                   \
  } while (0)

template <class T>
static T* dalloc(size_t count, int64_t* tally = nullptr) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  HIPCHK(hipMalloc(&p, bytes));
  if (tally) *tally += (int64_t)bytes;
  return static_cast<T*>(p);
}
static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// workspace: device scratch for one validate call at a time
// ---------------------------------------------------------------------------

constexpr int CTL_WORDS = 64;
// control block layout (uint64 words)
enum {
  CTL_MATCH = 0, CTL_VIOL = 1, CTL_MFP = 2, CTL_VFP = 3, CTL_VCOUNT = 4, CTL_FLAGS = 5,
  CTL_NEEDSEL = 6, CTL_THRVALID = 7, CTL_LEVEL_N = 8 /* +i */, CTL_LEVEL_T = 16 /* +i */,
  CTL_ENTRIES = 24 /* +u */, CTL_OUTCOUNT = 32, CTL_THR = 40 /* 4 words = 8 int32 */
};

struct Workspace {
  int64_t n = 0, m = 0;
  uint64_t cap = 0;          // frontier partials per level in use
  uint64_t alloc_cap = 0;    // frontier partials per level allocated
  uint64_t pcap = 0;         // prefix/beg entries per level (>= n, >= cap)
  int64_t bytes = 0;
  int32_t* cand[2 * MAXK] = {};
  uint8_t* mem[MAXK] = {};
  uint8_t* mark[MAXK] = {};
  int32_t* posmap[MAXK] = {};
  uint32_t* cpi_beg[MAXK] = {};
  uint32_t* cpi_len[MAXK] = {};
  int32_t* cpi_ent[MAXK] = {};
  uint64_t* rowP = nullptr;   // [n+1]
  uint64_t* masks = nullptr;  // [max(m, n)/64 + 2]
  uint64_t* pre = nullptr;    // [max(m, n)/64 + 2]
  int32_t* cols[MAXK] = {};   // level i columns (i >= 2)
  uint64_t* P[MAXK] = {};
  uint32_t* beg[MAXK] = {};
  uint64_t* dcnt = nullptr;   // [2*MAXK] candidate counts, + scratch totals
  unsigned long long* stat_bytes = nullptr;  // [8] algorithmic bytes per kernel class
  ScanWs scan{};
  // chunked-path violation staging and selection
  int32_t* vbig = nullptr;
  uint64_t vbig_cap = 0;
  uint32_t* sel_state = nullptr;
  uint32_t* sel_hist = nullptr;
  int32_t* sel_out = nullptr;
  // per-GFD blocks for the fast path (grown on demand)
  uint64_t* ctl = nullptr;
  int32_t* vsmall = nullptr;
  int32_t* res = nullptr;
  size_t ngfd_cap = 0;
  uint64_t vsmall_cap = 0;  // tuples per GFD
  int res_K = 0;
  uint64_t* hctl = nullptr; // pinned mirror of ctl
  uint8_t ep = 0;           // u8 epoch counter for mem/mark arrays
  int64_t budget = 0;

  ~Workspace() {
    for (auto p : cand) dfree(p);
    for (auto p : mem) dfree(p);
    for (auto p : mark) dfree(p);
    for (auto p : posmap) dfree(p);
    for (auto p : cpi_beg) dfree(p);
    for (auto p : cpi_len) dfree(p);
    for (auto p : cpi_ent) dfree(p);
    for (auto p : cols) dfree(p);
    for (auto p : P) dfree(p);
    for (auto p : beg) dfree(p);
    dfree(rowP); dfree(masks); dfree(pre); dfree(dcnt); dfree(stat_bytes);
    dfree(scan.tile_state); dfree(scan.ticket); dfree(scan.err);
    dfree(vbig); dfree(sel_state); dfree(sel_hist); dfree(sel_out);
    dfree(ctl); dfree(vsmall); dfree(res);
    if (hctl) (void)hipHostFree(hctl);
  }
};

struct gfd_graph {
  int device = 0;
  DevGraph dg{};
  int64_t n = 0, m = 0;
  int32_t num_attrs = 0, nvl = 0, nel = 0;
  std::vector<uint32_t> lab_off;       // host copy [nvl+1]
  std::vector<uint64_t> lab_out_sum;   // sum of out-degrees per vertex label
  std::vector<uint64_t> lab_in_sum;
  std::vector<void*> owned;
  int64_t device_bytes = 0;
  std::mutex mu;
  std::vector<Workspace*> pool;        // idle workspaces
  std::vector<Workspace*> all;
  ~gfd_graph() {
    for (auto w : all) delete w;
    for (auto p : owned) dfree(p);
  }
};

// ---------------------------------------------------------------------------
// loader (Section II: E is a set of ordered pairs, one label per vertex/edge)
// ---------------------------------------------------------------------------

template <class F>
static void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 100000) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; t++)
    th.emplace_back([=] {
      int64_t a = n * t / nt, b = n * (t + 1) / nt;
      f(a, b);
    });
  for (auto& x : th) x.join();
}

extern "C" int32_t gfd_load_graph(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                  const int32_t* vlabel, const int32_t* elabel, int32_t num_attrs,
                                  const int32_t* const* attr, const gfd_load_opts* opts,
                                  gfd_graph** out) {
  if (!out) return set_error(GFD_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || m < 0 || num_attrs < 0) return set_error(GFD_EINVAL, "negative size");
  if (n >= (int64_t(1) << 31)) return set_error(GFD_EUNSUPPORTED, "n >= 2^31");
  if (m >= (int64_t(1) << 32) - 1) return set_error(GFD_EUNSUPPORTED, "m >= 2^32-1");
  if (!row_ptr || (n > 0 && !vlabel) || (m > 0 && (!col || !elabel)) || (num_attrs > 0 && !attr))
    return set_error(GFD_EINVAL, "null input array");
  for (int32_t a = 0; a < num_attrs; a++)
    if (n > 0 && !attr[a]) return set_error(GFD_EINVAL, "attribute column %d is NULL", a);
  if (row_ptr[0] != 0 || row_ptr[n] != m) return set_error(GFD_EINVAL, "row_ptr must run from 0 to m");
  for (int64_t v = 0; v < n; v++)
    if (row_ptr[v + 1] < row_ptr[v]) return set_error(GFD_EINVAL, "row_ptr decreases at %lld", (long long)v);
  int32_t maxvl = -1, maxel = -1;
  for (int64_t v = 0; v < n; v++) {
    if (vlabel[v] < 0) return set_error(GFD_EINVAL, "negative vertex label at %lld", (long long)v);
    maxvl = std::max(maxvl, vlabel[v]);
  }
  for (int64_t e = 0; e < m; e++) {
    if (col[e] < 0 || col[e] >= n) return set_error(GFD_EINVAL, "col[%lld] out of range", (long long)e);
    if (elabel[e] < 0) return set_error(GFD_EINVAL, "negative edge label at %lld", (long long)e);
    maxel = std::max(maxel, elabel[e]);
  }
  for (int32_t a = 0; a < num_attrs; a++)
    for (int64_t v = 0; v < n; v++)
      if (attr[a][v] < GFD_ABSENT) return set_error(GFD_EINVAL, "attribute %d value < -1 at %lld", a, (long long)v);

  // sorted out-rows; reject self-loops and duplicate pairs
  std::vector<uint32_t> out_off(n + 1), in_off(n + 1, 0);
  std::vector<int32_t> out_nbr(m), out_lab(m), in_nbr(m), in_lab(m);
  for (int64_t v = 0; v <= n; v++) out_off[v] = (uint32_t)row_ptr[v];
  std::atomic<int64_t> bad{-1};
  parallel_for(n, [&](int64_t a, int64_t b) {
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int64_t v = a; v < b; v++) {
      int64_t s = row_ptr[v], e = row_ptr[v + 1];
      tmp.resize(e - s);
      for (int64_t i = s; i < e; i++) tmp[i - s] = {col[i], elabel[i]};
      std::sort(tmp.begin(), tmp.end());
      for (int64_t i = s; i < e; i++) {
        out_nbr[i] = tmp[i - s].first;
        out_lab[i] = tmp[i - s].second;
        if (out_nbr[i] == v || (i > s && out_nbr[i] == out_nbr[i - 1])) bad = v;
      }
    }
  });
  if (bad >= 0)
    return set_error(GFD_EINVAL, "self-loop or duplicate edge in row %lld", (long long)bad.load());
  for (int64_t e = 0; e < m; e++) in_off[out_nbr[e] + 1]++;
  for (int64_t v = 0; v < n; v++) in_off[v + 1] += in_off[v];
  {
    std::vector<uint32_t> fill(in_off.begin(), in_off.end() - 1);
    for (int64_t v = 0; v < n; v++)
      for (uint32_t e = out_off[v]; e < out_off[v + 1]; e++) {
        uint32_t s = fill[out_nbr[e]]++;
        in_nbr[s] = (int32_t)v;
        in_lab[s] = out_lab[e];
      }
  }
  // label buckets (counting sort, ascending ids within a label)
  int32_t nvl = maxvl + 1;
  std::vector<uint32_t> lab_off(nvl + 1, 0);
  std::vector<int32_t> lab_vtx(n);
  std::vector<uint64_t> lab_out(nvl, 0), lab_in(nvl, 0);
  for (int64_t v = 0; v < n; v++) {
    lab_off[vlabel[v] + 1]++;
    lab_out[vlabel[v]] += out_off[v + 1] - out_off[v];
    lab_in[vlabel[v]] += in_off[v + 1] - in_off[v];
  }
  for (int32_t l = 0; l < nvl; l++) lab_off[l + 1] += lab_off[l];
  {
    std::vector<uint32_t> fill(lab_off.begin(), lab_off.end() - 1);
    for (int64_t v = 0; v < n; v++) lab_vtx[fill[vlabel[v]]++] = (int32_t)v;
  }
  std::vector<int32_t> attr_flat((size_t)num_attrs * n);
  for (int32_t a = 0; a < num_attrs; a++)
    std::memcpy(attr_flat.data() + (size_t)a * n, attr[a], sizeof(int32_t) * n);

  gfd_graph* g = new gfd_graph();
  try {
    HIPCHK(hipGetDevice(&g->device));
    hipStream_t st = opts ? (hipStream_t)opts->hip_stream : nullptr;
    auto up = [&](const void* src, size_t bytes) -> void* {
      void* p = dalloc<uint8_t>(bytes, &g->device_bytes);
      g->owned.push_back(p);
      if (bytes) HIPCHK(hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, st));
      return p;
    };
    g->n = n; g->m = m; g->num_attrs = num_attrs; g->nvl = nvl; g->nel = maxel + 1;
    g->dg.n = (int32_t)n;
    g->dg.m = (uint32_t)m;
    g->dg.num_attrs = num_attrs;
    g->dg.out_off = (const uint32_t*)up(out_off.data(), 4 * (n + 1));
    g->dg.out_nbr = (const int32_t*)up(out_nbr.data(), 4 * m);
    g->dg.out_lab = (const int32_t*)up(out_lab.data(), 4 * m);
    g->dg.in_off = (const uint32_t*)up(in_off.data(), 4 * (n + 1));
    g->dg.in_nbr = (const int32_t*)up(in_nbr.data(), 4 * m);
    g->dg.in_lab = (const int32_t*)up(in_lab.data(), 4 * m);
    g->dg.vlab = (const int32_t*)up(vlabel, 4 * n);
    g->dg.attr = (const int32_t*)up(attr_flat.data(), 4 * attr_flat.size());
    g->dg.lab_off = (const uint32_t*)up(lab_off.data(), 4 * lab_off.size());
    g->dg.lab_vtx = (const int32_t*)up(lab_vtx.data(), 4 * n);
    HIPCHK(hipStreamSynchronize(st));
    g->lab_off = std::move(lab_off);
    g->lab_out_sum = std::move(lab_out);
    g->lab_in_sum = std::move(lab_in);
  } catch (const GfdError& e) {
    delete g;
    return set_error(e.code, "%s", e.msg.c_str());
  }
  *out = g;
  return GFD_OK;
}

extern "C" void gfd_free_graph(gfd_graph* g) { delete g; }

extern "C" int32_t gfd_get_graph_info(const gfd_graph* g, gfd_graph_info* info) {
  if (!g || !info) return set_error(GFD_EINVAL, "null argument");
  info->n = g->n; info->m = g->m; info->num_attrs = g->num_attrs;
  info->num_vertex_labels = g->nvl; info->num_edge_labels = g->nel;
  info->device_bytes = g->device_bytes;
  return GFD_OK;
}

extern "C" const char* gfd_last_error(void) { return g_last_error.c_str(); }
extern "C" int32_t gfd_version(void) { return 100; }

// ---------------------------------------------------------------------------
// planner (host): Section IV-B -- root, spanning tree, core-first order
// ---------------------------------------------------------------------------

struct Plan {
  int k = 0, root = 0;
  int32_t qlab[MAXK];
  int32_t qe[MAXK][MAXK];  // label of pattern edge a->b, ANY, or NOEDGE
  int bfs[MAXK], parent[MAXK], order[MAXK], pos[MAXK];
  int min_out[MAXK], min_in[MAXK];
  bool core[MAXK];
  // pattern neighbours processed before / after each vertex in BFS order
  std::vector<int> down[MAXK], up[MAXK];
  // CPI adjacency for tree edge (parent[u], u)
  int adj_dir[MAXK];
  int32_t adj_prim[MAXK], adj_other[MAXK];
  bool is_parent[MAXK];
  // enumeration step i (position i >= 1)
  int nchk[MAXK];
  int32_t chk_pos[MAXK][MAXK], chk_fwd[MAXK][MAXK], chk_bwd[MAXK][MAXK];
  int nx = 0, ny = 0, y_false = 0;
  DevLit lit[2 * MAXLIT];
};

static int32_t pair_code(const Plan& p, int a, int b, bool induced) {
  if (p.qe[a][b] != NOEDGE) return p.qe[a][b];
  return induced ? PC_ABSENT : PC_FREE;
}

// Validates one spec; returns GFD_OK or an error with a message.
static int32_t check_spec(const gfd_graph* g, const gfd_spec& s, int idx) {
  const int k = s.num_vertices;
  if (k < 1 || k > GFD_MAX_K)
    return set_error(k < 1 ? GFD_EINVAL : GFD_EUNSUPPORTED, "spec %d: num_vertices %d", idx, k);
  for (int i = 0; i < k; i++)
    if (s.vertex_labels[i] < GFD_WILDCARD) return set_error(GFD_EINVAL, "spec %d: vertex label", idx);
  if (s.num_edges < 0 || s.num_edges > GFD_MAX_PATTERN_EDGES)
    return set_error(GFD_EINVAL, "spec %d: num_edges", idx);
  bool seen[MAXK][MAXK] = {};
  for (int e = 0; e < s.num_edges; e++) {
    const gfd_edge& q = s.edges[e];
    if (q.src < 0 || q.src >= k || q.dst < 0 || q.dst >= k || q.src == q.dst || q.label < GFD_WILDCARD)
      return set_error(GFD_EINVAL, "spec %d: edge %d malformed", idx, e);
    if (seen[q.src][q.dst]) return set_error(GFD_EINVAL, "spec %d: duplicate edge %d", idx, e);
    seen[q.src][q.dst] = true;
  }
  if (s.num_x < 0 || s.num_x > GFD_MAX_LITERALS || s.num_y < 0 || s.num_y > GFD_MAX_LITERALS)
    return set_error(GFD_EINVAL, "spec %d: literal count", idx);
  for (int i = 0; i < s.num_x + s.num_y; i++) {
    const gfd_literal& l = i < s.num_x ? s.x[i] : s.y[i - s.num_x];
    if (l.kind != GFD_LIT_CONST && l.kind != GFD_LIT_VAR) return set_error(GFD_EINVAL, "spec %d: literal kind", idx);
    if (l.var < 0 || l.var >= k || l.attr < 0 || l.attr >= g->num_attrs)
      return set_error(GFD_EINVAL, "spec %d: literal %d variable/attribute", idx, i);
    if (l.kind == GFD_LIT_CONST && l.constant < 0)
      return set_error(GFD_EINVAL, "spec %d: constant must be >= 0", idx);
    if (l.kind == GFD_LIT_VAR && (l.var2 < 0 || l.var2 >= k || l.attr2 < 0 || l.attr2 >= g->num_attrs))
      return set_error(GFD_EINVAL, "spec %d: literal %d second variable/attribute", idx, i);
  }
  // connectivity of the undirected skeleton
  int comp[MAXK];
  for (int i = 0; i < k; i++) comp[i] = i;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int e = 0; e < s.num_edges; e++) {
      int a = s.edges[e].src, b = s.edges[e].dst, c = std::min(comp[a], comp[b]);
      if (comp[a] != c || comp[b] != c) { comp[a] = comp[b] = c; changed = true; }
    }
  }
  for (int i = 0; i < k; i++)
    if (comp[i] != 0) return set_error(GFD_EUNSUPPORTED, "spec %d: disconnected pattern", idx);
  return GFD_OK;
}

static uint64_t bucket_size(const gfd_graph* g, int32_t L) {
  if (L == ANY) return (uint64_t)g->n;
  if (L >= g->nvl) return 0;
  return g->lab_off[L + 1] - g->lab_off[L];
}

static void make_plan(const gfd_graph* g, const gfd_spec& s, bool induced, Plan& p) {
  const int k = s.num_vertices;
  p.k = k;
  for (int a = 0; a < MAXK; a++)
    for (int b = 0; b < MAXK; b++) p.qe[a][b] = NOEDGE;
  for (int i = 0; i < k; i++) p.qlab[i] = s.vertex_labels[i];
  for (int e = 0; e < s.num_edges; e++) p.qe[s.edges[e].src][s.edges[e].dst] = s.edges[e].label;
  bool adj[MAXK][MAXK] = {};
  int deg[MAXK] = {};
  for (int a = 0; a < k; a++) {
    p.min_out[a] = p.min_in[a] = 0;
    for (int b = 0; b < k; b++) {
      if (p.qe[a][b] != NOEDGE) { p.min_out[a]++; }
      if (p.qe[b][a] != NOEDGE) { p.min_in[a]++; }
      adj[a][b] = a != b && (p.qe[a][b] != NOEDGE || p.qe[b][a] != NOEDGE);
      deg[a] += adj[a][b];
    }
  }
  // 2-core of the skeleton: peel vertices of degree <= 1
  bool alive[MAXK];
  int d2[MAXK];
  for (int a = 0; a < k; a++) { alive[a] = true; d2[a] = deg[a]; }
  for (bool ch = true; ch;) {
    ch = false;
    for (int a = 0; a < k; a++)
      if (alive[a] && d2[a] <= 1) {
        alive[a] = false;
        ch = true;
        for (int b = 0; b < k; b++)
          if (adj[a][b]) d2[b]--;
      }
  }
  bool any_core = false;
  for (int a = 0; a < k; a++) { p.core[a] = alive[a]; any_core |= alive[a]; }
  // root: smallest estimated candidates per skeleton degree among core
  // vertices (all vertices for a tree pattern); ties to the lower index
  double best = 1e300;
  p.root = 0;
  for (int a = 0; a < k; a++) {
    if (any_core && !p.core[a]) continue;
    double c = (double)bucket_size(g, p.qlab[a]) / std::max(1, deg[a]);
    if (c < best) { best = c; p.root = a; }
  }
  if (!any_core) p.core[p.root] = true;
  // BFS spanning tree
  int head = 0, tail = 0;
  bool vis[MAXK] = {};
  p.bfs[tail++] = p.root;
  vis[p.root] = true;
  p.parent[p.root] = -1;
  while (head < tail) {
    int a = p.bfs[head++];
    for (int b = 0; b < k; b++)
      if (adj[a][b] && !vis[b]) { vis[b] = true; p.parent[b] = a; p.bfs[tail++] = b; }
  }
  // matching order: core (BFS order), then forest non-leaves, then leaves
  int o = 0;
  for (int pass = 0; pass < 3; pass++)
    for (int j = 0; j < k; j++) {
      int a = p.bfs[j];
      bool leaf = !p.core[a] && deg[a] <= 1;
      int cls = p.core[a] ? 0 : (leaf ? 2 : 1);
      if (cls == pass) p.order[o++] = a;
    }
  for (int i = 0; i < k; i++) p.pos[p.order[i]] = i;
  // CPI marking steps
  int bidx[MAXK];
  for (int j = 0; j < k; j++) bidx[p.bfs[j]] = j;
  for (int a = 0; a < k; a++) {
    p.down[a].clear();
    p.up[a].clear();
    p.is_parent[a] = false;
  }
  for (int j = 0; j < k; j++) {
    int u = p.bfs[j];
    for (int w = 0; w < k; w++) {
      if (!adj[u][w]) continue;
      if (bidx[w] < j) p.down[u].push_back(w);  // top-down: earlier neighbours
      else p.up[u].push_back(w);                // bottom-up: later neighbours
    }
  }
  for (int u = 0; u < k; u++) {
    if (u == p.root) continue;
    int q = p.parent[u];
    p.is_parent[q] = true;
    if (p.qe[q][u] != NOEDGE) {
      p.adj_dir[u] = 0;
      p.adj_prim[u] = p.qe[q][u];
      p.adj_other[u] = pair_code(p, u, q, induced);
    } else {
      p.adj_dir[u] = 1;
      p.adj_prim[u] = p.qe[u][q];
      p.adj_other[u] = pair_code(p, q, u, induced);
    }
  }
  // probes per step
  p.nchk[0] = 0;
  for (int i = 1; i < k; i++) {
    int u = p.order[i], ppos = p.pos[p.parent[u]];
    p.nchk[i] = 0;
    for (int j = 0; j < i; j++) {
      if (j == ppos) continue;
      int w = p.order[j];
      int32_t f = pair_code(p, w, u, induced), b = pair_code(p, u, w, induced);
      if (f == PC_FREE && b == PC_FREE) continue;
      int c = p.nchk[i]++;
      p.chk_pos[i][c] = j;
      p.chk_fwd[i][c] = f;
      p.chk_bwd[i][c] = b;
    }
  }
  // literals, variables mapped to matching-order positions
  p.nx = s.num_x;
  p.ny = s.num_y;
  p.y_false = s.y_is_false ? 1 : 0;
  for (int i = 0; i < s.num_x + s.num_y; i++) {
    const gfd_literal& l = i < s.num_x ? s.x[i] : s.y[i - s.num_x];
    DevLit d{};
    d.kind = l.kind;
    d.pos = p.pos[l.var];
    d.attr = l.attr;
    d.pos2 = l.kind == GFD_LIT_VAR ? p.pos[l.var2] : 0;
    d.attr2 = l.kind == GFD_LIT_VAR ? l.attr2 : 0;
    d.value = l.kind == GFD_LIT_CONST ? l.constant : 0;
    p.lit[i] = d;
  }
  if (p.y_false) p.ny = 0;
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------

struct Timer {
  bool on = false;
  uint32_t mask = 0xFFu;  // kernel classes to time
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipStream_t st = nullptr;
  int launches[8] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  template <class F>
  void run(int cls, F f) {
    launches[cls]++;
    if (!on || !((mask >> cls) & 1u)) { f(); return; }
    hipEvent_t a = get(), b = get();
    HIPCHK(hipEventRecord(a, st));
    f();
    HIPCHK(hipEventRecord(b, st));
    recs.push_back({cls, a, b});
  }
  void collect(double* ms) {
    for (auto& r : recs) {
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.cls] += t;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  ~Timer() {
    for (auto& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};
enum { K_FILTER = 0, K_MARK = 1, K_ADJ = 2, K_EXT = 3, K_LAST = 4, K_SCAN = 5, K_TOPK = 6, K_OTHER = 7 };

static int grid_for(uint64_t items) {
  uint64_t b = (items + BS - 1) / BS;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, 2048));
}

struct Ctx {
  const gfd_graph* g;
  Workspace* ws;
  hipStream_t st;
  bool induced;
  int K;
  Timer tm;
  gfd_stats* stats;
  unsigned long long* stat_bytes;  // device [8] per kernel class, or nullptr
};

static uint8_t next_ep(Workspace* ws) {
  if (ws->ep == 255) ws->ep = 0;  // callers reset per GFD before this can happen
  return ++ws->ep;
}

// Clears the epoch-tagged byte arrays when the epoch counter is close to wrapping.
static void epoch_guard(Ctx& c) {
  Workspace* ws = c.ws;
  if (ws->ep < 160) return;
  for (int j = 0; j < MAXK; j++) {
    fill_u8(c.st, ws->mem[j], 0, ws->n);
    fill_u8(c.st, ws->mark[j], 0, ws->n);
  }
  ws->ep = 0;
}

static void alloc_workspace(gfd_graph* g, Workspace* ws, int64_t budget) {
  const int64_t n = g->n, m = g->m;
  ws->n = n; ws->m = m; ws->budget = budget;
  // frontier levels 2..7: 4*i bytes of columns + 12 bytes (prefix, begin) per slot
  int64_t per_slot = 0;
  for (int i = 2; i < MAXK; i++) per_slot += 4 * i + 12;
  ws->cap = (uint64_t)std::max<int64_t>(1024, budget / per_slot);
  ws->alloc_cap = ws->cap;
  ws->pcap = std::max<uint64_t>(ws->cap, (uint64_t)n) + 1;
  int64_t* t = &ws->bytes;
  for (int j = 0; j < 2 * MAXK; j++) ws->cand[j] = dalloc<int32_t>(n, t);
  for (int j = 0; j < MAXK; j++) {
    ws->mem[j] = dalloc<uint8_t>(n, t);
    ws->mark[j] = dalloc<uint8_t>(n, t);
    ws->posmap[j] = dalloc<int32_t>(n, t);
    ws->cpi_beg[j] = dalloc<uint32_t>(n, t);
    ws->cpi_len[j] = dalloc<uint32_t>(n, t);
    ws->cpi_ent[j] = dalloc<int32_t>(m, t);
  }
  ws->rowP = dalloc<uint64_t>(n + 1, t);
  uint64_t words = (uint64_t)std::max(n, m) / 64 + 2;
  ws->masks = dalloc<uint64_t>(words, t);
  ws->pre = dalloc<uint64_t>(words + 1, t);
  for (int i = 1; i < MAXK; i++) {
    if (i >= 2) ws->cols[i] = dalloc<int32_t>((size_t)i * ws->cap, t);
    ws->P[i] = dalloc<uint64_t>(ws->pcap + 1, t);
    ws->beg[i] = dalloc<uint32_t>(ws->pcap, t);
  }
  ws->dcnt = dalloc<uint64_t>(4 * MAXK, t);
  ws->stat_bytes = dalloc<unsigned long long>(8, t);
  uint64_t max_items = std::max<uint64_t>({ws->pcap, (uint64_t)m, (uint64_t)n}) + 1;
  ws->scan.max_tiles = max_items / SCAN_TILE + 2;
  ws->scan.tile_state = dalloc<uint64_t>(ws->scan.max_tiles, t);
  ws->scan.ticket = dalloc<uint32_t>(1, t);
  ws->scan.err = dalloc<uint32_t>(1, t);
  ws->scan.epoch = 0;
  ws->sel_state = dalloc<uint32_t>(MAXK + 2, t);
  ws->sel_hist = dalloc<uint32_t>(RADIX_BINS, t);
  ws->sel_out = dalloc<int32_t>((size_t)SORT_MAX * MAXK, t);
  HIPCHK(hipMemset(ws->scan.tile_state, 0, sizeof(uint64_t) * ws->scan.max_tiles));
  HIPCHK(hipMemset(ws->scan.ticket, 0, 4));
  HIPCHK(hipMemset(ws->scan.err, 0, 4));
  HIPCHK(hipMemset(ws->sel_hist, 0, 4 * RADIX_BINS));
  for (int j = 0; j < MAXK; j++) {
    HIPCHK(hipMemset(ws->mem[j], 0, std::max<int64_t>(n, 1)));
    HIPCHK(hipMemset(ws->mark[j], 0, std::max<int64_t>(n, 1)));
  }
  HIPCHK(hipHostMalloc((void**)&ws->hctl, sizeof(uint64_t) * CTL_WORDS, hipHostMallocDefault));
  HIPCHK(hipDeviceSynchronize());
}

static void ensure_vbig(Workspace* ws, uint64_t vcap) {
  if (ws->vbig_cap >= vcap) return;
  dfree(ws->vbig);
  ws->vbig = nullptr;
  ws->vbig = dalloc<int32_t>((size_t)vcap * MAXK);
  ws->vbig_cap = vcap;
}

static void ensure_per_gfd(Workspace* ws, size_t ngfd, uint64_t vsmall, int K) {
  if (ws->ngfd_cap >= ngfd && ws->vsmall_cap >= vsmall && ws->res_K >= K) return;
  // every region is laid out with these strides, so allocate with them
  const size_t want = std::max(ngfd, ws->ngfd_cap);
  const uint64_t vs = std::max<uint64_t>({vsmall, ws->vsmall_cap, 1});
  const int rk = std::max({K, ws->res_K, 1});
  dfree(ws->ctl);
  dfree(ws->vsmall);
  dfree(ws->res);
  ws->ctl = nullptr;
  ws->vsmall = nullptr;
  ws->res = nullptr;
  ws->ngfd_cap = 0;
  if (ws->hctl) { (void)hipHostFree(ws->hctl); ws->hctl = nullptr; }
  ws->ctl = dalloc<uint64_t>(want * CTL_WORDS);
  ws->vsmall = dalloc<int32_t>(want * vs * MAXK);
  ws->res = dalloc<int32_t>(want * (size_t)rk * MAXK);
  HIPCHK(hipHostMalloc((void**)&ws->hctl, sizeof(uint64_t) * CTL_WORDS * want, hipHostMallocDefault));
  ws->ngfd_cap = want;
  ws->vsmall_cap = vs;
  ws->res_K = rk;
}

struct CandRef {
  int cur[MAXK];
  int32_t* list(Workspace* ws, int u) const { return ws->cand[2 * u + cur[u]]; }
  uint64_t* cnt(Workspace* ws, int u) const { return ws->dcnt + 2 * u + cur[u]; }
};

struct GfdState {
  Plan plan;
  CandRef cr;
  uint8_t mem_ep[MAXK];
  uint64_t cand_ub[MAXK];
};

static int tiles_grid(uint64_t items) {
  uint64_t t = (items + BS - 1) / BS;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(t, 512));
}

// Pull constraints on candidates of u from the current candidate sets of the
// pattern neighbours `nbrs`: one per pattern edge between u and a neighbour.
static void add_pull(Ctx& c, GfdState& S, int u, const std::vector<int>& nbrs, CandArgs& ca) {
  const Plan& p = S.plan;
  ca.ncons = 0;
  for (int w : nbrs) {
    if (p.qe[w][u] != NOEDGE)  // w -> u: v needs an in-neighbour in C(w)
      ca.cons[ca.ncons++] = PullCons{1, p.qe[w][u], c.ws->mem[w], S.mem_ep[w]};
    if (p.qe[u][w] != NOEDGE)  // u -> w: v needs an out-neighbour in C(w)
      ca.cons[ca.ncons++] = PullCons{0, p.qe[u][w], c.ws->mem[w], S.mem_ep[w]};
  }
}

// CPI construction (Section IV-B, step 1) for one GFD; all asynchronous.
static void build_cpi(Ctx& c, GfdState& S) {
  const gfd_graph* g = c.g;
  Workspace* ws = c.ws;
  Plan& p = S.plan;
  const int k = p.k;
  epoch_guard(c);
  for (int u = 0; u < k; u++) {
    S.cr.cur[u] = 0;
    S.cand_ub[u] = bucket_size(g, p.qlab[u]);
  }
  unsigned long long* by = c.stat_bytes;
  // candidate and CPI-entry counters are atomic output cursors
  fill_u64(c.st, ws->dcnt, 0, 2 * MAXK);
  fill_u64(c.st, ws->dcnt + 2 * MAXK + 8, 0, MAXK);
  // top-down, BFS order: label bucket, degree filter, adjacency to the
  // candidates of every earlier pattern neighbour
  for (int j = 0; j < k; j++) {
    const int u = p.bfs[j];
    CandArgs ca{};
    ca.g = g->dg;
    add_pull(c, S, u, p.down[u], ca);
    ca.min_out = p.min_out[u];
    ca.min_in = p.min_in[u];
    const uint64_t bs = S.cand_ub[u];
    if (p.qlab[u] == ANY) ca.list = nullptr;
    else ca.list = g->dg.lab_vtx + (bs ? g->lab_off[p.qlab[u]] : 0);
    ca.d_n = nullptr;
    ca.n_host = ca.cap = bs;
    ca.out = S.cr.list(ws, u);
    ca.d_out_n = S.cr.cnt(ws, u);
    ca.mem = ws->mem[u];
    ca.mem_ep = S.mem_ep[u] = next_ep(ws);
    ca.posmap = (p.up[u].empty() && p.is_parent[u]) ? ws->posmap[u] : nullptr;
    ca.bytes = by ? by + K_FILTER : nullptr;
    c.tm.run(K_FILTER, [&] { cand_filter(c.st, ca, tiles_grid(bs)); });
  }
  // bottom-up, reverse BFS order: drop dead ends (no neighbour in the
  // candidate set of a later pattern neighbour)
  for (int j = k - 1; j >= 0; j--) {
    const int u = p.bfs[j];
    if (p.up[u].empty()) continue;
    CandArgs ca{};
    ca.g = g->dg;
    add_pull(c, S, u, p.up[u], ca);
    ca.list = S.cr.list(ws, u);
    ca.d_n = S.cr.cnt(ws, u);
    ca.cap = S.cand_ub[u];
    S.cr.cur[u] ^= 1;
    ca.out = S.cr.list(ws, u);
    ca.d_out_n = S.cr.cnt(ws, u);
    ca.mem = ws->mem[u];
    ca.mem_ep = S.mem_ep[u] = next_ep(ws);
    ca.posmap = p.is_parent[u] ? ws->posmap[u] : nullptr;
    ca.bytes = by ? by + K_FILTER : nullptr;
    c.tm.run(K_FILTER, [&] { cand_filter(c.st, ca, tiles_grid(S.cand_ub[u])); });
  }
  // CPI adjacency lists per spanning-tree edge
  for (int u = 0; u < k; u++) {
    if (u == p.root) continue;
    const int q = p.parent[u];
    CpiArgs a{};
    a.g = g->dg;
    a.dir = p.adj_dir[u];
    a.list = S.cr.list(ws, q);
    a.d_n = S.cr.cnt(ws, q);
    a.cap = S.cand_ub[q];
    a.prim = p.adj_prim[u];
    a.other = p.adj_other[u];
    a.mem = ws->mem[u];
    a.ep = S.mem_ep[u];
    a.cpi_beg = ws->cpi_beg[u];
    a.cpi_len = ws->cpi_len[u];
    a.cpi_ent = ws->cpi_ent[u];
    a.d_entries = ws->dcnt + 2 * MAXK + 8 + u;
    a.bytes = by ? by + K_ADJ : nullptr;
    c.tm.run(K_ADJ, [&] { cpi_adjacency(c.st, a, tiles_grid(S.cand_ub[q])); });
  }
  if (getenv("GFD_DEBUG_CPI")) {  // diagnostics: sizes of the candidate sets and CPI lists
    uint64_t h[4 * MAXK];
    HIPCHK(hipMemcpyAsync(h, ws->dcnt, sizeof h, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    fprintf(stderr, "[gfd] k=%d root=%d", k, p.root);
    for (int u = 0; u < k; u++)
      fprintf(stderr, " | u%d L%d bucket %llu cand %llu ent %llu", u, p.qlab[u],
              (unsigned long long)S.cand_ub[u], (unsigned long long)h[2 * u + S.cr.cur[u]],
              (unsigned long long)h[2 * MAXK + 8 + u]);
    fprintf(stderr, "\n");
  }
}

static void fill_ext_common(Ctx& c, GfdState& S, ExtArgs& a, int i) {
  const Plan& p = S.plan;
  a.g = c.g->dg;
  a.i = i;
  a.nchk = p.nchk[i];
  for (int j = 0; j < MAXK; j++) {
    a.chk_pos[j] = j < p.nchk[i] ? p.chk_pos[i][j] : 0;
    a.chk_fwd[j] = j < p.nchk[i] ? p.chk_fwd[i][j] : PC_FREE;
    a.chk_bwd[j] = j < p.nchk[i] ? p.chk_bwd[i][j] : PC_FREE;
  }
  a.k = p.k;
  for (int v = 0; v < MAXK; v++) a.var_pos[v] = v < p.k ? p.pos[v] : 0;
  a.nx = p.nx;
  a.ny = p.ny;
  a.y_false = p.y_false;
  for (int j = 0; j < 2 * MAXLIT; j++) a.lit[j] = p.lit[j];
}

struct LevelView {
  const int32_t* cols;
  uint64_t stride;
  const uint64_t* d_n;
  uint64_t cap;
};

static LevelView level_view(Ctx& c, GfdState& S, int i, uint64_t* ctl) {
  Workspace* ws = c.ws;
  if (i == 1) {
    int r = S.plan.root;
    return {S.cr.list(ws, r), 0, S.cr.cnt(ws, r), S.cand_ub[r]};
  }
  return {ws->cols[i], ws->cap, ctl + CTL_LEVEL_N + i, ws->cap};
}

// Fast path: every level in one pass, nothing read back.
static void enumerate_fast(Ctx& c, GfdState& S, uint64_t* ctl, int32_t* vbuf, uint64_t vcap) {
  Workspace* ws = c.ws;
  const Plan& p = S.plan;
  ExtArgs a{};
  fill_ext_common(c, S, a, 0);
  a.counters = (unsigned long long*)(ctl + CTL_MATCH);
  a.vbuf = vbuf;
  a.d_vcount = ctl + CTL_VCOUNT;
  a.vcap = c.K > 0 ? vcap : 0;
  a.thr = nullptr;
  a.d_thr_valid = (const uint32_t*)(ctl + CTL_THRVALID);
  a.d_flags = (uint32_t*)(ctl + CTL_FLAGS);
  if (p.k == 1) {
    const int r = p.root;
    a.a_begin = 0;
    a.a_end = ~0ull;
    c.tm.run(K_LAST, [&] {
      single_vertex(c.st, a, S.cr.list(ws, r), S.cr.cnt(ws, r), S.cand_ub[r], grid_for(S.cand_ub[r]));
    });
    return;
  }
  for (int i = 1; i < p.k; i++) {
    const int u = p.order[i], q = p.parent[u];
    LevelView lv = level_view(c, S, i, ctl);
    const int32_t* par = lv.cols + (uint64_t)p.pos[q] * lv.stride;
    c.tm.run(K_SCAN, [&] {
      scan_sources(c.st, ws->scan, par, lv.d_n, lv.cap, ws->posmap[q], ws->cpi_beg[u], ws->cpi_len[u], ws->beg[i],
                   ws->P[i], ctl + CTL_LEVEL_T + i);
    });
    fill_ext_common(c, S, a, i);
    a.src_cols = lv.cols;
    a.src_stride = lv.stride;
    a.d_nsrc = lv.d_n;
    a.src_cap = lv.cap;
    a.P = ws->P[i];
    a.beg = ws->beg[i];
    a.cpi_ent = ws->cpi_ent[u];
    a.a_begin = 0;
    a.a_end = ~0ull;
    const bool last = i == p.k - 1;
    a.bytes = c.stat_bytes ? c.stat_bytes + (last ? K_LAST : K_EXT) : nullptr;
    if (!last) {
      a.dst_cols = ws->cols[i + 1];
      a.dst_cap = ws->cap;
      a.d_ndst = ctl + CTL_LEVEL_N + i + 1;
    }
    c.tm.run(last ? K_LAST : K_EXT, [&] { extend(c.st, a, last, 1024); });
  }
}

// Radix select of the K-th smallest staged tuple, then the first K sorted into
// ws->sel_out.  Requires count > K.
static void select_first_k(Ctx& c, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap,
                           int k, uint64_t* ctl) {
  Workspace* ws = c.ws;
  c.tm.run(K_TOPK, [&] { select_begin(c.st, ws->sel_state, c.K); });
  const int grid = grid_for(vcap);
  for (int w = 0; w < k; w++) {
    const int shifts[3] = {21, 10, 0}, bits[3] = {11, 11, 10};
    for (int ps = 0; ps < 3; ps++)
      c.tm.run(K_TOPK, [&] {
        select_pass(c.st, vbuf, d_vcount, vcap, k, w, shifts[ps], bits[ps], ws->sel_state,
                    ws->sel_hist, grid);
      });
  }
  fill_u64(c.st, ctl + CTL_OUTCOUNT, 0, 1);
  c.tm.run(K_TOPK, [&] {
    select_compact(c.st, vbuf, d_vcount, vcap, k, ws->sel_state, ws->sel_out, ctl + CTL_OUTCOUNT,
                   grid);
  });
  c.tm.run(K_TOPK, [&] { sort_tuples(c.st, ws->sel_out, ctl + CTL_OUTCOUNT, k); });
}

// Chunked path: frontier levels processed in windows that fit the budget;
// violation staging compacted to the first K whenever it could overflow.
struct Chunked {
  Ctx& c;
  GfdState& S;
  uint64_t* ctl;
  uint64_t* h;  // pinned mirror
  uint64_t rd(int word) {
    HIPCHK(hipMemcpyAsync(h + word, ctl + word, 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    return h[word];
  }
  void compact_if_needed(uint64_t incoming) {
    Workspace* ws = c.ws;
    const int k = S.plan.k;
    uint64_t vc = rd(CTL_VCOUNT);
    if (vc + incoming <= ws->vbig_cap || vc <= (uint64_t)c.K) return;
    select_first_k(c, ws->vbig, ctl + CTL_VCOUNT, ws->vbig_cap, k, ctl);
    // keep the first K, threshold = the K-th
    HIPCHK(hipMemcpyAsync(ws->vbig, ws->sel_out, sizeof(int32_t) * c.K * k, hipMemcpyDeviceToDevice, c.st));
    HIPCHK(hipMemcpyAsync((int32_t*)(ctl + CTL_THR), ws->sel_out + (size_t)(c.K - 1) * k,
                          sizeof(int32_t) * k, hipMemcpyDeviceToDevice, c.st));
    fill_u64(c.st, ctl + CTL_VCOUNT, (uint64_t)c.K, 1);
    fill_u64(c.st, ctl + CTL_THRVALID, 1, 1);
  }
  void level(int i) {
    Workspace* ws = c.ws;
    const Plan& p = S.plan;
    const int u = p.order[i], q = p.parent[u];
    LevelView lv = level_view(c, S, i, ctl);
    const int32_t* par = lv.cols + (uint64_t)p.pos[q] * lv.stride;
    c.tm.run(K_SCAN, [&] {
      scan_sources(c.st, ws->scan, par, lv.d_n, lv.cap, ws->posmap[q], ws->cpi_beg[u], ws->cpi_len[u], ws->beg[i],
                   ws->P[i], ctl + CTL_LEVEL_T + i);
    });
    const uint64_t T = rd(CTL_LEVEL_T + i);
    if (c.stats) c.stats->attempts += T;
    ExtArgs a{};
    fill_ext_common(c, S, a, i);
    a.src_cols = lv.cols;
    a.src_stride = lv.stride;
    a.d_nsrc = lv.d_n;
    a.src_cap = lv.cap;
    a.P = ws->P[i];
    a.beg = ws->beg[i];
    a.cpi_ent = ws->cpi_ent[u];
    a.d_flags = (uint32_t*)(ctl + CTL_FLAGS);
    const bool last = i == p.k - 1;
    if (last) {
      a.counters = (unsigned long long*)(ctl + CTL_MATCH);
      a.vbuf = ws->vbig;
      a.d_vcount = ctl + CTL_VCOUNT;
      a.vcap = c.K > 0 ? ws->vbig_cap : 0;
      a.thr = (const int32_t*)(ctl + CTL_THR);
      a.d_thr_valid = (const uint32_t*)(ctl + CTL_THRVALID);
      const uint64_t W = c.K > 0 ? ws->vbig_cap - (uint64_t)c.K : T;
      for (uint64_t A0 = 0; A0 < T; A0 += W) {
        const uint64_t A1 = std::min(T, A0 + W);
        if (c.K > 0) compact_if_needed(A1 - A0);
        a.a_begin = A0;
        a.a_end = A1;
        c.tm.run(K_LAST, [&] { extend(c.st, a, true, grid_for(A1 - A0)); });
      }
      return;
    }
    a.dst_cols = ws->cols[i + 1];
    a.dst_cap = ws->cap;
    a.d_ndst = ctl + CTL_LEVEL_N + i + 1;
    for (uint64_t A0 = 0; A0 < T; A0 += ws->cap) {
      const uint64_t A1 = std::min(T, A0 + ws->cap);
      fill_u64(c.st, ctl + CTL_LEVEL_N + i + 1, 0, 1);
      a.a_begin = A0;
      a.a_end = A1;
      c.tm.run(K_EXT, [&] { extend(c.st, a, false, grid_for(A1 - A0)); });
      const uint64_t N = rd(CTL_LEVEL_N + i + 1);
      if (c.stats) c.stats->partials += N;
      if (N) level(i + 1);
    }
  }
};

static void enumerate_chunked(Ctx& c, GfdState& S, uint64_t* ctl, uint64_t* hmirror) {
  Workspace* ws = c.ws;
  const Plan& p = S.plan;
  fill_u64(c.st, ctl, 0, CTL_WORDS);
  if (p.k == 1) {
    ExtArgs a{};
    fill_ext_common(c, S, a, 0);
    a.counters = (unsigned long long*)(ctl + CTL_MATCH);
    a.vbuf = ws->vbig;
    a.d_vcount = ctl + CTL_VCOUNT;
    a.vcap = c.K > 0 ? ws->vbig_cap : 0;
    a.thr = nullptr;
    a.d_thr_valid = (const uint32_t*)(ctl + CTL_THRVALID);
    a.d_flags = (uint32_t*)(ctl + CTL_FLAGS);
    const int r = p.root;
    Chunked ch{c, S, ctl, hmirror};
    HIPCHK(hipMemcpyAsync(hmirror, S.cr.cnt(ws, r), 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    const uint64_t N = hmirror[0];
    a.thr = (const int32_t*)(ctl + CTL_THR);
    const uint64_t W = c.K > 0 ? ws->vbig_cap - (uint64_t)c.K : std::max<uint64_t>(N, 1);
    for (uint64_t A0 = 0; A0 < N; A0 += W) {
      const uint64_t A1 = std::min(N, A0 + W);
      if (c.K > 0) ch.compact_if_needed(A1 - A0);
      a.a_begin = A0;
      a.a_end = A1;
      c.tm.run(K_LAST, [&] {
        single_vertex(c.st, a, S.cr.list(ws, r), S.cr.cnt(ws, r), S.cand_ub[r], grid_for(A1 - A0));
      });
    }
    return;
  }
  Chunked ch{c, S, ctl, hmirror};
  ch.level(1);
}

static int64_t default_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return int64_t(2) << 30;
  int64_t b = (int64_t)(fr / 8);
  return std::max<int64_t>(int64_t(64) << 20, std::min<int64_t>(b, int64_t(8) << 30));
}

static Workspace* acquire_ws(gfd_graph* g, int64_t budget) {
  {
    std::lock_guard<std::mutex> lk(g->mu);
    for (size_t i = 0; i < g->pool.size(); i++)
      if (g->pool[i]->budget == budget) {
        Workspace* w = g->pool[i];
        g->pool.erase(g->pool.begin() + i);
        return w;
      }
  }
  Workspace* w = new Workspace();
  try {
    alloc_workspace(g, w, budget);
  } catch (...) {
    delete w;
    throw;
  }
  std::lock_guard<std::mutex> lk(g->mu);
  g->all.push_back(w);
  return w;
}

static void release_ws(gfd_graph* g, Workspace* w) {
  std::lock_guard<std::mutex> lk(g->mu);
  g->pool.push_back(w);
}

extern "C" int32_t gfd_validate_ex(const gfd_graph* gc, const gfd_spec* specs, int32_t num_specs,
                                   const gfd_validate_opts* opts, gfd_result* results,
                                   gfd_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  gfd_graph* g = const_cast<gfd_graph*>(gc);
  if (!g) return set_error(GFD_EINVAL, "graph is NULL");
  if (num_specs < 0 || (num_specs > 0 && (!specs || !results)))
    return set_error(GFD_EINVAL, "specs/results");
  gfd_validate_opts o{};
  o.k_max = 1024;
  o.semantics = GFD_SEM_INDUCED;
  if (opts) o = *opts;
  if (o.k_max < 0 || o.k_max > SORT_MAX) return set_error(o.k_max < 0 ? GFD_EINVAL : GFD_EUNSUPPORTED, "k_max %d (max %d)", o.k_max, SORT_MAX);
  if (o.semantics != GFD_SEM_INDUCED && o.semantics != GFD_SEM_MONO) return set_error(GFD_EINVAL, "semantics");
  if (o.batched != 0) return set_error(GFD_EUNSUPPORTED, "batched must be 0");
  if (o.mem_budget_bytes < 0 || o.frontier_cap < 0 || o.violation_cap < 0) return set_error(GFD_EINVAL, "negative option");
  for (int32_t i = 0; i < num_specs; i++) {
    int32_t rc = check_spec(g, specs[i], i);
    if (rc) return rc;
    if (o.k_max > 0 && !results[i].violations) return set_error(GFD_EINVAL, "result %d: violations buffer is NULL", i);
  }
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (num_specs == 0) return GFD_OK;
  const int K = o.k_max;
  Workspace* ws = nullptr;
  try {
    int64_t per_slot = 0;
    for (int i = 2; i < MAXK; i++) per_slot += 4 * i + 12;
    if (o.mem_budget_bytes && o.mem_budget_bytes < 1024 * per_slot)
      return set_error(GFD_ENOMEM, "mem_budget_bytes below %lld", (long long)(1024 * per_slot));
    int64_t budget = o.mem_budget_bytes ? o.mem_budget_bytes : default_budget();
    if (o.frontier_cap) budget = std::max<int64_t>(1024, o.frontier_cap) * per_slot;
    ws = acquire_ws(g, budget);
    ws->cap = ws->alloc_cap;
    if (o.frontier_cap) ws->cap = std::min<uint64_t>(ws->alloc_cap, (uint64_t)o.frontier_cap);
    uint64_t vsmall = o.violation_cap ? (uint64_t)o.violation_cap : 32768;
    uint64_t vbig = o.violation_cap ? (uint64_t)o.violation_cap : (uint64_t)(4u << 20);
    vsmall = std::max<uint64_t>(vsmall, (uint64_t)K + 1);
    vbig = std::max<uint64_t>(vbig, (uint64_t)K + 64);
    ensure_per_gfd(ws, (size_t)num_specs, vsmall, K);
    Ctx c{g, ws, (hipStream_t)o.hip_stream, o.semantics == GFD_SEM_INDUCED, K, Timer{}, stats,
          stats ? ws->stat_bytes : nullptr};
    const uint32_t cls_mask = ((uint32_t)o.flags >> 8) & 0xFFu;
    c.tm.on = stats && ((o.flags & GFD_FLAG_TIMING) || cls_mask);
    c.tm.mask = cls_mask ? cls_mask : 0xFFu;
    c.tm.st = c.st;
    if (stats) fill_u64(c.st, (uint64_t*)ws->stat_bytes, 0, 8);
    std::vector<GfdState> S(num_specs);
    for (int32_t i = 0; i < num_specs; i++) make_plan(g, specs[i], c.induced, S[i].plan);
    HIPCHK(hipMemsetAsync(ws->scan.err, 0, 4, c.st));
    fill_u64(c.st, ws->ctl, 0, (uint64_t)num_specs * CTL_WORDS);
    const bool force_chunked = (o.flags & GFD_FLAG_FORCE_CHUNKED) != 0;
    std::vector<char> redo(num_specs, force_chunked ? 1 : 0);
    if (!force_chunked) {
      for (int32_t i = 0; i < num_specs; i++) {
        uint64_t* ctl = ws->ctl + (size_t)i * CTL_WORDS;
        int32_t* vb = ws->vsmall + (size_t)i * ws->vsmall_cap * MAXK;
        build_cpi(c, S[i]);
        enumerate_fast(c, S[i], ctl, vb, vsmall);
        if (K > 0)
          c.tm.run(K_TOPK, [&] {
            topk_small(c.st, vb, ctl + CTL_VCOUNT, vsmall, S[i].plan.k, K,
                       ws->res + (size_t)i * ws->res_K * MAXK, (uint32_t*)(ctl + CTL_NEEDSEL));
          });
      }
    }
    HIPCHK(hipMemcpyAsync(ws->hctl, ws->ctl, sizeof(uint64_t) * CTL_WORDS * num_specs,
                          hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    std::vector<uint64_t> H(ws->hctl, ws->hctl + (size_t)CTL_WORDS * num_specs);
    for (int32_t i = 0; i < num_specs && !force_chunked; i++) {
      const uint64_t* h = &H[(size_t)i * CTL_WORDS];
      if ((h[CTL_FLAGS] & 3u) || h[CTL_VCOUNT] > vsmall) redo[i] = 1;
    }
    for (int32_t i = 0; i < num_specs; i++) {
      uint64_t* ctl = ws->ctl + (size_t)i * CTL_WORDS;
      int32_t* res = ws->res + (size_t)i * ws->res_K * MAXK;
      const int k = S[i].plan.k;
      if (redo[i]) {
        if (stats) stats->chunked_gfds++;
        ensure_vbig(ws, vbig);
        build_cpi(c, S[i]);
        enumerate_chunked(c, S[i], ctl, ws->hctl);
        if (K > 0) {
          c.tm.run(K_TOPK, [&] {
            topk_small(c.st, ws->vbig, ctl + CTL_VCOUNT, ws->vbig_cap, k, K, res,
                       (uint32_t*)(ctl + CTL_NEEDSEL));
          });
        }
        HIPCHK(hipMemcpyAsync(&H[(size_t)i * CTL_WORDS], ctl, sizeof(uint64_t) * CTL_WORDS,
                              hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        if (K > 0 && H[(size_t)i * CTL_WORDS + CTL_NEEDSEL]) {
          select_first_k(c, ws->vbig, ctl + CTL_VCOUNT, ws->vbig_cap, k, ctl);
          HIPCHK(hipMemcpyAsync(res, ws->sel_out, sizeof(int32_t) * K * k, hipMemcpyDeviceToDevice, c.st));
        }
      } else if (K > 0 && H[(size_t)i * CTL_WORDS + CTL_NEEDSEL]) {
        int32_t* vb = ws->vsmall + (size_t)i * ws->vsmall_cap * MAXK;
        select_first_k(c, vb, ctl + CTL_VCOUNT, vsmall, k, ctl);
        HIPCHK(hipMemcpyAsync(res, ws->sel_out, sizeof(int32_t) * K * k, hipMemcpyDeviceToDevice, c.st));
      }
    }
    // results
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, ws->scan.err, 4, hipMemcpyDeviceToHost, c.st));
    std::vector<int32_t> hres((size_t)num_specs * std::max(K, 1) * MAXK);
    if (K > 0)
      for (int32_t i = 0; i < num_specs; i++)
        HIPCHK(hipMemcpyAsync(hres.data() + (size_t)i * K * MAXK, ws->res + (size_t)i * ws->res_K * MAXK,
                              sizeof(int32_t) * K * S[i].plan.k, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    if (err) throw GfdError{GFD_EDEVICE, "scan look-back did not complete"};
    int32_t rc = GFD_OK;
    for (int32_t i = 0; i < num_specs; i++) {
      const uint64_t* h = &H[(size_t)i * CTL_WORDS];
      gfd_result& r = results[i];
      r.match_count = h[CTL_MATCH];
      r.violation_count = h[CTL_VIOL];
      r.match_fp = h[CTL_MFP];
      r.violation_fp = h[CTL_VFP];
      r.satisfied = r.violation_count == 0;
      r.num_reported = (int32_t)std::min<uint64_t>((uint64_t)K, r.violation_count);
      if (K > 0 && r.num_reported)
        std::memcpy(r.violations, hres.data() + (size_t)i * K * MAXK,
                    sizeof(int32_t) * r.num_reported * S[i].plan.k);
      if ((r.match_count >> 63) || (r.violation_count >> 63))
        rc = set_error(GFD_EOVERFLOW, "spec %d: counter passed 2^63", i);
      if (stats) {
        for (int l = 1; l < MAXK; l++) {
          if (!redo[i]) stats->attempts += h[CTL_LEVEL_T + l];
          if (!redo[i] && l >= 2) stats->partials += h[CTL_LEVEL_N + l];
        }
      }
    }
    if (stats) {
      unsigned long long hb[8];
      HIPCHK(hipMemcpy(hb, ws->stat_bytes, sizeof hb, hipMemcpyDeviceToHost));
      for (int j = 0; j < 8; j++) stats->class_bytes[j] = hb[j];
      if (c.tm.on) c.tm.collect(stats->class_ms);
      for (int j = 0; j < 8; j++) { stats->class_launches[j] = c.tm.launches[j]; stats->launches += c.tm.launches[j]; }
      stats->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    release_ws(g, ws);
    return rc;
  } catch (const GfdError& e) {
    if (ws) release_ws(g, ws);
    return set_error(e.code, "%s", e.msg.c_str());
  } catch (const std::bad_alloc&) {
    if (ws) release_ws(g, ws);
    return set_error(GFD_ENOMEM, "host allocation failed");
  }
}

extern "C" int32_t gfd_validate(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                                const gfd_validate_opts* opts, gfd_result* results) {
  return gfd_validate_ex(g, specs, num_specs, opts, results, nullptr);
}
