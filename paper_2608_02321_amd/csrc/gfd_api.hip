// C ABI, graph loader, per-GFD planner and launch driver.
//
// Path per GFD (FastGFDs paper, Section IV-B, on one GPU):
//   plan (host, microseconds): 2-core of the pattern skeleton, root, BFS
//     spanning tree, core-first matching order, per-step probes;
//   CPI build (device): label/degree candidate filter, one top-down and one
//     bottom-up marking pass, CPI adjacency lists per spanning-tree edge;
//   enumeration (device): level-synchronous extension over the CPI, the
//     X -> Y check fused into the last level, first-K selection.
// A batch's main pass is queued without host round trips (and replayed from
// a captured graph once its shape repeats); one synchronisation per batch
// reads the status words.  A GFD whose frontiers or CPI lists did not fit
// runs again once the pool or arena has grown, then in a smaller batch, then
// alone, and last on the bounded path, which bounds every level by the
// budget; one whose violation staging overflowed runs its last level again
// under a threshold.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <optional>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <functional>
#include <memory>
#include <vector>

#include "gfd.h"
#include "gfd_internal.h"
#include "gfd_serve_queue.h"

using namespace gfd;

// A named range of host time for profilers (roctx: `rocprofv3 --marker-trace`
// lists it beside the kernels the range enqueued); nearly free when no tool
// is attached.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

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

// Device memory of a graph or a workspace: the caller's allocator callbacks,
// or hipMalloc / hipFree when none is given.
struct DevAlloc {
  gfd_allocator cb{};
  hipStream_t st = nullptr;  // the stream handed to cb.alloc
  int64_t live = 0;          // bytes handed out and not yet returned
  // fixed area (the entry point that allocates nothing): blocks are carved
  // from [area, area + area_cap) in order; returning the last one takes it back
  uint8_t* area = nullptr;
  size_t area_cap = 0, area_top = 0;
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  void* get(size_t bytes) {
    bytes = std::max<size_t>(bytes, 1);
    void* p = nullptr;
    if (area) {
      if (area_top + round(bytes) > area_cap)
        throw GfdError{GFD_ENOMEM, "the call needs more than the " + std::to_string(area_cap >> 20) +
                                       " MiB scratch area (" + std::to_string(bytes) + " more bytes)"};
      p = area + area_top;
      area_top += round(bytes);
    } else if (cb.alloc) {
      p = cb.alloc(cb.ctx, (int64_t)bytes, (void*)st);
      if (!p)
        throw GfdError{GFD_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
      if ((uintptr_t)p % 256) {
        cb.free(cb.ctx, p, (int64_t)bytes);
        throw GfdError{GFD_EINVAL, "allocator callback returned memory not aligned to 256 bytes"};
      }
    } else {
      HIPCHK(hipMalloc(&p, bytes));
    }
    live += (int64_t)bytes;
    return p;
  }
  void put(void* p, size_t bytes) {
    if (!p) return;
    bytes = std::max<size_t>(bytes, 1);
    live -= (int64_t)bytes;
    if (area) {
      if ((uint8_t*)p + round(bytes) == area + area_top) area_top -= round(bytes);
    } else if (cb.alloc) {
      cb.free(cb.ctx, p, (int64_t)bytes);
    } else {
      (void)hipFree(p);
    }
  }
  bool same(const gfd_allocator& o) const {
    return cb.alloc == o.alloc && cb.free == o.free && cb.ctx == o.ctx;
  }
};

// An allocator option: alloc without free is malformed.
static int32_t check_allocator(const gfd_allocator& a) {
  if (a.alloc && !a.free) return set_error(GFD_EINVAL, "allocator has alloc but no free");
  return GFD_OK;
}

template <class T>
static T* dalloc(DevAlloc& al, size_t count) {
  return static_cast<T*>(al.get(std::max<size_t>(count, 1) * sizeof(T)));
}
// Returns p (count elements of T) to al and clears it.
template <class T>
static void dfree(DevAlloc& al, T*& p, size_t count) {
  al.put((void*)p, std::max<size_t>(count, 1) * sizeof(T));
  p = nullptr;
}
// Device-side address of mapped pinned host memory, or null if the runtime
// gives none (uploads from it then take the DMA copy).
static const uint8_t* mapped_ptr(void* h) {
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return static_cast<const uint8_t*>(d);
}

// ---------------------------------------------------------------------------
// workspace: device memory for one validate call at a time
// ---------------------------------------------------------------------------

constexpr int CTL_WORDS = 64;
// per-job control block layout (uint64 words)
enum {
  CTL_MATCH = 0, CTL_VIOL = 1, CTL_MFP = 2, CTL_VFP = 3, CTL_VCOUNT = 4, CTL_FLAGS = 5,
  CTL_NEEDSEL = 6, CTL_THRVALID = 7, CTL_LEVEL_N = 8 /* +i */, CTL_LEVEL_T = 16 /* +i */,
  CTL_TOTAL = 24, CTL_OUTCOUNT = 25, CTL_TICKET = 26, CTL_CPIBASE = 27, CTL_CPIASK = 28,
  CTL_CAND = 32 /* +2u+b */,
  CTL_THR = 48 /* 4 words = 8 int32 */
};

constexpr int SEL_STATE_WORDS = 16;

struct GraphEntry;
struct Workspace;
static void drop_graphs(Workspace* ws);

struct Workspace {
  uint8_t* arena = nullptr;         // per-job regions of the current batch
  size_t arena_bytes = 0;
  int32_t* cpi_arena = nullptr;     // CPI entries of every job of a batch
  uint64_t cpi_cap = 0;
  uint8_t* jobrec = nullptr;        // device job records
  size_t jobrec_bytes = 0;
  uint8_t* hjobrec = nullptr;       // pinned staging for the records
  const uint8_t* hjobrec_dev = nullptr;  // its device-side address (mapped), or null
  size_t hjobrec_bytes = 0;
  uint64_t* hctl = nullptr;         // pinned mirror of control blocks
  size_t hctl_words = 0;
  int32_t* hres = nullptr;          // pinned mirror of a batch's first-K slots
  uint32_t* hitpool = nullptr;      // filter hit bitmaps of a batch, zero at rest
  size_t hitpool_words = 0;
  bool hitpool_dirty = false;       // a call using it did not finish: clear before use
  size_t hres_words = 0;
  unsigned long long* misc = nullptr;  // [0] CPI cursor, [8..15] bytes per class
  uint32_t* err = nullptr;
  uint32_t epoch = 0;
  // bounded path: per-level prefixes, violation staging, selection
  uint8_t* chunk = nullptr;
  size_t chunk_bytes = 0;
  int32_t* vbig = nullptr;
  uint64_t vbig_cap = 0;
  // batched radix select: per-job state and histograms, records
  uint32_t* sel_state = nullptr;    // [MAX_JOBS * SEL_STATE_WORDS]
  uint32_t* sel_hist = nullptr;     // [MAX_JOBS * RADIX_BINS], zero at rest
  int32_t* sel_out = nullptr;       // [SORT_MAX * MAXK]
  uint8_t* selrec = nullptr;        // [MAX_JOBS] SelJob records
  uint8_t* hselrec = nullptr;       // pinned staging for them
  const uint8_t* hselrec_dev = nullptr;
  uint64_t* hmisc = nullptr;        // pinned: [0] CPI cursor, [1] error word, [2..9] class bytes,
                                    // [10] frontier pool cursor
  int32_t* pack = nullptr;          // a batch's reported tuples, back to back
  size_t pack_words = 0;
  uint8_t* front = nullptr;         // frontier pool of a batch (fast path), bump-allocated
  size_t front_bytes = 0;           //   on the device level by level (cursor misc[1])
  size_t front_want = 0;            // pool size the next batch should have (grows with use)
  size_t cpi_want = 0;              // CPI arena entries the next batch should have
  hipEvent_t pack_ev = nullptr;     // the last packed copy to ws->hres has landed
  int64_t budget = 0;
  DevAlloc al;                      // where every device buffer above comes from
  bool pageable = false;            // host staging in ordinary memory (no pinned allocation)

  void* host_get(size_t bytes, bool mapped) {
    if (pageable) return ::operator new(std::max<size_t>(bytes, 1));
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, std::max<size_t>(bytes, 1), mapped ? hipHostMallocMapped : hipHostMallocDefault));
    return p;
  }
  void host_put(void* p) {
    if (!p) return;
    if (pageable) ::operator delete(p);
    else (void)hipHostFree(p);
  }
  // Drops every device buffer without returning it: a fixed area is carved
  // again from its start by the next call.
  void forget_device_buffers() {
    forget_call_buffers();
    misc = nullptr; err = nullptr; sel_state = nullptr; sel_hist = nullptr; sel_out = nullptr;
    selrec = nullptr; front_want = 0; cpi_want = 0;
    al.area_top = 0;
    area_mark = 0;
    al.live = 0;
  }
  // The buffers above the fixed ones (control words, selection state).
  void forget_call_buffers() {
    arena = nullptr; arena_bytes = 0; cpi_arena = nullptr; cpi_cap = 0; jobrec = nullptr;
    jobrec_bytes = 0; hitpool = nullptr; hitpool_words = 0; hitpool_dirty = false;
    chunk = nullptr; chunk_bytes = 0; vbig = nullptr; vbig_cap = 0; pack = nullptr; pack_words = 0;
    front = nullptr; front_bytes = 0;
  }
  size_t area_mark = 0;             // fixed area: where the fixed buffers end
  // captured main passes of batches, replayed when a batch of the same shape
  // comes again (oldest first); a graph is valid only for the generation of
  // the buffers it was captured on
  uint64_t gen = 0;
  std::vector<GraphEntry*> graphs;
  hipStream_t cap_stream = nullptr;
  std::deque<size_t> seen;          // hashes of batch shapes run once (captured on the second run)
  // the last call's plans and batches, reused by a call with the same GFDs and
  // options (validating one set again and again): planning is host time the
  // GPU waits through at the start of every call
  std::shared_ptr<struct PlanMemo> memo;

  ~Workspace() {
    drop_graphs(this);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    dfree(al, arena, arena_bytes);
    dfree(al, cpi_arena, cpi_cap);
    dfree(al, hitpool, hitpool_words);
    dfree(al, jobrec, jobrec_bytes);
    dfree(al, misc, 16);
    dfree(al, err, 1);
    dfree(al, chunk, chunk_bytes);
    dfree(al, vbig, (size_t)vbig_cap * MAXK);
    dfree(al, sel_state, (size_t)MAX_JOBS * SEL_STATE_WORDS);
    dfree(al, sel_hist, (size_t)MAX_JOBS * RADIX_BINS);
    dfree(al, sel_out, (size_t)SORT_MAX * MAXK);
    dfree(al, selrec, sizeof(SelJob) * MAX_JOBS);
    dfree(al, pack, pack_words);
    dfree(al, front, front_bytes);
    host_put(hjobrec);
    host_put(hselrec);
    host_put(hmisc);
    if (pack_ev) (void)hipEventDestroy(pack_ev);
    host_put(hctl);
    host_put(hres);
  }
};

static uint64_t front_usable(const Workspace* ws);
static uint64_t cpi_usable(const Workspace* ws);

struct gfd_graph {
  int device = 0;
  DevGraph dg{};
  int64_t n = 0, m = 0;
  int32_t num_attrs = 0, nvl = 0, nel = 0;
  std::vector<uint32_t> lab_off;       // host copy [nvl+1]
  std::vector<uint32_t> elb_blk[2];    // host: first row of each (vertex label, edge label) block
  std::vector<uint32_t> elt_blk[2];    // host: the same per (vertex label, edge label, far label)
  std::vector<uint32_t> elb_ent[2];    // host: first entry of each (vertex label, edge label) block
  std::vector<uint32_t> elt_ent[2];    // host: the same per (vertex label, edge label, far label)
  bool triples = false;                // elt_* built
  std::vector<uint64_t> lab_out_sum;   // sum of out-degrees per vertex label
  std::vector<uint64_t> lab_in_sum;
  DevAlloc al;                         // where the graph's device arrays come from
  std::vector<std::pair<void*, size_t>> owned;
  int64_t device_bytes = 0;
  std::mutex mu;
  std::vector<Workspace*> pool;        // idle workspaces
  std::vector<Workspace*> all;
  void drop_workspaces() {
    if (!all.empty()) {  // with this graph's device current (restored after)
      int cur = -1;
      (void)hipGetDevice(&cur);
      if (cur != device) (void)hipSetDevice(device);
      (void)hipDeviceSynchronize();
      if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    }
    for (auto w : all) delete w;
    all.clear();
    pool.clear();
  }
  ~gfd_graph() {
    drop_workspaces();
    for (auto& p : owned) al.put(p.first, p.second);
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

// The loader proper; may throw (GfdError, std::bad_alloc, ...), which the
// C entry point turns into status codes.
static int32_t load_graph_impl(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                               const int32_t* vlabel, const int32_t* elabel, int32_t num_attrs,
                               const int32_t* const* attr, const gfd_load_opts* opts,
                               gfd_graph** out) {
  if (!out) return set_error(GFD_EINVAL, "out is NULL");
  *out = nullptr;
  const Range whole("gfd_load_graph");
  gfd_load_opts lo{};
  if (opts) lo = *opts;
  if (lo.mem_kind != GFD_MEM_HOST && lo.mem_kind != GFD_MEM_DEVICE)
    return set_error(GFD_EINVAL, "mem_kind %d", lo.mem_kind);
  if (int32_t rc = check_allocator(lo.allocator)) return rc;
  if (n < 0 || m < 0 || num_attrs < 0) return set_error(GFD_EINVAL, "negative size");
  if (n >= (int64_t(1) << 31)) return set_error(GFD_EUNSUPPORTED, "n >= 2^31");
  if (m >= (int64_t(1) << 32) - 1) return set_error(GFD_EUNSUPPORTED, "m >= 2^32-1");
  if (!row_ptr || (n > 0 && !vlabel) || (m > 0 && (!col || !elabel)) || (num_attrs > 0 && !attr))
    return set_error(GFD_EINVAL, "null input array");
  for (int32_t a = 0; a < num_attrs; a++)
    if (n > 0 && !attr[a]) return set_error(GFD_EINVAL, "attribute column %d is NULL", a);
  hipStream_t st = (hipStream_t)lo.hip_stream;
  // device-resident inputs are read into host copies first (the views below
  // are built on the host)
  std::vector<int64_t> h_row;
  std::vector<int32_t> h_col, h_vl, h_el, h_attr;
  std::vector<const int32_t*> h_attr_ptr;
  if (lo.mem_kind == GFD_MEM_DEVICE) {
    auto rd = [&](auto& vec, const void* src, size_t count) {
      vec.resize(count);
      if (count)
        HIPCHK(hipMemcpyAsync(vec.data(), src, count * sizeof(vec[0]), hipMemcpyDeviceToHost, st));
    };
    rd(h_row, row_ptr, (size_t)n + 1);
    rd(h_col, col, (size_t)m);
    rd(h_vl, vlabel, (size_t)n);
    rd(h_el, elabel, (size_t)m);
    h_attr.resize((size_t)num_attrs * n);
    for (int32_t a = 0; a < num_attrs; a++)
      if (n)
        HIPCHK(hipMemcpyAsync(h_attr.data() + (size_t)a * n, attr[a], sizeof(int32_t) * n,
                              hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int32_t a = 0; a < num_attrs; a++) h_attr_ptr.push_back(h_attr.data() + (size_t)a * n);
    row_ptr = h_row.data();
    col = h_col.data();
    vlabel = h_vl.data();
    elabel = h_el.data();
    attr = h_attr_ptr.data();
  }
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
  // host tables are sized by the largest label ids (label buckets) and by
  // their product (edge-label block keys)
  if (maxvl > GFD_MAX_LABEL || maxel > GFD_MAX_LABEL)
    return set_error(GFD_EUNSUPPORTED, "label id above %d (vertex %d, edge %d)", GFD_MAX_LABEL, maxvl, maxel);
  if ((int64_t)(maxvl + 1) * (int64_t)std::max(maxel + 1, 1) > (int64_t)GFD_MAX_LABEL_PAIRS)
    return set_error(GFD_EUNSUPPORTED, "more than %d (vertex label, edge label) pairs", GFD_MAX_LABEL_PAIRS);
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
  const int32_t nvl = maxvl + 1;  // <= GFD_MAX_LABEL + 1: no overflow
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
  std::vector<uint32_t> lab_pos(n);  // position of v within its label bucket
  for (int32_t l = 0; l < nvl; l++)
    for (uint32_t p = lab_off[l]; p < lab_off[l + 1]; p++) lab_pos[lab_vtx[p]] = p - lab_off[l];
  {
  }
  // label-ordered view: the rows of lab_vtx[0..n) laid out in that order, so
  // the rows of one label bucket form one contiguous slice
  std::vector<uint32_t> lv_out_off(n + 1, 0), lv_in_off(n + 1, 0);
  std::vector<int32_t> lv_out_nbr(m), lv_out_lab(m), lv_in_nbr(m), lv_in_lab(m);
  for (int64_t p = 0; p < n; p++) {
    const int32_t v = lab_vtx[p];
    lv_out_off[p + 1] = lv_out_off[p] + (out_off[v + 1] - out_off[v]);
    lv_in_off[p + 1] = lv_in_off[p] + (in_off[v + 1] - in_off[v]);
  }
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t p = a; p < b; p++) {
      const int32_t v = lab_vtx[p];
      std::memcpy(&lv_out_nbr[lv_out_off[p]], &out_nbr[out_off[v]], 4 * (out_off[v + 1] - out_off[v]));
      std::memcpy(&lv_out_lab[lv_out_off[p]], &out_lab[out_off[v]], 4 * (out_off[v + 1] - out_off[v]));
      std::memcpy(&lv_in_nbr[lv_in_off[p]], &in_nbr[in_off[v]], 4 * (in_off[v + 1] - in_off[v]));
      std::memcpy(&lv_in_lab[lv_in_off[p]], &in_lab[in_off[v]], 4 * (in_off[v + 1] - in_off[v]));
    }
  });
  // combined rows: for every vertex the ascending union of its out- and
  // in-neighbours, each with the labels of both edges (v -> w, w -> v), so one
  // search answers a constraint on both directions of a pair
  std::vector<uint64_t> sym_off(n + 1, 0);
  auto merge_row = [&](int64_t v, int32_t* nb, int32_t* lb) -> uint64_t {
    uint32_t i = out_off[v], ie = out_off[v + 1], j = in_off[v], je = in_off[v + 1];
    uint64_t c = 0;
    while (i < ie || j < je) {
      const int32_t a = i < ie ? out_nbr[i] : INT32_MAX, b = j < je ? in_nbr[j] : INT32_MAX;
      const int32_t w = a < b ? a : b;
      int32_t lo = NOEDGE, li = NOEDGE;
      if (a == w) lo = out_lab[i++];
      if (b == w) li = in_lab[j++];
      if (nb) {
        nb[c] = w;
        lb[2 * c] = lo;
        lb[2 * c + 1] = li;
      }
      c++;
    }
    return c;
  };
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t v = a; v < b; v++) sym_off[v + 1] = merge_row(v, nullptr, nullptr);
  });
  for (int64_t v = 0; v < n; v++) sym_off[v + 1] += sym_off[v];
  std::vector<int32_t> sym_nbr(sym_off[n]), sym_lab(2 * sym_off[n]);
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t v = a; v < b; v++)
      merge_row(v, sym_nbr.data() + sym_off[v], sym_lab.data() + 2 * sym_off[v]);
  });
  // neighbour tables of the long combined rows
  std::vector<uint64_t> hub_off(n + 1, 0);
  for (int64_t v = 0; v < n; v++) {
    const uint64_t d = sym_off[v + 1] - sym_off[v];
    uint64_t t = 0;
    if (d >= HUB_MIN) {
      t = 1;
      while (t < 2 * d) t <<= 1;
    }
    hub_off[v + 1] = hub_off[v] + t;
  }
  std::vector<uint8_t> hub_tab(hub_off[n], 0);
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t v = a; v < b; v++) {
      const uint64_t t = hub_off[v + 1] - hub_off[v];
      if (!t) continue;
      uint8_t* tab = hub_tab.data() + hub_off[v];
      for (uint64_t e = sym_off[v]; e < sym_off[v + 1]; e++) {
        uint64_t i = hub_slot(sym_nbr[e], t);
        while (tab[i] != 0) i = (i + 1) & (t - 1);
        tab[i] = hub_fp(sym_nbr[e]);
      }
    }
  });
  // edge-label blocks per direction: for every (vertex label, edge label) the
  // bucket rows with such edges, in bucket order, and those edges' far ends;
  // and the same keyed by (vertex label, edge label, far end's label), built
  // when there are at most LABEL_TRIPLES_MAX such keys.  A block's rows list a
  // bucket row once per run of entries with the block's key.
  const int32_t nel = maxel + 1;
  const size_t npair = (size_t)nvl * (size_t)std::max(nel, 1);
  const bool triples = npair * (size_t)nvl <= LABEL_TRIPLES_MAX;
  struct Blocks {
    std::vector<uint32_t> row, start, blk;  // blk: [keys + 1] first row of each block
    std::vector<uint32_t> ent;              // [keys + 1] first entry of each block
    std::vector<int32_t> nbr;
  };
  Blocks elb[2], elt[2];
  auto build_blocks = [&](int d, bool tri, Blocks& B) {
    const std::vector<uint32_t>& off = d ? lv_in_off : lv_out_off;
    const std::vector<int32_t>& nb = d ? lv_in_nbr : lv_out_nbr;
    const std::vector<int32_t>& lb = d ? lv_in_lab : lv_out_lab;
    const size_t nkeys = tri ? npair * (size_t)nvl : npair;
    std::vector<uint64_t> rows(nkeys + 1, 0), ents(nkeys + 1, 0);
    // a row's entries as (key within the bucket, neighbour), grouped by key with
    // the neighbour order kept within a key
    auto grouped = [&](uint32_t p, std::vector<std::pair<int64_t, int32_t>>& es) {
      es.clear();
      for (uint32_t e = off[p]; e < off[p + 1]; e++)
        es.push_back({tri ? (int64_t)lb[e] * nvl + vlabel[nb[e]] : (int64_t)lb[e], nb[e]});
      std::stable_sort(es.begin(), es.end(),
                       [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                         return x.first < y.first;
                       });
    };
    const size_t per_label = tri ? (size_t)nel * nvl : (size_t)nel;
    parallel_for(nvl, [&](int64_t l0, int64_t l1) {  // blocks of one vertex label are disjoint
      std::vector<std::pair<int64_t, int32_t>> es;
      for (int64_t L = l0; L < l1; L++)
        for (uint32_t p = lab_off[L]; p < lab_off[L + 1]; p++) {
          grouped(p, es);
          for (size_t i = 0; i < es.size(); i++) {
            const size_t b = (size_t)L * per_label + es[i].first;
            ents[b + 1]++;
            if (i == 0 || es[i].first != es[i - 1].first) rows[b + 1]++;
          }
        }
    });
    for (size_t b = 0; b < nkeys; b++) {
      rows[b + 1] += rows[b];
      ents[b + 1] += ents[b];
    }
    B.row.assign(rows[nkeys], 0);
    B.start.assign(rows[nkeys] + 1, 0);
    B.nbr.assign(ents[nkeys], 0);
    B.blk.assign(rows.begin(), rows.end());
    B.ent.assign(ents.begin(), ents.end());
    std::vector<uint64_t> rcur(rows.begin(), rows.end() - 1), ecur(ents.begin(), ents.end() - 1);
    parallel_for(nvl, [&](int64_t l0, int64_t l1) {
      std::vector<std::pair<int64_t, int32_t>> es;
      for (int64_t L = l0; L < l1; L++)
        for (uint32_t p = lab_off[L]; p < lab_off[L + 1]; p++) {
          grouped(p, es);
          for (size_t i = 0; i < es.size(); i++) {
            const size_t b = (size_t)L * per_label + es[i].first;
            if (i == 0 || es[i].first != es[i - 1].first) {
              const uint64_t r = rcur[b]++;
              B.row[r] = p - lab_off[L];
              B.start[r] = (uint32_t)ecur[b];
            }
            B.nbr[ecur[b]++] = es[i].second;
          }
        }
    });
    B.start[rows[nkeys]] = (uint32_t)ents[nkeys];
  };
  for (int d = 0; d < 2; d++) {
    build_blocks(d, false, elb[d]);
    if (triples) build_blocks(d, true, elt[d]);
  }
  std::vector<int32_t> attr_flat((size_t)num_attrs * n);
  for (int32_t a = 0; a < num_attrs; a++)
    std::memcpy(attr_flat.data() + (size_t)a * n, attr[a], sizeof(int32_t) * n);

  std::unique_ptr<gfd_graph> gp(new gfd_graph());
  gfd_graph* g = gp.get();
  {
    HIPCHK(hipGetDevice(&g->device));
    g->al.cb = lo.allocator;
    g->al.st = st;
    auto up = [&](const void* src, size_t bytes) -> void* {
      void* p = g->al.get(bytes);
      g->owned.push_back({p, std::max<size_t>(bytes, 1)});
      g->device_bytes += (int64_t)std::max<size_t>(bytes, 1);
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
    g->dg.lab_pos = (const uint32_t*)up(lab_pos.data(), 4 * n);
    g->dg.lv_out_off = (const uint32_t*)up(lv_out_off.data(), 4 * (n + 1));
    g->dg.lv_out_nbr = (const int32_t*)up(lv_out_nbr.data(), 4 * m);
    g->dg.lv_out_lab = (const int32_t*)up(lv_out_lab.data(), 4 * m);
    g->dg.lv_in_off = (const uint32_t*)up(lv_in_off.data(), 4 * (n + 1));
    g->dg.lv_in_nbr = (const int32_t*)up(lv_in_nbr.data(), 4 * m);
    g->dg.lv_in_lab = (const int32_t*)up(lv_in_lab.data(), 4 * m);
    g->dg.hub_off = (const uint64_t*)up(hub_off.data(), 8 * (n + 1));
    g->dg.hub_tab = (const uint8_t*)up(hub_tab.data(), hub_tab.size());
    g->dg.sym_off = (const uint64_t*)up(sym_off.data(), 8 * (n + 1));
    g->dg.sym_nbr = (const int32_t*)up(sym_nbr.data(), 4 * sym_nbr.size());
    g->dg.sym_lab = (const int2*)up(sym_lab.data(), 4 * sym_lab.size());
    for (int d = 0; d < 2; d++) {
      g->dg.elb_row[d] = (const uint32_t*)up(elb[d].row.data(), 4 * elb[d].row.size());
      g->dg.elb_start[d] = (const uint32_t*)up(elb[d].start.data(), 4 * elb[d].start.size());
      g->dg.elb_nbr[d] = (const int32_t*)up(elb[d].nbr.data(), 4 * elb[d].nbr.size());
      g->elb_blk[d] = std::move(elb[d].blk);
      g->elb_ent[d] = std::move(elb[d].ent);
      if (triples) {
        g->dg.elt_row[d] = (const uint32_t*)up(elt[d].row.data(), 4 * elt[d].row.size());
        g->dg.elt_start[d] = (const uint32_t*)up(elt[d].start.data(), 4 * elt[d].start.size());
        g->dg.elt_nbr[d] = (const int32_t*)up(elt[d].nbr.data(), 4 * elt[d].nbr.size());
        g->elt_blk[d] = std::move(elt[d].blk);
        g->elt_ent[d] = std::move(elt[d].ent);
      }
    }
    g->triples = triples;
    HIPCHK(hipStreamSynchronize(st));
    g->lab_off = std::move(lab_off);
    g->lab_out_sum = std::move(lab_out);
    g->lab_in_sum = std::move(lab_in);
  }
  *out = gp.release();
  return GFD_OK;
}

// Runs f, turning every exception into a status code and message: no C++
// exception crosses the C ABI.
template <class F>
static int32_t guarded(F f) {
  try {
    return f();
  } catch (const GfdError& e) {
    return set_error(e.code, "%s", e.msg.c_str());
  } catch (const std::bad_alloc&) {
    return set_error(GFD_ENOMEM, "host allocation failed");
  } catch (const std::length_error& e) {
    return set_error(GFD_ENOMEM, "host allocation too large: %s", e.what());
  } catch (const std::exception& e) {
    return set_error(GFD_EDEVICE, "unexpected failure: %s", e.what());
  } catch (...) {
    return set_error(GFD_EDEVICE, "unexpected failure");
  }
}

extern "C" int32_t gfd_load_graph(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                  const int32_t* vlabel, const int32_t* elabel, int32_t num_attrs,
                                  const int32_t* const* attr, const gfd_load_opts* opts,
                                  gfd_graph** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    return load_graph_impl(n, m, row_ptr, col, vlabel, elabel, num_attrs, attr, opts, out);
  });
}

extern "C" void gfd_free_graph(gfd_graph* g) {
  try {
    delete g;
  } catch (...) {
  }
}

extern "C" int32_t gfd_trim(gfd_graph* g) {
  if (!g) return set_error(GFD_EINVAL, "graph is NULL");
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->pool.size() != g->all.size()) return set_error(GFD_EINVAL, "a validate call is running");
    g->drop_workspaces();
    return GFD_OK;
  });
}

extern "C" int32_t gfd_get_graph_info(const gfd_graph* g, gfd_graph_info* info) {
  if (!g || !info) return set_error(GFD_EINVAL, "null argument");
  info->n = g->n; info->m = g->m; info->num_attrs = g->num_attrs;
  info->num_vertex_labels = g->nvl; info->num_edge_labels = g->nel;
  info->device_bytes = g->device_bytes;
  return GFD_OK;
}

extern "C" const char* gfd_last_error(void) { return g_last_error.c_str(); }
extern "C" int32_t gfd_version(void) { return 200; }

// ---------------------------------------------------------------------------
// planner (host): Section IV-B -- root, spanning tree, core-first order
// ---------------------------------------------------------------------------

struct Plan {
  int k = 0, root = 0;
  int32_t qlab[MAXK];
  int32_t qe[MAXK][MAXK];  // label of pattern edge a->b, ANY, or NOEDGE
  int bfs[MAXK], parent[MAXK], order[MAXK], pos[MAXK];
  bool virt[MAXK];  // the tree edge from parent[u] is virtual (u roots a further component)
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
  // leaf postponement (count-only calls): the last leaf_r vertices of the
  // matching order are counted, not enumerated; k_enum vertices are enumerated
  int leaf_r = 0, k_enum = 0, leaf_par = -1;
  int32_t lit_leaf[2 * MAXLIT];
  // two leaves under different parents (leaf_r == 2): order[k-2] (slot 0,
  // parent leaf_par2) and order[k-1] (slot 1, parent leaf_par)
  bool leaf_split = false;
  int leaf_par2 = -1;
  // a count-only call with K > 0: the one counted leaf's level is laid out
  // but deferred; after the counts, it runs over the first-K window only
  bool leaf_window = false;
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
  // a pattern of several connected components is allowed (Section IV-A):
  // its components are joined by a cross product in the enumeration
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
  for (int a = 0; a < k; a++) p.core[a] = alive[a];
  // connected components of the skeleton (a pattern may have several,
  // Section IV-A)
  int comp[MAXK];
  for (int a = 0; a < k; a++) comp[a] = -1;
  int ncomp = 0;
  for (int a = 0; a < k; a++) {
    if (comp[a] >= 0) continue;
    int st[MAXK], sp = 0;
    st[sp++] = a;
    comp[a] = ncomp;
    while (sp) {
      const int x = st[--sp];
      for (int b = 0; b < k; b++)
        if (adj[x][b] && comp[b] < 0) { comp[b] = ncomp; st[sp++] = b; }
    }
    ncomp++;
  }
  // a root per component: smallest estimated candidates per skeleton degree
  // among its core vertices (all its vertices when it is a tree, the root
  // then being its core); ties to the lower index.  Components go most
  // selective root first.
  int croot[MAXK];
  double cbest[MAXK];
  for (int cc = 0; cc < ncomp; cc++) {
    bool has_core = false;
    for (int a = 0; a < k; a++) has_core |= comp[a] == cc && p.core[a];
    cbest[cc] = 1e300;
    croot[cc] = -1;
    for (int a = 0; a < k; a++) {
      if (comp[a] != cc || (has_core && !p.core[a])) continue;
      const double c = (double)bucket_size(g, p.qlab[a]) / std::max(1, deg[a]);
      if (c < cbest[cc]) { cbest[cc] = c; croot[cc] = a; }
    }
    if (!has_core) p.core[croot[cc]] = true;
  }
  int corder[MAXK];
  for (int cc = 0; cc < ncomp; cc++) corder[cc] = cc;
  std::stable_sort(corder, corder + ncomp, [&](int x, int y) { return cbest[x] < cbest[y]; });
  p.root = croot[corder[0]];
  // BFS spanning tree of each component from its root, one after another; a
  // later component's root hangs from the first root by a virtual tree edge
  // (no pattern edge: its candidates are all of C(root'), the cross product)
  int head = 0, tail = 0;
  bool vis[MAXK] = {};
  for (int a = 0; a < k; a++) p.virt[a] = false;
  for (int ci = 0; ci < ncomp; ci++) {
    const int r = croot[corder[ci]];
    p.bfs[tail++] = r;
    vis[r] = true;
    p.parent[r] = ci == 0 ? -1 : p.root;
    p.virt[r] = ci > 0;
    while (head < tail) {
      int a = p.bfs[head++];
      for (int b = 0; b < k; b++)
        if (adj[a][b] && !vis[b]) { vis[b] = true; p.parent[b] = a; p.bfs[tail++] = b; }
    }
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
    if (p.virt[u]) {  // no CPI lists: the enumeration takes all of C(u)
      p.adj_dir[u] = 0;
      p.adj_prim[u] = ANY;
      p.adj_other[u] = PC_FREE;
      continue;
    }
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
  // probes per step: pairs that need an edge first (a random pair rarely has
  // one, so they reject most candidates), the absence-only pairs of the
  // induced reading after them (they rarely fail); the order only changes
  // how soon a conjunction stops
  p.nchk[0] = 0;
  for (int i = 1; i < k; i++) {
    int u = p.order[i], ppos = p.pos[p.parent[u]];
    p.nchk[i] = 0;
    for (int pass = 0; pass < 2; pass++)
      for (int j = 0; j < i; j++) {
        if (j == ppos && !p.virt[u]) continue;  // the CPI list holds that edge
        int w = p.order[j];
        int32_t f = pair_code(p, w, u, induced), b = pair_code(p, u, w, induced);
        if (f == PC_FREE && b == PC_FREE) continue;
        const bool needs_edge = (f != PC_FREE && f != PC_ABSENT) || (b != PC_FREE && b != PC_ABSENT);
        if (needs_edge != (pass == 0)) continue;
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
// driver: GFDs run in batches of jobs; every phase of a batch is one launch
// per kernel, whatever the number of jobs in it
// ---------------------------------------------------------------------------

enum { K_FILTER = 0, K_PULL = 1, K_CPI = 2, K_EXT = 3, K_LAST = 4, K_SCAN = 5, K_TOPK = 6, K_OTHER = 7 };

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

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Host-side capacities of one job.
struct JobCaps {
  uint64_t cap_u[MAXK];   // label bucket of u (items of its direct filters, position maps)
  uint64_t lcap_u[MAXK];  // bound on |C(u)| (list_cap): candidate lists, CPI heads
  uint64_t cap_f;   // frontier partial matches per level
  uint64_t pcap;    // largest scan (items) + 1
  uint64_t tiles;   // scan tile states
  uint64_t hits, begs, vcap;
  uint64_t hit_words, hit_cons;  // hit bitmaps: words per constraint, constraints
  uint64_t hit_region;           // words of the job's hit region (either layout)
  size_t bytes;     // region size (excluding control block, tile states, results)
};

struct JobMem {
  int32_t* pos[MAXK];
  uint32_t* bits[MAXK][2];
  int32_t* cand[MAXK][2];
  uint32_t* hits;
  uint64_t* P;
  uint32_t* cpi_beg[MAXK];
  uint32_t* cpi_len[MAXK];
  uint32_t* cpi_cur[MAXK];
  int32_t* cols[MAXK];
  uint32_t* begs;
  int32_t* vbuf;
  uint64_t* ctl;
  uint64_t* tstate;
  int32_t* res;
  uint32_t* leaf_cnt;  // leaf postponement: [|C(parent)| * LEAF_WORDS]
  uint32_t* leaf_cnt2;  // split leaves: the same for the other leaf's parent
};

struct Job {
  int spec;       // index of the GFD in the call
  Plan plan;
  JobCaps caps;
  JobMem mem;
  int cur[MAXK];  // which candidate buffer holds C(u) at the current step
  size_t last_rec = SIZE_MAX;  // offset of its last-level record in the batch's records
  bool last_single = false;    // that record is a single-vertex (k == 1) one
  size_t leaf_rec = SIZE_MAX;  // offset of its leaf-count record, if any
};

// A call's plans, capacities and batches, with what they depend on besides
// the graph: the GFDs and (reading, counts only, staging per job, budget,
// batch size).
struct PlanMemo {
  std::vector<gfd_spec> specs;
  uint64_t key[6] = {};
  std::vector<Job> all;
  std::vector<std::vector<int>> batches;
  double est = 0;  // frontier bytes estimated for the call's GFDs
};

// Data edges of the label block (bucket L, edge label e, far end's label
// far) in direction dir: an upper bound on the distinct far ends it holds.
static uint64_t block_entries(const gfd_graph* g, int32_t L, int32_t e, int32_t far, int dir) {
  if (L == ANY) return (uint64_t)g->m;
  if (L >= g->nvl) return 0;
  if (e == ANY) return dir ? g->lab_in_sum[L] : g->lab_out_sum[L];
  if (e >= g->nel) return 0;
  const size_t b = (size_t)L * g->nel + e;
  if (g->triples && far != ANY) {
    if (far >= g->nvl) return 0;
    const size_t t = b * g->nvl + far;
    return g->elt_ent[dir][t + 1] - g->elt_ent[dir][t];
  }
  return g->elb_ent[dir][b + 1] - g->elb_ent[dir][b];
}

// Upper bound on |C(u)| at every step: u's label bucket, and for each
// pattern edge to an earlier neighbour w in BFS order, the far ends of that
// edge's label block -- the top-down step keeps only vertices adjacent to a
// candidate of w through such an edge, and later steps only drop members.
static uint64_t list_cap(const gfd_graph* g, const Plan& p, int u) {
  uint64_t cap = bucket_size(g, p.qlab[u]);
  for (int w : p.down[u]) {
    if (p.qe[w][u] != NOEDGE) cap = std::min(cap, block_entries(g, p.qlab[w], p.qe[w][u], p.qlab[u], 0));
    if (p.qe[u][w] != NOEDGE) cap = std::min(cap, block_entries(g, p.qlab[w], p.qe[u][w], p.qlab[u], 1));
  }
  return cap;
}

static int pattern_edges_between(const Plan& p, int u, const std::vector<int>& nbrs) {
  int c = 0;
  for (int w : nbrs) c += (p.qe[w][u] != NOEDGE) + (p.qe[u][w] != NOEDGE);
  return c;
}

static uint64_t per_slot_bytes(int k) {
  uint64_t b = 12;  // prefix + list start of one source
  for (int i = 2; i < k; i++) b += 4ull * i;
  return b;
}

// frontiers: the job gets its own frontier columns of cap_f partial matches
// for every level (the bounded path); the fast path reserves its frontiers
// from the batch's pool instead, by the attempts each level counts.
static void job_caps(const gfd_graph* g, const Plan& p, uint64_t cap_f, uint64_t vcap, bool frontiers,
                     JobCaps& c) {
  const int k = p.k;
  uint64_t items = 1, hits = 1, cons = 1;
  for (int u = 0; u < k; u++) {
    c.cap_u[u] = bucket_size(g, p.qlab[u]);
    c.lcap_u[u] = list_cap(g, p, u);
    hits = std::max(hits, c.cap_u[u]);
    const uint64_t nc = (uint64_t)std::max(pattern_edges_between(p, u, p.down[u]),
                                           pattern_edges_between(p, u, p.up[u]));
    cons = std::max(cons, nc);
    items = std::max(items, c.lcap_u[u] * std::max<uint64_t>(nc, 1));
  }
  c.hit_words = hits / 32 + 1;
  c.hit_cons = cons;
  c.hit_region = cons * c.hit_words * 8;  // hit bytes (32 * hit_words per constraint) or bitmaps
  c.cap_f = (frontiers && k > 2) ? cap_f : 0;
  items = std::max(items, c.cap_f);
  c.pcap = items + 1;
  c.tiles = items / SCAN_TILE + 2;
  c.hits = hits;
  c.begs = std::max(c.cap_u[p.root], c.cap_f);
  c.vcap = vcap;
  size_t b = 0;
  for (int u = 0; u < k; u++)  // positions (parents), indexed by bucket position
    if (p.is_parent[u]) b += align_up(sizeof(int32_t) * std::max<size_t>(c.cap_u[u], 1));
  b += 2 * align_up(4 * ((size_t)g->n / 32 + 1)) * k;                  // membership bitmaps
  for (int u = 0; u < k; u++) b += 2 * align_up(4 * c.lcap_u[u]);      // candidate lists
  b += align_up(8 * c.pcap);
  for (int u = 0; u < k; u++)
    if (u != p.root) b += 3 * align_up(4 * c.lcap_u[p.parent[u]]);   // CPI list heads
  for (int i = 2; i < k; i++) b += align_up(4ull * i * c.cap_f);      // frontier columns
  b += align_up(4 * c.begs);
  b += align_up(4 * c.vcap * k);
  if (p.leaf_r) b += align_up(4ull * LEAF_WORDS * c.lcap_u[p.leaf_par]);
  if (p.leaf_split) b += align_up(4ull * LEAF_WORDS * c.lcap_u[p.leaf_par2]);
  c.bytes = b;
}

static void job_layout(uint8_t* base, const gfd_graph* g, const Plan& p, const JobCaps& c,
                       JobMem& m) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* q = base + off;
    off += align_up(bytes);
    return q;
  };
  const int k = p.k;
  std::memset(&m.pos, 0, sizeof m.pos);
  // position maps are read only through the CPI lists of tree children
  for (int u = 0; u < k; u++)
    m.pos[u] = p.is_parent[u] ? (int32_t*)take(sizeof(int32_t) * std::max<size_t>(c.cap_u[u], 1)) : nullptr;
  for (int u = 0; u < k; u++) {
    m.bits[u][0] = (uint32_t*)take(4 * ((size_t)g->n / 32 + 1));
    m.bits[u][1] = (uint32_t*)take(4 * ((size_t)g->n / 32 + 1));
  }
  for (int u = 0; u < k; u++) {
    m.cand[u][0] = (int32_t*)take(4 * c.lcap_u[u]);
    m.cand[u][1] = (int32_t*)take(4 * c.lcap_u[u]);
  }
  m.P = (uint64_t*)take(8 * c.pcap);
  for (int u = 0; u < k; u++) {
    m.cpi_beg[u] = m.cpi_len[u] = m.cpi_cur[u] = nullptr;
    if (u == p.root) continue;
    const uint64_t cp = c.lcap_u[p.parent[u]];
    m.cpi_beg[u] = (uint32_t*)take(4 * cp);
    m.cpi_len[u] = (uint32_t*)take(4 * cp);
    m.cpi_cur[u] = (uint32_t*)take(4 * cp);
  }
  for (int i = 0; i < MAXK; i++) m.cols[i] = nullptr;
  for (int i = 2; i < k; i++) m.cols[i] = (int32_t*)take(4ull * i * c.cap_f);
  m.begs = (uint32_t*)take(4 * c.begs);
  m.vbuf = (int32_t*)take(4 * c.vcap * k);
  m.leaf_cnt = p.leaf_r ? (uint32_t*)take(4ull * LEAF_WORDS * c.lcap_u[p.leaf_par]) : nullptr;
  m.leaf_cnt2 = p.leaf_split ? (uint32_t*)take(4ull * LEAF_WORDS * c.lcap_u[p.leaf_par2]) : nullptr;
}

struct Ctx {
  const gfd_graph* g;
  Workspace* ws;
  hipStream_t st;
  bool induced;
  int K;
  uint64_t front_limit;  // testing: at most this many partial matches per level (0: none)
  Timer tm;
  gfd_stats* stats;
  unsigned long long* stat_bytes;  // device [8] per kernel class, or nullptr
  uint8_t* recbase = nullptr;  // device records the launches read (nullptr: ws->jobrec)
  gfd_tuning tune{};           // launch shapes (0: defaults)
};


static unsigned long long* cls_bytes(Ctx& c, int cls) {
  return c.stat_bytes ? c.stat_bytes + cls : nullptr;
}

static uint32_t next_epoch(Ctx& c) {
  c.ws->epoch = (c.ws->epoch + 1) & 0xFFFFu;
  if (c.ws->epoch == 0) c.ws->epoch = 1;
  return c.ws->epoch;
}

static CandSet cand_set(const Job& J, int u) {
  return CandSet{J.mem.cand[u][J.cur[u]], J.mem.ctl + CTL_CAND + 2 * u + J.cur[u], J.mem.pos[u],
                 J.mem.bits[u][J.cur[u]], J.plan.qlab[u] != ANY ? 1 : 0};
}

// The level of u when u roots a further component: its attempts are all of
// C(u) for every source.
static void set_cross(const Job& J, int u, ExtJob& e) {
  if (!J.plan.virt[u]) return;
  const CandSet cs = cand_set(J, u);
  e.cross = 1;
  e.cpi_ent = cs.list;
  e.cross_n = cs.cnt;
  e.cross_cap = J.caps.lcap_u[u];
}

static JobScan job_scan_rec(Ctx& c, const Job& J, uint64_t* d_total, uint32_t epoch) {
  return JobScan{J.mem.P, d_total, J.mem.tstate, (uint32_t*)(J.mem.ctl + CTL_TICKET), c.ws->err,
                 epoch};
}

static void add_pulls(const Job& J, int u, const std::vector<int>& nbrs, FilterJob& f) {
  const Plan& p = J.plan;
  f.ncons = 0;
  for (int w : nbrs) {
    if (p.qe[w][u] != NOEDGE)  // w -> u: v needs an in-neighbour in C(w)
      f.cons[f.ncons++] = PullC{1, p.qe[w][u], cand_set(J, w), 0, 0, 0, p.qlab[w]};
    if (p.qe[u][w] != NOEDGE)  // u -> w: v needs an out-neighbour in C(w)
      f.cons[f.ncons++] = PullC{0, p.qe[u][w], cand_set(J, w), 0, 0, 0, p.qlab[w]};
  }
}

// The edge-label block of bucket L's rows in direction dir for edge label e
// (both labelled): keyed by the far end's label too when that label is known
// (far labels ANY or absent from the graph keep the pair block).
static void set_block(const gfd_graph* g, int32_t L, int32_t e, int32_t far, int32_t dir,
                      int32_t& blk, uint32_t& rb, uint32_t& re) {
  const size_t b = (size_t)L * g->nel + e;
  if (g->triples && far != ANY && far < g->nvl) {
    const size_t t = b * g->nvl + far;
    blk = 2;
    rb = g->elt_blk[dir][t];
    re = g->elt_blk[dir][t + 1];
  } else {
    blk = 1;
    rb = g->elb_blk[dir][b];
    re = g->elb_blk[dir][b + 1];
  }
}

// A filter over the whole bucket of u (all of V for a wildcard): consecutive
// rows of the label-ordered view, each labelled constraint read from its
// edge-label block.
static void make_direct(const gfd_graph* g, const Plan& p, int u, uint64_t bs, FilterJob& f) {
  f.base = (p.qlab[u] == ANY || bs == 0) ? 0u : g->lab_off[p.qlab[u]];
  f.list = p.qlab[u] == ANY ? nullptr : g->dg.lab_vtx + f.base;
  f.direct = 1;
  f.d_n = nullptr;
  f.n_host = f.cap = bs;
  for (int q = 0; q < f.ncons; q++) {
    PullC& pc = f.cons[q];
    pc.blk = 0;
    if (p.qlab[u] == ANY || pc.elab == ANY || p.qlab[u] >= g->nvl || pc.elab >= g->nel) continue;
    set_block(g, p.qlab[u], pc.elab, pc.nlab, pc.dir, pc.blk, pc.rb, pc.re);
  }
}

static int gx_for(uint64_t items, int njobs, int cap = 256) {
  const uint64_t want = (items + BS - 1) / BS;
  const int per_job = std::max(8, std::min(cap, 4096 / std::max(1, njobs)));
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)per_job));
}
// 1-D grid of a flat (load-balanced) launch whose jobs together have at most
// `chunks` chunks of LBS_CHUNK positions: enough blocks to fill the chip.
constexpr uint64_t FLAT_GRID_MAX = 2048;
static uint64_t chunks_of(uint64_t positions) { return (positions + LBS_CHUNK - 1) / LBS_CHUNK; }
// A grid of at least NXCD blocks is rounded up to a multiple of NXCD (the
// kernels then give each die a contiguous slice of the chunks).
// Whether the last level loads its first probes ahead: when the graph fits
// the 256 MB last-level cache (MALL) with room to spare, the level waits on
// instruction issue and cache latency, and eight probes in flight per thread
// beat the extra wave per SIMD that the plain form keeps (5% on the
// 20K-vertex Twitch-shaped graph); on graphs that live in HBM the extra wave
// wins (2% on the 4M/20M graph).
constexpr int64_t PROBE_AHEAD_MAX_BYTES = int64_t(128) << 20;
static bool probe_ahead(const gfd_graph* g) { return g->device_bytes <= PROBE_AHEAD_MAX_BYTES; }

// Launch shapes of the enumeration (tuned or default).
static uint64_t enum_grid(const Ctx& c) { return c.tune.flat_grid ? (uint64_t)c.tune.flat_grid : FLAT_GRID_MAX; }
static int enum_scan_grid(const Ctx& c) { return c.tune.scan_grid ? c.tune.scan_grid : (int)FLAT_GRID_MAX; }
static bool use_ahead(const Ctx& c) {
  return c.tune.probe_ahead == 1 || (c.tune.probe_ahead == 0 && probe_ahead(c.g));
}
// Enumeration kernels limited to 64 VGPRs (8 waves per SIMD): by default for
// graphs too large to stay in cache, where the last level waits on HBM.
static bool use_occ8(const Ctx& c) {
  return c.tune.ext_occupancy == 2 || (c.tune.ext_occupancy == 0 && !probe_ahead(c.g));
}

static int flat_grid(uint64_t chunks, uint64_t cap = FLAT_GRID_MAX) {
  uint64_t g = std::max<uint64_t>(1, std::min<uint64_t>(chunks, cap));
  if (g >= (uint64_t)NXCD) g = std::min<uint64_t>((g + NXCD - 1) / NXCD * NXCD, cap);
  return (int)g;
}
// 1-D grid of a level scan whose njobs jobs have at most max_items sources
// each: the blocks are shared among the jobs by their tiles.
static int scan_grid(int njobs, uint64_t max_items) {
  const uint64_t t = (max_items + SCAN_TILE - 1) / SCAN_TILE;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)std::max(njobs, 1) * std::max<uint64_t>(t, 1),
                                                       FLAT_GRID_MAX));
}

static uint64_t rows_ub(const gfd_graph* g, int32_t L, int dir) {
  if (L == ANY) return (uint64_t)g->m;
  if (L >= g->nvl) return 0;
  return dir ? g->lab_in_sum[L] : g->lab_out_sum[L];
}

// Estimated frontier-pool bytes of one job's fast enumeration: the level-i
// reservation takes (attempts of level i) slots, and attempts are estimated
// level by level as sources times the tree edge's mean fan-out -- the data
// edges from the parent's label bucket with the edge's label and direction
// and the child's label, over the bucket's size.  Non-tree checks and
// injectivity are ignored, so inner levels are over-estimated, while skewed
// degrees can make real fan-outs larger than the mean: the estimate sizes the
// pool of a fresh workspace and serving admission, and the pool still grows
// to what batches ask for.
static double fan_out(const gfd_graph* g, int32_t L, int32_t e, int32_t far, int dir) {
  const double nb = (double)std::max<uint64_t>(1, L == ANY ? (uint64_t)g->n
                                                   : (L < g->nvl ? g->lab_off[L + 1] - g->lab_off[L] : 0));
  if (L == ANY || L >= g->nvl) return (double)g->m / std::max<int64_t>(1, g->n);
  if (e == ANY || e >= g->nel) return (double)rows_ub(g, L, dir) / nb;
  const size_t b = (size_t)L * g->nel + e;
  if (g->triples && far != ANY && far < g->nvl) {
    const size_t t = b * g->nvl + far;
    return (double)(g->elt_ent[dir][t + 1] - g->elt_ent[dir][t]) / nb;
  }
  return (double)(g->elb_ent[dir][b + 1] - g->elb_ent[dir][b]) / nb;
}
static uint64_t est_front_bytes(const gfd_graph* g, const Plan& p) {
  double N = (double)bucket_size(g, p.qlab[p.root]), bytes = 0;
  for (int i = 1; i < p.k_enum; i++) {
    const int u = p.order[i], q = p.parent[u];
    const double T = N * (p.virt[u] ? (double)bucket_size(g, p.qlab[u])
                                     : fan_out(g, p.qlab[q], p.adj_prim[u], p.qlab[u], p.adj_dir[u]));
    const bool last = p.leaf_r == 0 && i == p.k - 1;
    if (!last) bytes += T * (4.0 * (i + 1) + 12.0) + 1024.0;
    N = T;
  }
  return (uint64_t)std::min(bytes, 1e18);
}

// Frontier bytes a job whose frontiers overflowed the pool asks for, from its
// control words: each inner level's attempts (known for every level it
// reached, the failed one included) sized as the device's reservation sizes
// them. A level past the failed one was not reached; the levels not reached
// are counted as much again as those reached.
static uint64_t reached_front_bytes(const Plan& p, const uint64_t* h, uint64_t front_limit) {
  auto al = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
  uint64_t bytes = 0;
  bool short_of = false;
  for (int i = 1; i < p.k_enum; i++) {
    if (p.leaf_r == 0 && i == p.k - 1) break;  // the last level keeps no frontier
    uint64_t T = h[CTL_LEVEL_T + i];
    if (!T) {
      short_of = true;
      continue;
    }
    if (front_limit && T > front_limit) T = front_limit;
    bytes += al(4ull * (uint64_t)(i + 1) * T) + al(8ull * (T + 1)) + al(4ull * T + 4) +
             al(8ull * (T / SCAN_TILE + 2));
  }
  return short_of ? 2 * bytes : bytes;
}

// Job records of every step of a batch, staged host side and uploaded once.
struct Recs {
  std::vector<uint8_t> blob;
  template <class T>
  size_t add(const std::vector<T>& v) {
    size_t off = align_up(blob.size());
    blob.resize(off + sizeof(T) * v.size());
    std::memcpy(blob.data() + off, v.data(), sizeof(T) * v.size());
    return off;
  }
};

// Grows the record buffers; the caller has synchronised its stream, since a
// copy kernel still in flight may be reading the old host staging.
static void ensure_recs(Workspace* ws, size_t bytes) {
  if (ws->jobrec_bytes < bytes) {
    dfree(ws->al, ws->jobrec, ws->jobrec_bytes);
    ws->jobrec_bytes = 0;
    ws->jobrec = dalloc<uint8_t>(ws->al, bytes);
    ws->jobrec_bytes = bytes;
  }
  if (ws->hjobrec_bytes < bytes) {
    ws->host_put(ws->hjobrec);
    ws->hjobrec = nullptr;
    ws->hjobrec_bytes = 0;
    ws->hjobrec_dev = nullptr;
    ws->hjobrec = (uint8_t*)ws->host_get(bytes, true);
    ws->hjobrec_bytes = bytes;
    ws->hjobrec_dev = ws->pageable ? nullptr : mapped_ptr(ws->hjobrec);
  }
}

// Small host-to-device upload of staged records on the call's stream.  A copy
// kernel that reads the mapped pinned staging keeps the upload on the compute
// queue: a DMA copy between kernels costs a hand-off between engines of about
// 20 us each time, and a batch uploads records before most of its phases.
static void upload(Ctx& c, void* dst, const void* hsrc, const uint8_t* hsrc_dev, size_t bytes) {
  if (bytes == 0) return;
  const uintptr_t h = (uintptr_t)hsrc, d = (uintptr_t)dst;
  if (hsrc_dev && (h % 8) == 0 && (d % 8) == 0 && (bytes % 8) == 0 && bytes <= (size_t(1) << 20)) {
    copy_words(c.st, (const uint64_t*)hsrc_dev, (uint64_t*)dst, bytes / 8);
    return;
  }
  HIPCHK(hipMemcpyAsync(dst, hsrc, bytes, hipMemcpyHostToDevice, c.st));
}
static void upload_recs(Ctx& c, size_t off, size_t bytes) {
  upload(c, c.ws->jobrec + off, c.ws->hjobrec + off, c.ws->hjobrec_dev ? c.ws->hjobrec_dev + off : nullptr,
         bytes);
}

// Phase plan of a batch: which kernels run, on which record arrays.
struct Launch {
  int kind;     // 0 filter, 1 cpi, 2 ext, 3 single, 4 topk, 5 leaf counts
  size_t off;   // record array offset
  int njobs;
  int gx_scan, gx_work, gx_item, gx_clear;
  bool scan, last_any, inner_any;
  bool row_scan = false;  // filter: some job's pull needs the (item, constraint) row scan
  bool hit_bitmaps = false;  // filter: the jobs record hits in bitmaps (top-down steps)
  bool cpi_two_pass = false;  // CPI: count kept entries first (the bounded path)
  size_t next_off = SIZE_MAX;  // enumeration: the next level's records (frontier reservation)
  size_t leaf_off = SIZE_MAX;  // enumeration: the leaf-count records, if any
  size_t prep2_off = SIZE_MAX; // leaf counts: the records that fill split leaves' second tables
};

// The launches of a batch in order.  When on_add is set (the fast path), it
// runs as each launch is appended, so the GPU starts on the first filter step
// while the host still builds the records of later ones.
struct LaunchList {
  std::vector<Launch> v;
  std::function<void(const Launch&)> on_add;
  void push_back(const Launch& l) {
    v.push_back(l);
    if (on_add) on_add(l);
  }
};

// Builds every record of the CPI construction and the fast enumeration of
// `jobs` (Section IV-B steps 1 and 2) into `R` and the launch list `L`.
static void plan_batch(Ctx& c, std::vector<Job>& jobs, Recs& R, LaunchList& L,
                       bool fast_enum) {
  const gfd_graph* g = c.g;
  const int nj = (int)jobs.size();
  int maxk = 0;
  for (auto& J : jobs) {
    maxk = std::max(maxk, J.plan.k);
    for (int u = 0; u < MAXK; u++) J.cur[u] = 0;
  }
  // top-down, BFS order
  for (int j = 0; j < maxk; j++) {
    std::vector<FilterJob> F(nj);
    uint64_t items = 1, pull_ub = 0, pairs = 1, item_ch = 0;  // *_ub, *_ch: chunks over all jobs
    bool any_cons = false;
    const uint32_t ep = next_epoch(c);
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      const Plan& p = J.plan;
      FilterJob& f = F[x];
      f = FilterJob{};
      if (j >= p.k) continue;
      const int u = p.bfs[j];
      f.active = 1;
      add_pulls(J, u, p.down[u], f);
      f.min_out = p.min_out[u];
      f.min_in = p.min_in[u];
      const uint64_t bs = J.caps.cap_u[u];
      // top-down items: the whole bucket
      make_direct(g, p, u, bs, f);
      f.hits = J.mem.hits;
      f.hit_words = J.caps.hit_words;
      f.hitmode = 1;  // top-down: few items meet a constraint (settled per launch below)
      f.sc = job_scan_rec(c, J, J.mem.ctl + CTL_TOTAL, ep);
      J.cur[u] = 0;
      f.out = J.mem.cand[u][0];
      f.out_cap = J.caps.lcap_u[u];
      f.d_out_n = J.mem.ctl + CTL_CAND + 2 * u;
      f.pos = J.mem.pos[u];
      f.pos_by_bucket = p.qlab[u] != ANY ? 1 : 0;
      f.bits = J.mem.bits[u][0];
      f.nwords = (uint64_t)g->n / 32 + 1;
      items = std::max(items, bs);
      pairs = std::max(pairs, bs * (uint64_t)std::max(f.ncons, 1));
      for (int q = 0; q < f.ncons; q++) pull_ub += chunks_of(rows_ub(g, p.qlab[u], f.cons[q].dir));
      any_cons |= f.ncons > 0;
    }
    // bitmaps when every active job has a constraint (all but the roots' step)
    bool all_cons = true;
    for (const FilterJob& f : F) all_cons &= !f.active || f.ncons > 0;
    item_ch = 0;
    for (int x = 0; x < nj; x++) {
      FilterJob& f = F[x];
      f.hitmode = all_cons ? 1 : 0;
      if (f.active)
        item_ch += all_cons ? (f.n_host + 32ull * BS - 1) / (32ull * BS) : chunks_of(f.n_host);
    }
    L.push_back(Launch{0, R.add(F), nj, scan_grid(nj, pairs), flat_grid(pull_ub), flat_grid(item_ch),
                       gx_for((uint64_t)g->n / 32 + 1, nj, 64), any_cons, false, false, false,
                       all_cons});
  }
  // bottom-up, reverse BFS order: drop dead ends
  for (int j = maxk - 1; j >= 0; j--) {
    std::vector<FilterJob> F(nj);
    uint64_t items = 1, pull_ub = 0, pairs = 1, item_ch = 0;  // *_ub, *_ch: chunks over all jobs
    bool any = false, row_scan = false;
    const uint32_t ep = next_epoch(c);
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      const Plan& p = J.plan;
      FilterJob& f = F[x];
      f = FilterJob{};
      if (j >= p.k) continue;
      const int u = p.bfs[j];
      if (p.up[u].empty()) continue;
      f.active = 1;
      add_pulls(J, u, p.up[u], f);
      const CandSet cur = cand_set(J, u);
      if (p.down[u].empty()) {
        // C(u) is its bucket less the degree filter (no top-down constraint):
        // stream the bucket directly and keep the current members
        make_direct(g, p, u, J.caps.cap_u[u], f);
        f.keep = cur.bits;
      } else {
        f.list = cur.list;
        f.d_n = cur.cnt;
        f.cap = J.caps.lcap_u[u];
        // labelled constraints read the item's run in the edge-label block
        for (int q = 0; q < f.ncons; q++) {
          PullC& pc = f.cons[q];
          if (p.qlab[u] != ANY && pc.elab != ANY && p.qlab[u] < g->nvl && pc.elab < g->nel)
            set_block(g, p.qlab[u], pc.elab, pc.nlab, pc.dir, pc.blk, pc.rb, pc.re);
        }
      }
      f.hits = J.mem.hits;
      f.hit_words = J.caps.hit_words;
      f.hitmode = 0;  // bottom-up: most current members meet their constraints
      f.sc = job_scan_rec(c, J, J.mem.ctl + CTL_TOTAL, ep);
      J.cur[u] ^= 1;
      f.out = J.mem.cand[u][J.cur[u]];
      f.out_cap = J.caps.lcap_u[u];
      f.d_out_n = J.mem.ctl + CTL_CAND + 2 * u + J.cur[u];
      f.pos = J.mem.pos[u];
      f.pos_by_bucket = p.qlab[u] != ANY ? 1 : 0;
      f.bits = J.mem.bits[u][J.cur[u]];
      f.nwords = (uint64_t)g->n / 32 + 1;
      items = std::max(items, f.cap);
      item_ch += chunks_of(f.cap);
      row_scan |= !f.direct && f.ncons > 0;
      pairs = std::max(pairs, f.cap * (uint64_t)f.ncons);
      for (int q = 0; q < f.ncons; q++) pull_ub += chunks_of(rows_ub(g, p.qlab[u], f.cons[q].dir));
      any = true;
    }
    if (any)
      L.push_back(Launch{0, R.add(F), nj, scan_grid(nj, pairs), flat_grid(pull_ub), flat_grid(item_ch),
                         gx_for((uint64_t)g->n / 32 + 1, nj, 64), true, false, false, row_scan});
  }
  // CPI adjacency lists per spanning-tree edge, in BFS order
  for (int j = 1; j < maxk; j++) {
    std::vector<CpiJob> C(nj);
    uint64_t items = 1, rows = 0;  // rows: chunks over all jobs
    bool any = false;
    const uint32_t ep = next_epoch(c);
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      const Plan& p = J.plan;
      CpiJob& a = C[x];
      a = CpiJob{};
      if (j >= p.k) continue;
      const int u = p.bfs[j], q = p.parent[u];
      if (p.virt[u]) continue;  // a further component's root: no CPI lists
      a.active = 1;
      a.dir = p.adj_dir[u];
      a.prim = p.adj_prim[u];
      a.other = p.adj_other[u];
      a.p = cand_set(J, q);
      a.u = cand_set(J, u);
      a.cap_p = J.caps.lcap_u[q];
      a.beg = J.mem.cpi_beg[u];
      a.len = J.mem.cpi_len[u];
      a.cur = J.mem.cpi_cur[u];
      a.d_base = J.mem.ctl + CTL_CPIBASE;
      a.d_asked = J.mem.ctl + CTL_CPIASK;
      a.arena = c.ws->cpi_arena;
      a.arena_cursor = c.ws->misc;
      a.arena_cap = cpi_usable(c.ws);
      a.flags = (uint32_t*)(J.mem.ctl + CTL_FLAGS);
      a.sc = job_scan_rec(c, J, J.mem.ctl + CTL_TOTAL, ep);
      a.blk = 0;
      if (p.qlab[q] != ANY && a.prim != ANY && p.qlab[q] < g->nvl && a.prim < g->nel) {
        set_block(g, p.qlab[q], a.prim, p.qlab[u], a.dir, a.blk, a.rb, a.re);
        a.base = g->lab_off[p.qlab[q]];
      }
      items = std::max(items, a.cap_p);
      rows += chunks_of(rows_ub(g, p.qlab[q], a.dir));
      any = true;
    }
    if (any)
      L.push_back(Launch{1, R.add(C), nj, scan_grid(nj, items), flat_grid(rows), gx_for(items, nj), 0,
                         true, false, false, false, false, !fast_enum});
  }
  if (!fast_enum) return;
  // enumeration levels (core-first matching order) with the fused check.
  // Every level's records (and the leaf counts') are built and added before
  // the first level is enqueued: an inner level's frontier reservation
  // writes the next level's records on the device.
  std::vector<std::vector<ExtJob>> E(maxk);
  std::vector<LeafJob> F(nj), F2(nj);
  bool any_leaf = false, any_split = false;
  uint64_t leaf_np = 1;
  for (int i = 1; i < maxk; i++) {
    E[i].resize(nj);
    const uint32_t ep = next_epoch(c);
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      const Plan& p = J.plan;
      ExtJob& e = E[i][x];
      e = ExtJob{};
      // postponed leaves are counted, not enumerated; a window job keeps its
      // last level's record, deferred
      const bool deferred = p.leaf_window && i == p.k - 1;
      if (i >= p.k_enum && !deferred) continue;
      const int u = p.order[i], q = p.parent[u];
      e.active = 1;
      e.deferred = deferred ? 1 : 0;
      e.i = i;
      e.k = p.k;
      e.last = (p.leaf_r == 0 || deferred) && i == p.k - 1;
      e.begs = J.mem.begs;
      e.sc = job_scan_rec(c, J, J.mem.ctl + CTL_LEVEL_T + i, ep);
      e.home_P = J.mem.P;
      if (i == 1) {
        const CandSet r = cand_set(J, p.root);
        e.src_cols = r.list;
        e.src_stride = 0;
        e.d_nsrc = r.cnt;
        e.src_cap = J.caps.lcap_u[p.root];
      } else {
        // the previous level's reservation points src_*, begs and the scan's
        // prefix and tile states at its pool slots; until then (and if the
        // pool could not hold it) the level has no sources and its scan
        // writes only its zero total into the job's own arrays
        e.src_cols = J.mem.cand[p.root][0];
        e.src_stride = 0;
        e.d_nsrc = J.mem.ctl + CTL_LEVEL_N + i;
        e.src_cap = 0;
      }
      e.par_pos = p.pos[q];
      e.par_posmap = J.mem.pos[q];
      e.par_by_bucket = p.qlab[q] != ANY ? 1 : 0;
      e.cpi_beg = J.mem.cpi_beg[u];
      e.cpi_len = J.mem.cpi_len[u];
      e.cpi_ent = c.ws->cpi_arena;
      set_cross(J, u, e);
      e.a_begin = 0;
      e.a_end = ~0ull;
      e.nchk = p.nchk[i];
      for (int t = 0; t < MAXK; t++) {
        e.chk_pos[t] = t < p.nchk[i] ? p.chk_pos[i][t] : 0;
        e.chk_fwd[t] = t < p.nchk[i] ? p.chk_fwd[i][t] : PC_FREE;
        e.chk_bwd[t] = t < p.nchk[i] ? p.chk_bwd[i][t] : PC_FREE;
      }
      if (!e.last) {  // dst_* come from the reservation
        e.front_limit = c.front_limit;
        e.d_ndst = J.mem.ctl + CTL_LEVEL_N + i + 1;
      }
      e.flags = (uint32_t*)(J.mem.ctl + CTL_FLAGS);
      for (int v = 0; v < MAXK; v++) e.var_pos[v] = v < p.k ? p.pos[v] : 0;
      e.nx = p.nx;
      e.ny = p.ny;
      e.y_false = p.y_false;
      for (int t = 0; t < 2 * MAXLIT; t++) e.lit[t] = p.lit[t];
      e.counters = (unsigned long long*)(J.mem.ctl + CTL_MATCH);
      e.vbuf = J.mem.vbuf;
      e.d_vcount = J.mem.ctl + CTL_VCOUNT;
      e.vcap = c.K > 0 ? J.caps.vcap : 0;
      e.thr = nullptr;
      e.d_thr_valid = (const uint32_t*)(J.mem.ctl + CTL_THRVALID);
    }
  }
  // postponed leaves: completions counted per partial match of the inner part
  for (int x = 0; x < nj; x++) {
    Job& J = jobs[x];
    const Plan& p = J.plan;
    LeafJob& f = F[x];
    f = LeafJob{};
    if (!p.leaf_r) continue;
    const int u0 = p.order[p.k - 1], q = p.leaf_par;
    f.active = 1;
    f.i = p.k_enum;
    f.r = p.leaf_r;
    if (p.k_enum == 1) {
      const CandSet r = cand_set(J, p.root);
      f.src_cols = r.list;
      f.src_stride = 0;
      f.d_nsrc = r.cnt;
      f.src_cap = J.caps.lcap_u[p.root];
    } else {  // the last inner level's reservation sets src_*
      f.src_cols = J.mem.cand[p.root][0];
      f.src_stride = 0;
      f.d_nsrc = J.mem.ctl + CTL_LEVEL_N + p.k_enum;
      f.src_cap = 0;
    }
    f.par_pos = p.pos[q];
    f.par_posmap = J.mem.pos[q];
    f.par_by_bucket = p.qlab[q] != ANY ? 1 : 0;
    const CandSet pc = cand_set(J, q);
    f.d_np = pc.cnt;
    f.cap_p = J.caps.lcap_u[q];
    f.cpi_beg = J.mem.cpi_beg[u0];
    f.cpi_len = J.mem.cpi_len[u0];
    f.cpi_ent = c.ws->cpi_arena;
    f.u = cand_set(J, u0);
    f.dir = p.adj_dir[u0];
    f.prim = p.adj_prim[u0];
    f.other = p.adj_other[u0];
    f.cnt = J.mem.leaf_cnt;
    f.nx = p.nx;
    f.ny = p.ny;
    f.y_false = p.y_false;
    for (int t = 0; t < 2 * MAXLIT; t++) {
      f.lit[t] = p.lit[t];
      f.lit_leaf[t] = p.lit_leaf[t];
    }
    f.counters = (unsigned long long*)(J.mem.ctl + CTL_MATCH);
    f.flags = (uint32_t*)(J.mem.ctl + CTL_FLAGS);
    leaf_np = std::max(leaf_np, f.cap_p);
    any_leaf = true;
    if (p.leaf_split) {
      // this record counts the last leaf (slot 1 of the plan) as a leaf of its
      // own; F2 fills the table of the other (slot 0) under its parent
      const int ua = p.order[p.k - 2], q2 = p.leaf_par2;
      f.r = 1;
      for (int t = 0; t < 2 * MAXLIT; t++) {
        f.lit_leaf[t] = p.lit_leaf[t] == 1 ? 0 : -1;
        f.lit_leaf2[t] = p.lit_leaf[t] == 0 ? 0 : -1;
      }
      f.split = 1;
      const int ub = p.order[p.k - 1];
      f.split_overlap = p.qlab[ua] == ANY || p.qlab[ub] == ANY || p.qlab[ua] == p.qlab[ub];
      f.par2_pos = p.pos[q2];
      f.par2_posmap = J.mem.pos[q2];
      f.par2_by_bucket = p.qlab[q2] != ANY ? 1 : 0;
      f.cpi2_beg = J.mem.cpi_beg[ua];
      f.cpi2_len = J.mem.cpi_len[ua];
      f.u2 = cand_set(J, ua);
      f.dir2 = p.adj_dir[ua];
      f.prim2 = p.adj_prim[ua];
      f.other2 = p.adj_other[ua];
      f.cnt2 = J.mem.leaf_cnt2;
      LeafJob& f2 = F2[x];
      f2 = LeafJob{};
      f2.active = 1;
      f2.i = f.i;
      f2.r = 1;
      const CandSet pc2 = cand_set(J, q2);
      f2.d_np = pc2.cnt;
      f2.cap_p = J.caps.lcap_u[q2];
      f2.cpi_beg = J.mem.cpi_beg[ua];
      f2.cpi_len = J.mem.cpi_len[ua];
      f2.cpi_ent = c.ws->cpi_arena;
      f2.u = f.u2;
      f2.cnt = J.mem.leaf_cnt2;
      f2.nx = p.nx;
      f2.ny = p.ny;
      f2.y_false = p.y_false;
      for (int t = 0; t < 2 * MAXLIT; t++) {
        f2.lit[t] = p.lit[t];
        f2.lit_leaf[t] = f.lit_leaf2[t];
      }
      leaf_np = std::max(leaf_np, f2.cap_p);
      any_split = true;
    }
  }
  std::vector<size_t> eoff(maxk, SIZE_MAX);
  for (int i = 1; i < maxk; i++) eoff[i] = R.add(E[i]);
  const size_t leaf_off = any_leaf ? R.add(F) : SIZE_MAX;
  const size_t prep2_off = any_split ? R.add(F2) : SIZE_MAX;
  if (any_leaf)
    for (int x = 0; x < nj; x++)
      if (F[x].active) jobs[x].leaf_rec = leaf_off + sizeof(LeafJob) * x;
  for (int i = 1; i < maxk; i++) {
    bool any_last = false, any_inner = false;
    for (int x = 0; x < nj; x++) {
      const ExtJob& e = E[i][x];
      if (!e.active) continue;
      if (e.last) jobs[x].last_rec = eoff[i] + sizeof(ExtJob) * x;
      if (e.deferred) continue;  // runs after the main pass, over its window
      any_last |= e.last != 0;
      any_inner |= e.last == 0;
    }
    // level 1's sources are the roots' candidates; deeper levels' sizes are
    // known only on the device, so their scans get the full grid
    uint64_t srcs = i == 1 ? 1 : ~0ull;
    if (i == 1)
      for (int x = 0; x < nj; x++)
        if (E[i][x].active) srcs = std::max(srcs, E[i][x].src_cap);
    Launch l{2, eoff[i], nj, i == 1 ? std::min(scan_grid(nj, srcs), enum_scan_grid(c)) : enum_scan_grid(c),
             flat_grid(enum_grid(c), enum_grid(c)), 0, 0,
             true, any_last, any_inner};
    l.next_off = i + 1 < maxk ? eoff[i + 1] : SIZE_MAX;
    l.leaf_off = leaf_off;
    L.push_back(l);
  }
  // single-vertex patterns
  {
    std::vector<ExtJob> S(nj);
    bool any = false;
    uint64_t items = 1;
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      const Plan& p = J.plan;
      ExtJob& e = S[x];
      e = ExtJob{};
      if (p.k != 1) continue;
      const CandSet r = cand_set(J, p.root);
      e.active = 1;
      e.k = 1;
      e.last = 1;
      e.src_cols = r.list;
      e.d_nsrc = r.cnt;
      e.src_cap = J.caps.lcap_u[p.root];
      e.a_begin = 0;
      e.a_end = ~0ull;
      e.flags = (uint32_t*)(J.mem.ctl + CTL_FLAGS);
      e.var_pos[0] = 0;
      e.nx = p.nx;
      e.ny = p.ny;
      e.y_false = p.y_false;
      for (int t = 0; t < 2 * MAXLIT; t++) e.lit[t] = p.lit[t];
      e.counters = (unsigned long long*)(J.mem.ctl + CTL_MATCH);
      e.vbuf = J.mem.vbuf;
      e.d_vcount = J.mem.ctl + CTL_VCOUNT;
      e.vcap = c.K > 0 ? J.caps.vcap : 0;
      e.d_thr_valid = (const uint32_t*)(J.mem.ctl + CTL_THRVALID);
      items = std::max(items, e.src_cap);
      any = true;
    }
    if (any) {
      const size_t off = R.add(S);
      for (int x = 0; x < nj; x++)
        if (S[x].active) {
          jobs[x].last_rec = off + sizeof(ExtJob) * x;
          jobs[x].last_single = true;
        }
      L.push_back(Launch{3, off, nj, 0, gx_for(items, nj), 0, 0, false, true, false});
    }
  }
  if (any_leaf) {
    Launch l{5, leaf_off, nj, 0, flat_grid(enum_grid(c), enum_grid(c)), (int)std::min<uint64_t>(
                 FLAT_GRID_MAX, std::max<uint64_t>(1, (leaf_np + BS - 1) / BS * (uint64_t)nj)),
             0, false, false, false};
    l.prep2_off = prep2_off;
    L.push_back(l);
  }
  if (c.K > 0) {
    std::vector<TopkJob> T(nj);
    for (int x = 0; x < nj; x++) {
      Job& J = jobs[x];
      T[x] = TopkJob{1, J.plan.k, c.K, J.mem.vbuf, J.mem.ctl + CTL_VCOUNT, J.caps.vcap, J.mem.res,
                     (uint32_t*)(J.mem.ctl + CTL_NEEDSEL)};
    }
    L.push_back(Launch{4, R.add(T), nj, 0, 0, 0, 0, false, false, false});
  }
}

static void run_launch(Ctx& c, const Launch& l) {
  const DevGraph& g = c.g->dg;
  uint8_t* base = c.recbase ? c.recbase : c.ws->jobrec;
  {
    switch (l.kind) {
      case 0: {
        auto* r = (const FilterJob*)(base + l.off);
        if (l.scan) {
          if (l.row_scan) c.tm.run(K_SCAN, [&] { filter_scan(c.st, g, r, l.njobs, l.gx_scan, cls_bytes(c, K_SCAN)); });
          c.tm.run(K_PULL, [&] {
            filter_pull(c.st, g, r, l.njobs, l.gx_work, l.hit_bitmaps, cls_bytes(c, K_PULL));
          });
        }
        c.tm.run(K_OTHER, [&] { filter_clear(c.st, r, l.njobs, l.gx_clear); });
        c.tm.run(K_FILTER,
                 [&] { filter_compact(c.st, g, r, l.njobs, l.gx_item, l.hit_bitmaps, cls_bytes(c, K_FILTER)); });
        break;
      }
      case 1: {
        auto* r = (const CpiJob*)(base + l.off);
        c.tm.run(K_SCAN, [&] { cpi_scan(c.st, g, r, l.njobs, l.gx_scan, cls_bytes(c, K_SCAN)); });
        if (l.cpi_two_pass) {  // lists sized by their kept entries
          c.tm.run(K_CPI, [&] { cpi_count(c.st, g, r, l.njobs, l.gx_work, cls_bytes(c, K_CPI)); });
          c.tm.run(K_CPI, [&] { cpi_alloc(c.st, g, r, l.njobs, l.gx_item); });
        } else {  // lists placed by their members' rows
          c.tm.run(K_OTHER, [&] { cpi_reserve(c.st, r, l.njobs); });
        }
        c.tm.run(K_CPI, [&] {
          cpi_fill(c.st, g, r, l.njobs, l.gx_work, !l.cpi_two_pass, cls_bytes(c, K_CPI));
        });
        break;
      }
      case 2: {
        auto* r = (const ExtJob*)(base + l.off);
        c.tm.run(K_SCAN, [&] { ext_scan(c.st, g, r, l.njobs, l.gx_scan, cls_bytes(c, K_SCAN)); });
        if (l.inner_any)  // next frontiers, sized by this level's attempts
          c.tm.run(K_OTHER, [&] {
            front_reserve(c.st, (ExtJob*)(base + l.off),
                          l.next_off == SIZE_MAX ? nullptr : (ExtJob*)(base + l.next_off),
                          l.leaf_off == SIZE_MAX ? nullptr : (LeafJob*)(base + l.leaf_off), l.njobs,
                          c.ws->front, front_usable(c.ws), c.ws->misc + 1);
          });
        if (l.inner_any)
          c.tm.run(K_EXT, [&] { ext_run(c.st, g, r, l.njobs, l.gx_work, false, false, use_occ8(c), cls_bytes(c, K_EXT)); });
        if (l.last_any)
          c.tm.run(K_LAST, [&] {
            ext_run(c.st, g, r, l.njobs, l.gx_work, true, use_ahead(c), use_occ8(c), cls_bytes(c, K_LAST));
          });
        break;
      }
      case 3: {
        auto* r = (const ExtJob*)(base + l.off);
        c.tm.run(K_LAST, [&] { ext_single(c.st, g, r, l.njobs, l.gx_work, cls_bytes(c, K_LAST)); });
        break;
      }
      case 5: {
        auto* r = (const LeafJob*)(base + l.off);
        c.tm.run(K_OTHER, [&] { leaf_prep(c.st, g, r, l.njobs, l.gx_item); });
        if (l.prep2_off != SIZE_MAX)  // the split leaves' second tables
          c.tm.run(K_OTHER, [&] { leaf_prep(c.st, g, (const LeafJob*)(base + l.prep2_off), l.njobs, l.gx_item); });
        c.tm.run(K_LAST, [&] { leaf_count(c.st, g, r, l.njobs, l.gx_work, false, cls_bytes(c, K_LAST)); });
        if (l.prep2_off != SIZE_MAX)  // the jobs with split leaves
          c.tm.run(K_LAST, [&] { leaf_count(c.st, g, r, l.njobs, l.gx_work, true, cls_bytes(c, K_LAST)); });
        break;
      }
      case 4: {
        auto* r = (const TopkJob*)(base + l.off);
        c.tm.run(K_TOPK, [&] { topk_small(c.st, r, l.njobs, cls_bytes(c, K_TOPK)); });
        break;
      }
    }
  }
}

static void run_launches(Ctx& c, const std::vector<Launch>& L) {
  for (const Launch& l : L) run_launch(c, l);
}

static void upload_recs(Ctx& c, const Recs& R) {
  HIPCHK(hipStreamSynchronize(c.st));  // nothing in flight reads the staging
  ensure_recs(c.ws, std::max<size_t>(R.blob.size(), 256));
  std::memcpy(c.ws->hjobrec, R.blob.data(), R.blob.size());
  upload_recs(c, 0, R.blob.size());
}

// Upper bound of the record bytes plan_batch writes for a batch: at most 2k
// filter steps, k CPI edges, k enumeration launches of each form, the leaf
// counts (two arrays with split leaves) and the top-K records, each array
// aligned.
static size_t recs_bound(const std::vector<Job>& jobs) {
  int maxk = 1;
  for (const Job& J : jobs) maxk = std::max(maxk, J.plan.k);
  const size_t nj = jobs.size();
  const size_t per = 2 * (size_t)maxk * sizeof(FilterJob) + (size_t)maxk * sizeof(CpiJob) +
                     2 * (size_t)maxk * sizeof(ExtJob) + 2 * sizeof(LeafJob) + sizeof(TopkJob);
  return nj * per + 256 * (6 * (size_t)maxk + 5);
}

// Records and launches of a batch, each launch enqueued as soon as its records
// are built and uploaded (to the same offsets of the device buffer, from
// disjoint parts of the pinned staging).
static void plan_and_run_batch(Ctx& c, std::vector<Job>& jobs, Recs& R, LaunchList& L) {
  Workspace* ws = c.ws;
  HIPCHK(hipStreamSynchronize(c.st));  // nothing in flight reads the staging
  ensure_recs(ws, std::max<size_t>(recs_bound(jobs), 256));
  size_t up = 0;
  L.on_add = [&](const Launch& l) {
    const size_t end = R.blob.size();
    if (end > ws->jobrec_bytes) throw GfdError{GFD_EDEVICE, "internal: record bound exceeded"};
    if (end > up) {
      std::memcpy(ws->hjobrec + up, R.blob.data() + up, end - up);
      upload_recs(c, up, end - up);
      up = end;
    }
    run_launch(c, l);
  };
  plan_batch(c, jobs, R, L, true);
  L.on_add = nullptr;
}

// Arena of a batch: [control blocks][tile states][results][job regions].
static void ensure_hres(Workspace* ws, size_t words) {
  if (ws->hres_words >= words) return;
  ws->host_put(ws->hres);
  ws->hres = nullptr;
  ws->hres_words = 0;
  ws->hres = (int32_t*)ws->host_get(sizeof(int32_t) * words, false);
  ws->hres_words = words;
}

// A batch's first-K tuples go to the callers' buffers in at most two rounds:
// the device packs the listed jobs' tuples back to back, one copy brings them
// into pinned memory, and the host moves them out, while the device works on
// the jobs still open where there are any.
struct ResultDrain {
  Ctx& c;
  const std::vector<Job>& jobs;
  gfd_result* results;
  const std::vector<uint64_t>& H;  // control words per spec
  int K;
  size_t used = 0;                 // words of ws->pack / ws->hres handed out
  struct Item { int x; size_t off, words; };
  std::vector<Item> pending;       // copied or in flight, not yet moved out

  ResultDrain(Ctx& c_, const std::vector<Job>& j, gfd_result* r, const std::vector<uint64_t>& h, int k)
      : c(c_), jobs(j), results(r), H(h), K(k) {
    // both only grow, and before anything of this batch is in them
    const size_t words = (size_t)K * MAXK * jobs.size();
    ensure_hres(c.ws, words);
    if (c.ws->pack_words < words) {
      dfree(c.ws->al, c.ws->pack, c.ws->pack_words);
      c.ws->pack_words = 0;
      c.ws->pack = dalloc<int32_t>(c.ws->al, words);
      c.ws->pack_words = words;
    }
  }
  void issue(const std::vector<int>& xs) {
    Workspace* ws = c.ws;
    std::vector<PackJob> P;
    for (int x : xs) {
      const uint64_t n = std::min<uint64_t>((uint64_t)K, H[(size_t)jobs[x].spec * CTL_WORDS + CTL_VIOL]);
      const size_t words = (size_t)n * jobs[x].plan.k;
      if (!words) continue;
      P.push_back(PackJob{jobs[x].mem.res, used, words});
      pending.push_back(Item{x, used, words});
      used += words;
    }
    if (P.empty()) return;
    const size_t w0 = P.front().dst, nw = used - w0;
    const int32_t* src = P.front().src;  // one job: its slot is already contiguous
    if (P.size() > 1) {
      HIPCHK(hipStreamSynchronize(c.st));  // the record staging is reused per launch
      ensure_recs(ws, sizeof(PackJob) * P.size());
      std::memcpy(ws->hjobrec, P.data(), sizeof(PackJob) * P.size());
      upload_recs(c, 0, sizeof(PackJob) * P.size());
      pack_results(c.st, (const PackJob*)ws->jobrec, (int)P.size(), ws->pack);
      src = ws->pack + w0;
    }
    HIPCHK(hipMemcpyAsync(ws->hres + w0, src, sizeof(int32_t) * nw, hipMemcpyDeviceToHost, c.st));
    if (ws->pack_ev) HIPCHK(hipEventRecord(ws->pack_ev, c.st));
  }
  void drain() {
    if (pending.empty()) return;
    if (c.ws->pack_ev) HIPCHK(hipEventSynchronize(c.ws->pack_ev));
    else HIPCHK(hipStreamSynchronize(c.st));
    for (const Item& it : pending)
      std::memcpy(results[jobs[it.x].spec].violations, c.ws->hres + it.off, sizeof(int32_t) * it.words);
    pending.clear();
  }
};

// Frontier pool and CPI arena: sized by what batches asked of them.  They
// start at a sixteenth of the budget (at most 256 MiB) and, when a batch asks
// for more, grow to its demand plus a quarter, up to a quarter of the budget
// (frontiers) and an eighth (CPI entries); the jobs that overflowed then run
// again in the fast path.
constexpr int64_t ADAPT_START_MAX = int64_t(256) << 20;
constexpr int MAX_REGROW = 4;  // fast-path retries of one GFD while the pool or arena grows
static size_t adapt_start(const Workspace* ws) {
  return (size_t)std::max<int64_t>(int64_t(4) << 20, std::min<int64_t>(ws->budget / 16, ADAPT_START_MAX));
}
static bool grow_to(size_t& want, size_t have, uint64_t asked, int64_t limit) {
  if (asked <= have) return false;
  const size_t lim = (size_t)std::max<int64_t>(limit, (int64_t)have);
  const size_t w = std::min<size_t>(lim, std::max<size_t>(2 * have, asked + asked / 4));
  if (w <= have) return false;
  want = std::max(want, w);
  return true;
}
// What a call may use of them: a workspace kept from calls with larger
// budgets can hold more than this call's share.
static uint64_t front_usable(const Workspace* ws) {
  return std::min<uint64_t>(ws->front_bytes, (uint64_t)std::max<int64_t>(ws->budget / 4, int64_t(4) << 20));
}
static uint64_t cpi_usable(const Workspace* ws) {
  return std::min<uint64_t>(ws->cpi_cap, (uint64_t)std::max<int64_t>(ws->budget / 32, int64_t(1) << 20));
}
static bool grow_front(Workspace* ws, uint64_t asked_bytes) {
  return grow_to(ws->front_want, front_usable(ws), asked_bytes, ws->budget / 4);
}
static bool grow_cpi(Workspace* ws, uint64_t asked_entries) {
  size_t want = ws->cpi_want * 4;
  const bool g = grow_to(want, cpi_usable(ws) * 4, asked_entries * 4, ws->budget / 8);
  ws->cpi_want = want / 4;
  return g;
}
static void ensure_front(Workspace* ws) {
  const size_t want = std::max(ws->front_want, adapt_start(ws));
  if (ws->front_bytes >= want) return;
  dfree(ws->al, ws->front, ws->front_bytes);
  ws->front_bytes = 0;
  ws->front = dalloc<uint8_t>(ws->al, want);
  ws->front_bytes = want;
  ws->gen++;
}
static void ensure_cpi(Workspace* ws) {
  const size_t want = std::max(ws->cpi_want, adapt_start(ws) / 4);
  if (ws->cpi_cap >= want) return;
  dfree(ws->al, ws->cpi_arena, ws->cpi_cap);
  ws->cpi_cap = 0;
  ws->cpi_arena = dalloc<int32_t>(ws->al, want);
  ws->cpi_cap = want;
  ws->gen++;
}

// The batch arena only grows (allocations of this size are slow).
static void ensure_arena(Workspace* ws, size_t bytes) {
  if (ws->arena_bytes >= bytes) return;
  dfree(ws->al, ws->arena, ws->arena_bytes);
  ws->arena_bytes = 0;
  ws->arena = dalloc<uint8_t>(ws->al, bytes);
  ws->arena_bytes = bytes;
  ws->gen++;
}

// Places every job's buffers (growing the workspace where needed) and, when
// `fills` is set, enqueues the clears a batch starts from; returns the bytes
// of control blocks and tile states those clears zero (batch_fills).
static size_t layout_batch(Ctx& c, std::vector<Job>& jobs, bool fills = true);
static void batch_fills(Ctx& c, size_t zero_bytes) {
  // zero the control blocks and tile states; the CPI arena and the frontier
  // pool start empty
  fill_u64(c.st, (uint64_t*)c.ws->arena, 0, zero_bytes / 8);
  fill_u64(c.st, (uint64_t*)c.ws->misc, 0, 2);
}
static size_t layout_batch(Ctx& c, std::vector<Job>& jobs, bool fills) {
  Workspace* ws = c.ws;
  const size_t nj = jobs.size();
  uint64_t tiles = 0;
  size_t body = 0;
  for (auto& J : jobs) {
    tiles = std::max(tiles, J.caps.tiles);
    body += align_up(J.caps.bytes);
  }
  const size_t ctl_b = align_up(sizeof(uint64_t) * CTL_WORDS * nj);
  const size_t ts_b = align_up(sizeof(uint64_t) * tiles * nj);
  const size_t res_b = align_up(sizeof(int32_t) * (size_t)std::max(c.K, 1) * MAXK * nj);
  const size_t total = ctl_b + ts_b + res_b + body;
  ensure_arena(ws, total);
  uint8_t* p = ws->arena + ctl_b + ts_b + res_b;
  // hit bitmaps live outside the arena, in a pool that every compaction leaves
  // zeroed, so no step clears them
  size_t hw = 0;
  for (auto& J : jobs) hw += (J.caps.hit_region + 63) / 64 * 64;
  if (ws->hitpool_words < hw) {
    dfree(ws->al, ws->hitpool, ws->hitpool_words);
    ws->hitpool_words = 0;
    ws->hitpool = dalloc<uint32_t>(ws->al, hw);
    ws->hitpool_words = hw;
    ws->gen++;
    fill_u32(c.st, ws->hitpool, 0u, hw);
  }
  size_t hoff = 0;
  for (size_t x = 0; x < nj; x++) {
    Job& J = jobs[x];
    J.mem.hits = ws->hitpool + hoff;
    hoff += (J.caps.hit_region + 63) / 64 * 64;
    J.mem.ctl = (uint64_t*)ws->arena + CTL_WORDS * x;
    J.mem.tstate = (uint64_t*)(ws->arena + ctl_b) + tiles * x;
    J.mem.res = (int32_t*)(ws->arena + ctl_b + ts_b) + (size_t)std::max(c.K, 1) * MAXK * x;
    job_layout(p, c.g, J.plan, J.caps, J.mem);
    p += align_up(J.caps.bytes);
  }
  if (ws->hctl_words < CTL_WORDS * nj) {
    ws->host_put(ws->hctl);
    ws->hctl = nullptr;
    ws->hctl_words = 0;
    ws->hctl = (uint64_t*)ws->host_get(sizeof(uint64_t) * CTL_WORDS * nj, false);
    ws->hctl_words = CTL_WORDS * nj;
    ws->gen++;
  }
  ensure_front(ws);
  ensure_cpi(ws);
  if (fills) batch_fills(c, ctl_b + ts_b);
  return ctl_b + ts_b;
}

// ---------------------------------------------------------------------------
// captured main passes (HIP graphs): a batch's clears, every launch of its
// CPI construction and enumeration, the first K and the read-back of its
// control words, replayed as one graph launch when a batch of the same shape
// comes again on the same workspace
// ---------------------------------------------------------------------------

struct GraphEntry {
  std::string key;
  uint64_t gen = 0;
  hipGraphExec_t exec = nullptr;
  uint8_t* recs = nullptr;  // the batch's records, uploaded once at capture
  size_t recs_bytes = 0;
  std::vector<Job> jobs;    // the jobs as planned (record offsets, candidate buffers)
  int launches[8] = {};
};
constexpr size_t GRAPHS_MAX = 512;  // captured shapes kept per workspace

static void drop_entry(Workspace* ws, GraphEntry* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  dfree(ws->al, e->recs, e->recs_bytes);
  delete e;
}
static void drop_graphs(Workspace* ws) {
  for (GraphEntry* e : ws->graphs) drop_entry(ws, e);
  ws->graphs.clear();
}

// What the main pass of a batch depends on besides the buffers' generation:
// the GFDs, the reading, K, the staging and frontier limits, the pool and
// arena shares and whether class bytes are counted.
static std::string graph_key(const Ctx& c, const std::vector<int>& batch, const gfd_spec* specs,
                             bool count_only, uint64_t vsmall) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  const uint64_t w[] = {(uint64_t)c.K, (uint64_t)c.induced, (uint64_t)count_only, c.front_limit, vsmall,
                        (uint64_t)c.tune.flat_grid, (uint64_t)c.tune.scan_grid, (uint64_t)use_ahead(c), (uint64_t)use_occ8(c),
                        front_usable(c.ws), cpi_usable(c.ws), (uint64_t)(c.stat_bytes != nullptr),
                        (uint64_t)batch.size()};
  k.reserve(sizeof w + sizeof(gfd_spec) * batch.size());
  put(w, sizeof w);
  for (int i : batch) put(&specs[i], sizeof(gfd_spec));
  return k;
}

static GraphEntry* find_graph(Workspace* ws, const std::string& key) {
  for (size_t i = 0; i < ws->graphs.size(); i++) {
    GraphEntry* e = ws->graphs[i];
    if (e->key != key) continue;
    if (e->gen == ws->gen) return e;
    drop_entry(ws, e);  // captured on buffers that have moved since
    ws->graphs.erase(ws->graphs.begin() + (ptrdiff_t)i);
    return nullptr;
  }
  return nullptr;
}

// Reads the batch's control words and the CPI and frontier cursors back.
static void read_back(Ctx& c, const std::vector<Job>& jobs) {
  Workspace* ws = c.ws;
  HIPCHK(hipMemcpyAsync(ws->hctl, jobs[0].mem.ctl, sizeof(uint64_t) * CTL_WORDS * jobs.size(),
                        hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipMemcpyAsync(ws->hmisc, ws->misc, 8, hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipMemcpyAsync(ws->hmisc + 10, ws->misc + 1, 8, hipMemcpyDeviceToHost, c.st));
}

// Plans the batch, uploads its records to a buffer of their own and captures
// the main pass on the workspace's capture stream.
static GraphEntry* capture_batch(Ctx& c, std::vector<Job>& jobs, size_t zero_bytes, std::string key) {
  Workspace* ws = c.ws;
  Recs R;
  LaunchList L;
  plan_batch(c, jobs, R, L, true);
  std::unique_ptr<GraphEntry> e(new GraphEntry());
  e->key = std::move(key);
  e->gen = ws->gen;
  e->recs_bytes = std::max<size_t>(R.blob.size(), 256);
  e->recs = dalloc<uint8_t>(ws->al, e->recs_bytes);
  HIPCHK(hipMemcpyAsync(e->recs, R.blob.data(), R.blob.size(), hipMemcpyHostToDevice, c.st));
  if (!ws->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ws->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamSynchronize(c.st));  // the capture stream does not order after the call's
  // one capture at a time in the process
  static std::mutex capture_mu;
  std::lock_guard<std::mutex> cap_lock(capture_mu);
  const hipStream_t st0 = c.st;
  int before[8];
  std::memcpy(before, c.tm.launches, sizeof before);
  c.st = ws->cap_stream;
  c.recbase = e->recs;
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(c.st, hipStreamCaptureModeRelaxed));
  try {
    batch_fills(c, zero_bytes);
    run_launches(c, L.v);
    read_back(c, jobs);
  } catch (...) {
    (void)hipStreamEndCapture(c.st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    c.st = st0;
    throw;
  }
  HIPCHK(hipStreamEndCapture(c.st, &graph));
  c.st = st0;
  const hipError_t ie = hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  for (int j = 0; j < 8; j++) e->launches[j] = c.tm.launches[j] - before[j];
  e->jobs = jobs;
  if (ws->graphs.size() >= GRAPHS_MAX) {  // the oldest shape goes
    drop_entry(ws, ws->graphs.front());
    ws->graphs.erase(ws->graphs.begin());
  }
  ws->graphs.push_back(e.get());
  return e.release();
}


static void ensure_chunk(Workspace* ws, size_t bytes) {
  if (ws->chunk_bytes >= bytes) return;
  dfree(ws->al, ws->chunk, ws->chunk_bytes);
  ws->chunk_bytes = 0;
  ws->chunk = dalloc<uint8_t>(ws->al, bytes);
  ws->chunk_bytes = bytes;
}

static void ensure_vbig(Workspace* ws, uint64_t vcap) {
  if (ws->vbig_cap >= vcap) return;
  dfree(ws->al, ws->vbig, (size_t)ws->vbig_cap * MAXK);
  ws->vbig_cap = 0;
  ws->vbig = dalloc<int32_t>(ws->al, (size_t)vcap * MAXK);
  ws->vbig_cap = vcap;
}

// Batched radix select over the jobs in S (at most MAX_JOBS; each with more
// than K staged tuples).  threshold == false: the first K of each job, sorted,
// into S[j].out.  threshold == true: the K-th tuple becomes the job's staging
// threshold (inclusive) and its staging count restarts at zero.
static void run_select(Ctx& c, std::vector<SelJob>& S, bool threshold) {
  Workspace* ws = c.ws;
  const int nj = (int)S.size();
  if (nj == 0) return;
  if (nj > MAX_JOBS) throw GfdError{GFD_EINVAL, "internal: selection batch too large"};
  int maxk = 0;
  uint64_t maxcap = 1;
  for (int j = 0; j < nj; j++) {
    S[j].state = ws->sel_state + (size_t)j * SEL_STATE_WORDS;
    S[j].hist = ws->sel_hist + (size_t)j * RADIX_BINS;
    if (S[j].active) {
      maxk = std::max(maxk, S[j].k);
      maxcap = std::max(maxcap, S[j].vcap);
    }
  }
  HIPCHK(hipStreamSynchronize(c.st));  // the pinned staging is reused per call
  std::memcpy(ws->hselrec, S.data(), sizeof(SelJob) * nj);
  upload(c, ws->selrec, ws->hselrec, ws->hselrec_dev, sizeof(SelJob) * nj);
  const SelJob* r = (const SelJob*)ws->selrec;
  const int gx = (int)std::max<uint64_t>(
      1, std::min<uint64_t>((maxcap + BS - 1) / BS, (uint64_t)std::max(4, 1024 / nj)));
  c.tm.run(K_TOPK, [&] { sel_begin(c.st, r, nj); });
  // tuple words are vertex ids < n: digits of at most RADIX_BITS cover the
  // id's bit width, from the top
  int idbits = 1;
  while (idbits < 31 && (int64_t(1) << idbits) < (int64_t)c.g->n) idbits++;
  const int npass = (idbits + RADIX_BITS - 1) / RADIX_BITS;
  for (int w = 0; w < maxk; w++)
    for (int ps = 0; ps < npass; ps++) {
      const int shift = std::max(0, idbits - RADIX_BITS * (ps + 1));
      const int bits = idbits - RADIX_BITS * ps - shift;
      c.tm.run(K_TOPK, [&] { sel_pass(c.st, r, nj, w, shift, bits, gx, cls_bytes(c, K_TOPK)); });
    }
  if (threshold) c.tm.run(K_TOPK, [&] { sel_threshold(c.st, r, nj); });
  else c.tm.run(K_TOPK, [&] { sel_first_k(c.st, r, nj, gx, cls_bytes(c, K_TOPK)); });
}

static SelJob sel_job(Ctx& c, int k, const int32_t* vbuf, uint64_t* ctl, uint64_t vcap) {
  SelJob s{};
  s.active = 1;
  s.k = k;
  s.K = c.K;
  s.d_vcount = ctl + CTL_VCOUNT;
  s.vbuf = vbuf;
  s.vcap = vcap;
  s.d_outcount = (unsigned long long*)(ctl + CTL_OUTCOUNT);
  s.thr = (int32_t*)(ctl + CTL_THR);
  s.d_thr_valid = (uint32_t*)(ctl + CTL_THRVALID);
  return s;
}

// First K of one job's staged tuples, sorted, into ws->sel_out.  Requires
// count > K.
static void select_first_k(Ctx& c, const int32_t* vbuf, uint64_t vcap, int k, uint64_t* ctl) {
  std::vector<SelJob> S{sel_job(c, k, vbuf, ctl, vcap)};
  S[0].out = c.ws->sel_out;
  run_select(c, S, false);
}

// Bounded path for one job whose fast pass overflowed: the frontier of every
// level is processed in windows of attempts that fit the job's capacity, and
// violation staging is cut to the first K whenever it could overflow.
struct Bounded {
  Ctx& c;
  Job& J;
  uint64_t* P[MAXK];
  uint32_t* begs[MAXK];
  uint64_t rd(int word) {
    HIPCHK(hipMemcpyAsync(c.ws->hctl + word, J.mem.ctl + word, 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    return c.ws->hctl[word];
  }
  void upload_one(const ExtJob& e) {
    HIPCHK(hipStreamSynchronize(c.st));  // the staging buffer is reused per launch
    ensure_recs(c.ws, sizeof(ExtJob));
    std::memcpy(c.ws->hjobrec, &e, sizeof e);
    upload_recs(c, 0, sizeof e);
  }
  void compact_if_needed(uint64_t incoming) {
    Workspace* ws = c.ws;
    const int k = J.plan.k;
    const uint64_t vc = rd(CTL_VCOUNT);
    if (vc + incoming <= ws->vbig_cap || vc <= (uint64_t)c.K) return;
    select_first_k(c, ws->vbig, ws->vbig_cap, k, J.mem.ctl);
    // keep the first K; the K-th becomes the staging threshold
    HIPCHK(hipMemcpyAsync(ws->vbig, ws->sel_out, sizeof(int32_t) * c.K * k,
                          hipMemcpyDeviceToDevice, c.st));
    HIPCHK(hipMemcpyAsync((int32_t*)(J.mem.ctl + CTL_THR), ws->sel_out + (size_t)(c.K - 1) * k,
                          sizeof(int32_t) * k, hipMemcpyDeviceToDevice, c.st));
    fill_u64(c.st, J.mem.ctl + CTL_VCOUNT, (uint64_t)c.K, 1);
    fill_u64(c.st, J.mem.ctl + CTL_THRVALID, 1, 1);
  }
  ExtJob base(int i) {
    const Plan& p = J.plan;
    ExtJob e{};
    e.active = 1;
    e.i = i;
    e.k = p.k;
    e.flags = (uint32_t*)(J.mem.ctl + CTL_FLAGS);
    for (int v = 0; v < MAXK; v++) e.var_pos[v] = v < p.k ? p.pos[v] : 0;
    e.nx = p.nx;
    e.ny = p.ny;
    e.y_false = p.y_false;
    for (int t = 0; t < 2 * MAXLIT; t++) e.lit[t] = p.lit[t];
    e.counters = (unsigned long long*)(J.mem.ctl + CTL_MATCH);
    e.vbuf = c.ws->vbig;
    e.d_vcount = J.mem.ctl + CTL_VCOUNT;
    e.vcap = c.K > 0 ? c.ws->vbig_cap : 0;
    e.thr = (const int32_t*)(J.mem.ctl + CTL_THR);
    e.d_thr_valid = (const uint32_t*)(J.mem.ctl + CTL_THRVALID);
    e.thr_incl = 0;  // the first K are kept apart; later tuples must precede the K-th
    return e;
  }
  void level(int i) {
    const Plan& p = J.plan;
    const int u = p.order[i], q = p.parent[u];
    ExtJob e = base(i);
    e.last = i == p.k - 1;
    if (i == 1) {
      const CandSet r = cand_set(J, p.root);
      e.src_cols = r.list;
      e.src_stride = 0;
      e.d_nsrc = r.cnt;
      e.src_cap = J.caps.lcap_u[p.root];
    } else {
      e.src_cols = J.mem.cols[i];
      e.src_stride = J.caps.cap_f;
      e.d_nsrc = J.mem.ctl + CTL_LEVEL_N + i;
      e.src_cap = J.caps.cap_f;
    }
    e.par_pos = p.pos[q];
    e.par_posmap = J.mem.pos[q];
    e.par_by_bucket = p.qlab[q] != ANY ? 1 : 0;
    e.cpi_beg = J.mem.cpi_beg[u];
    e.cpi_len = J.mem.cpi_len[u];
    e.cpi_ent = c.ws->cpi_arena;
    set_cross(J, u, e);
    e.begs = begs[i];
    e.sc = JobScan{P[i], J.mem.ctl + CTL_LEVEL_T + i, J.mem.tstate,
                   (uint32_t*)(J.mem.ctl + CTL_TICKET), c.ws->err, next_epoch(c)};
    e.nchk = p.nchk[i];
    for (int t = 0; t < MAXK; t++) {
      e.chk_pos[t] = t < p.nchk[i] ? p.chk_pos[i][t] : 0;
      e.chk_fwd[t] = t < p.nchk[i] ? p.chk_fwd[i][t] : PC_FREE;
      e.chk_bwd[t] = t < p.nchk[i] ? p.chk_bwd[i][t] : PC_FREE;
    }
    if (!e.last) {
      e.dst_cols = J.mem.cols[i + 1];
      e.dst_cap = J.caps.cap_f;
      e.d_ndst = J.mem.ctl + CTL_LEVEL_N + i + 1;
    }
    upload_one(e);
    const DevGraph& g = c.g->dg;
    const ExtJob* rec = (const ExtJob*)c.ws->jobrec;
    c.tm.run(K_SCAN, [&] { ext_scan(c.st, g, rec, 1, scan_grid(1, e.src_cap), cls_bytes(c, K_SCAN)); });
    const uint64_t T = rd(CTL_LEVEL_T + i);
    if (c.stats) c.stats->attempts += T;
    const uint64_t W = e.last ? (c.K > 0 ? c.ws->vbig_cap - (uint64_t)c.K : std::max<uint64_t>(T, 1))
                              : J.caps.cap_f;
    for (uint64_t A0 = 0; A0 < T; A0 += W) {
      const uint64_t A1 = std::min(T, A0 + W);
      if (e.last && c.K > 0) compact_if_needed(A1 - A0);
      if (!e.last) fill_u64(c.st, J.mem.ctl + CTL_LEVEL_N + i + 1, 0, 1);
      e.a_begin = A0;
      e.a_end = A1;
      upload_one(e);
      const int cls = e.last ? K_LAST : K_EXT;
      c.tm.run(cls, [&] {
        ext_run(c.st, g, rec, 1, flat_grid(chunks_of(A1 - A0), enum_grid(c)), e.last != 0, e.last != 0 && use_ahead(c),
                use_occ8(c), cls_bytes(c, cls));
      });
      if (!e.last) {
        const uint64_t N = rd(CTL_LEVEL_N + i + 1);
        if (c.stats) c.stats->partials += N;
        if (N) level(i + 1);
      }
    }
  }
  void single() {
    const Plan& p = J.plan;
    ExtJob e = base(0);
    const CandSet r = cand_set(J, p.root);
    e.k = 1;
    e.last = 1;
    e.src_cols = r.list;
    e.d_nsrc = r.cnt;
    e.src_cap = J.caps.lcap_u[p.root];
    HIPCHK(hipMemcpyAsync(c.ws->hctl, r.cnt, 8, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    const uint64_t N = c.ws->hctl[0];
    const uint64_t W = c.K > 0 ? c.ws->vbig_cap - (uint64_t)c.K : std::max<uint64_t>(N, 1);
    for (uint64_t A0 = 0; A0 < N; A0 += W) {
      const uint64_t A1 = std::min(N, A0 + W);
      if (c.K > 0) compact_if_needed(A1 - A0);
      e.a_begin = A0;
      e.a_end = A1;
      upload_one(e);
      const ExtJob* rec = (const ExtJob*)c.ws->jobrec;
      c.tm.run(K_LAST, [&] {
        ext_single(c.st, c.g->dg, rec, 1,
                   (int)std::max<uint64_t>(1, std::min<uint64_t>((A1 - A0 + BS - 1) / BS, 1024)),
                   cls_bytes(c, K_LAST));
      });
    }
  }
};

static uint64_t frontier_cap_of(const gfd_graph* g, const Plan& p, int64_t fbytes, int64_t forced);

// Fixed area (the entry point that allocates nothing): nothing above the
// fixed buffers is needed from one batch to the next, or by a bounded run, so
// each of them carves the area again from the same point (no holes).
static void rewind_area(Workspace* ws) {
  if (!ws->al.area) return;
  ws->forget_call_buffers();
  ws->al.area_top = ws->area_mark;
}

static void run_bounded(Ctx& c, Job& J, uint64_t vbig) {
  Workspace* ws = c.ws;
  rewind_area(ws);
  std::vector<Job> one{J};
  // the job alone, with its own frontier columns for every level: an eighth
  // of the budget (or the testing cap)
  job_caps(c.g, J.plan, frontier_cap_of(c.g, J.plan, ws->budget / 8, (int64_t)c.front_limit), J.caps.vcap,
           true, one[0].caps);
  layout_batch(c, one);
  Job& B = one[0];
  Recs R;
  LaunchList L;
  plan_batch(c, one, R, L, false);
  upload_recs(c, R);
  run_launches(c, L.v);
  HIPCHK(hipMemcpyAsync(ws->hctl, B.mem.ctl, sizeof(uint64_t) * CTL_WORDS, hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  if (ws->hctl[CTL_FLAGS] & 4u)
    throw GfdError{GFD_ENOMEM, "CPI lists exceed the entry arena; raise mem_budget_bytes"};
  ensure_vbig(ws, vbig);
  Bounded b{c, B, {}, {}};
  const uint64_t pc = B.caps.begs + 1;
  ensure_chunk(ws, (size_t)MAXK * (align_up(8 * (pc + 1)) + align_up(4 * pc)));
  uint8_t* p = ws->chunk;
  for (int i = 0; i < MAXK; i++) {
    b.P[i] = (uint64_t*)p;
    p += align_up(8 * (pc + 1));
    b.begs[i] = (uint32_t*)p;
    p += align_up(4 * pc);
  }
  if (B.plan.k == 1) b.single();
  else b.level(1);
  if (c.K > 0) {
    std::vector<TopkJob> T{TopkJob{1, B.plan.k, c.K, ws->vbig, B.mem.ctl + CTL_VCOUNT, ws->vbig_cap,
                                   B.mem.res, (uint32_t*)(B.mem.ctl + CTL_NEEDSEL)}};
    HIPCHK(hipStreamSynchronize(c.st));  // nothing in flight reads the staging
    ensure_recs(ws, sizeof(TopkJob));
    std::memcpy(ws->hjobrec, T.data(), sizeof(TopkJob));
    upload_recs(c, 0, sizeof(TopkJob));
    c.tm.run(K_TOPK, [&] { topk_small(c.st, (const TopkJob*)ws->jobrec, 1, cls_bytes(c, K_TOPK)); });
    HIPCHK(hipMemcpyAsync(ws->hctl, B.mem.ctl, sizeof(uint64_t) * CTL_WORDS, hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    if (ws->hctl[CTL_NEEDSEL]) {
      select_first_k(c, ws->vbig, ws->vbig_cap, B.plan.k, B.mem.ctl);
      HIPCHK(hipMemcpyAsync(B.mem.res, ws->sel_out, sizeof(int32_t) * c.K * B.plan.k,
                            hipMemcpyDeviceToDevice, c.st));
    }
  }
  J.mem = B.mem;
}

// Jobs whose fast pass overflowed only the violation staging: their counts
// and fingerprints are exact, only the first K are missing.  The K-th smallest
// staged tuple bounds the K-th smallest violation from above, so the last
// level is run again over its kept frontier, collecting only violations up to
// that threshold; repeated (each pass strictly lowers the threshold) until the
// collected ones fit.  Every pass is one launch for all such jobs of a batch.
// Leaves each finished job's control block in ws->hctl; jobs still over after
// the pass limit go to the bounded path (redo).
static void rerun_last_levels(Ctx& c, std::vector<Job>& jobs, std::vector<int> over,
                              const std::vector<ExtJob>& lastrec, uint64_t vsmall, std::vector<char>& redo,
                              const std::function<void()>& while_busy, bool preset = false) {
  Workspace* ws = c.ws;
  const DevGraph& g = c.g->dg;
  for (int pass = 0; !over.empty(); pass++) {
    if (pass == 8) {
      for (int x : over) redo[x] = 1;
      return;
    }
    if (pass > 0 || !preset) {  // preset: the first pass's thresholds are already set
      std::vector<SelJob> S;
      for (int x : over) S.push_back(sel_job(c, jobs[x].plan.k, jobs[x].mem.vbuf, jobs[x].mem.ctl, vsmall));
      run_select(c, S, true);
    }
    // last-level records in collect-only form, multi-vertex and single-vertex
    std::vector<ExtJob> E[2];
    for (int x : over) {
      ExtJob e = lastrec[x];
      e.deferred = 0;
      e.collect_only = 1;
      e.thr = (const int32_t*)(jobs[x].mem.ctl + CTL_THR);
      e.thr_incl = 1;
      e.prune = 1;
      e.sc.epoch = next_epoch(c);
      E[jobs[x].last_single ? 1 : 0].push_back(e);
    }
    const size_t b0 = align_up(sizeof(ExtJob) * E[0].size());
    const size_t bytes = b0 + sizeof(ExtJob) * E[1].size() + sizeof(TopkJob) * over.size();
    HIPCHK(hipStreamSynchronize(c.st));  // nothing in flight reads the staging
    ensure_recs(ws, bytes);
    std::memcpy(ws->hjobrec, E[0].data(), sizeof(ExtJob) * E[0].size());
    std::memcpy(ws->hjobrec + b0, E[1].data(), sizeof(ExtJob) * E[1].size());
    std::vector<TopkJob> T;
    for (int x : over)
      T.push_back(TopkJob{1, jobs[x].plan.k, c.K, jobs[x].mem.vbuf, jobs[x].mem.ctl + CTL_VCOUNT,
                          vsmall, jobs[x].mem.res, (uint32_t*)(jobs[x].mem.ctl + CTL_NEEDSEL)});
    const size_t bt = b0 + sizeof(ExtJob) * E[1].size();
    std::memcpy(ws->hjobrec + bt, T.data(), sizeof(TopkJob) * T.size());
    upload_recs(c, 0, bytes);
    const int n0 = (int)E[0].size(), n1 = (int)E[1].size();
    uint64_t srcs = 1;
    for (auto& e : E[0]) srcs = std::max(srcs, e.src_cap);
    if (n0)  // attempts again, without the sources the threshold rules out
      c.tm.run(K_SCAN, [&] {
        ext_scan(c.st, g, (const ExtJob*)ws->jobrec, n0, scan_grid(n0, srcs), cls_bytes(c, K_SCAN));
      });
    if (n0)
      c.tm.run(K_LAST, [&] {
        ext_run(c.st, g, (const ExtJob*)ws->jobrec, n0, flat_grid(enum_grid(c), enum_grid(c)), true, use_ahead(c),
                use_occ8(c), cls_bytes(c, K_LAST));
      });
    if (n1) {
      uint64_t items = 1;
      for (auto& e : E[1]) items = std::max(items, e.src_cap);
      c.tm.run(K_LAST, [&] {
        ext_single(c.st, g, (const ExtJob*)(ws->jobrec + b0), n1, gx_for(items, n1),
                   cls_bytes(c, K_LAST));
      });
    }
    // the jobs whose collection now fits get their first K (sorted, or flagged
    // for the radix select)
    c.tm.run(K_TOPK, [&] { topk_small(c.st, (const TopkJob*)(ws->jobrec + bt), (int)T.size(), cls_bytes(c, K_TOPK)); });
    // the batch's control blocks are contiguous: one copy (the other jobs'
    // words are unchanged since the main pass's read-back)
    HIPCHK(hipMemcpyAsync(ws->hctl, jobs[0].mem.ctl, sizeof(uint64_t) * CTL_WORDS * jobs.size(),
                          hipMemcpyDeviceToHost, c.st));
    while_busy();
    HIPCHK(hipStreamSynchronize(c.st));
    if (c.stats) c.stats->threshold_passes++;
    std::vector<int> next;
    for (int x : over)
      if (ws->hctl[CTL_WORDS * x + CTL_VCOUNT] > vsmall) next.push_back(x);
    over.swap(next);
  }
}

// Device records of jobs xs (offset off(x) in the batch's records at base)
// into out[x]: one gather launch into the mapped staging (the main pass is
// done with it) instead of a small DMA copy per job, where there is one.
template <class Rec, class Off>
static void read_recs(Ctx& c, const uint8_t* base, const std::vector<int>& xs, Off off,
                      std::vector<Rec>& out) {
  static_assert(sizeof(Rec) % 8 == 0, "records are copied as 8-byte words");
  Workspace* ws = c.ws;
  if (xs.empty()) return;
  if (xs.size() > (size_t)MAX_JOBS) throw GfdError{GFD_EINVAL, "internal: too many records to read"};
  if (ws->hjobrec_dev && ws->hjobrec_bytes >= sizeof(Rec) * xs.size()) {
    RecGather gr{};
    gr.n = (int32_t)xs.size();
    gr.words = (uint32_t)(sizeof(Rec) / 8);
    for (size_t i = 0; i < xs.size(); i++) gr.off[i] = off(xs[i]);
    gather_recs(c.st, base, gr, (uint64_t*)ws->hjobrec_dev);
    HIPCHK(hipStreamSynchronize(c.st));
    for (size_t i = 0; i < xs.size(); i++) std::memcpy(&out[xs[i]], ws->hjobrec + i * sizeof(Rec), sizeof(Rec));
  } else {
    for (int x : xs)
      HIPCHK(hipMemcpyAsync(&out[x], base + off(x), sizeof(Rec), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
  }
}

// First-K windows of count-only jobs whose last leaf was counted (their
// counts are final): a radix select over the variable-0 vertices of the
// partial matches, weighted by each one's violating completions (the leaf
// count again, in window form, over the partial matches of the decided
// prefix), gives the variable-0 vertex d of the K-th violation, or no bound
// when the job has fewer than K.  The deferred last level then runs
// collect-only with the threshold (d, all ones): sources past d get no
// attempts, and what it stages holds the first K.  Records: leafrec and
// lastrec hold the jobs' device records as the main pass left them.
static void run_windows(Ctx& c, std::vector<Job>& jobs, const std::vector<int>& win,
                        const std::vector<LeafJob>& leafrec, const std::vector<ExtJob>& lastrec,
                        uint64_t vsmall, std::vector<char>& redo, const std::function<void()>& while_busy) {
  Workspace* ws = c.ws;
  const DevGraph& g = c.g->dg;
  const int nw = (int)win.size();
  if (nw == 0) return;
  int idbits = 1;
  while (idbits < 31 && (int64_t(1) << idbits) < (int64_t)c.g->n) idbits++;
  const int npass = (idbits + RADIX_BITS - 1) / RADIX_BITS;
  std::vector<WinJob> W(nw);
  std::vector<LeafJob> F(nw);
  // per job: the histogram, prefix and rank, in the bounded path's chunk
  // buffer (that path runs after the windows, if at all)
  ensure_chunk(ws, sizeof(unsigned long long) * (RADIX_BINS + 2) * (size_t)nw);
  for (int i = 0; i < nw; i++) {
    Job& J = jobs[win[i]];
    auto* hist = (unsigned long long*)ws->chunk + (size_t)i * (RADIX_BINS + 2);
    W[i] = WinJob{1, J.plan.k, (uint64_t)c.K, hist, (uint32_t*)(hist + RADIX_BINS), hist + RADIX_BINS + 1,
                  (int32_t*)(J.mem.ctl + CTL_THR), (uint32_t*)(J.mem.ctl + CTL_THRVALID),
                  J.mem.ctl + CTL_VCOUNT};
    F[i] = leafrec[win[i]];
    F[i].whist = hist;
    F[i].wprefix = W[i].prefix;
    F[i].wkey_pos = J.plan.pos[0];
  }
  // every pass's records at once (the staging is read when the copy runs)
  const size_t wb = align_up(sizeof(WinJob) * nw), fb = align_up(sizeof(LeafJob) * nw);
  const size_t bytes = wb + fb * npass;
  HIPCHK(hipStreamSynchronize(c.st));  // nothing in flight reads the staging
  ensure_recs(ws, bytes);
  std::memcpy(ws->hjobrec, W.data(), sizeof(WinJob) * nw);
  auto digit = [&](int ps, int& shift, int& bits) {
    shift = std::max(0, idbits - RADIX_BITS * (ps + 1));
    bits = idbits - RADIX_BITS * ps - shift;
  };
  for (int ps = 0; ps < npass; ps++) {
    int shift, bits;
    digit(ps, shift, bits);
    for (LeafJob& f : F) {
      f.wshift = shift;
      f.wbits = bits;
    }
    std::memcpy(ws->hjobrec + wb + fb * ps, F.data(), sizeof(LeafJob) * nw);
  }
  upload_recs(c, 0, bytes);
  const WinJob* wr = (const WinJob*)ws->jobrec;
  c.tm.run(K_TOPK, [&] { win_begin(c.st, wr, nw); });
  for (int ps = 0; ps < npass; ps++) {
    int shift, bits;
    digit(ps, shift, bits);
    const LeafJob* fr = (const LeafJob*)(ws->jobrec + wb + fb * ps);
    c.tm.run(K_LAST, [&] {
      leaf_count(c.st, g, fr, nw, flat_grid(enum_grid(c), enum_grid(c)), false, cls_bytes(c, K_LAST));
    });
    c.tm.run(K_TOPK, [&] { win_digit(c.st, wr, nw, shift, bits, ps == npass - 1); });
  }
  rerun_last_levels(c, jobs, win, lastrec, vsmall, redo, while_busy, true);
}

// Leaf postponement for a count-only call under the non-induced reading: the
// longest tail of the matching order made of leaves (skeleton degree 1) with
// one common parent, the same vertex label and the same edges to it, and
// literals that touch no vertex but themselves.  Their completions of a
// partial match are then counted per parent candidate instead of enumerated.
// When only the last leaf has that form but the one before it is a leaf too,
// under another parent, the two are counted together (split leaves): the
// product of their lists' counts less the vertices both lists hold.
// (Under the induced reading a leaf must also avoid edges to every other
// matched vertex, which the per-list counts cannot see.)  A call that lists
// the first K > 0 violations counts only the last leaf, and only when it is
// not variable 0: the window of the first K is bounded by the variable-0
// vertex of the partial matches, whose violating completions the counts give.
static void plan_leaves(const gfd_spec& s, bool induced, bool count_only, int K, Plan& p) {
  p.leaf_r = 0;
  p.k_enum = p.k;
  p.leaf_par = -1;
  p.leaf_split = false;
  p.leaf_par2 = -1;
  p.leaf_window = false;
  for (int t = 0; t < 2 * MAXLIT; t++) p.lit_leaf[t] = -1;
  if (!count_only || induced || p.k < 2) return;
  if (K > 0 && p.order[p.k - 1] == 0) return;
  int deg[MAXK] = {};
  for (int a = 0; a < p.k; a++)
    for (int b = 0; b < p.k; b++)
      if (a != b && (p.qe[a][b] != NOEDGE || p.qe[b][a] != NOEDGE)) deg[a]++;
  int r = 0;
  const int rmax = K > 0 ? 1 : MAX_LEAVES;
  for (int i = p.k - 1; i >= 1 && r < rmax; i--) {
    const int u = p.order[i], u0 = p.order[p.k - 1], q = p.parent[u];
    if (deg[u] != 1 || p.core[u] || q != p.parent[u0] || p.pos[q] >= p.k - 1 - r) break;
    if (p.qlab[u] != p.qlab[u0] || p.qe[q][u] != p.qe[q][u0] || p.qe[u][q] != p.qe[u0][q]) break;
    r++;
  }
  if (r == 0) return;
  // literals: each on one leaf alone, or on inner vertices alone
  int32_t lit_leaf[2 * MAXLIT];
  auto literals_fit = [&](int rr) {
    for (int t = 0; t < s.num_x + s.num_y; t++) {
      const gfd_literal& l = t < s.num_x ? s.x[t] : s.y[t - s.num_x];
      const bool a = p.pos[l.var] >= p.k - rr;
      const bool b = l.kind == GFD_LIT_VAR && p.pos[l.var2] >= p.k - rr;
      if (l.kind == GFD_LIT_VAR && (a != b || (a && l.var2 != l.var))) return false;
      lit_leaf[t] = a ? p.pos[l.var] - (p.k - rr) : -1;
    }
    return true;
  };
  bool split = false;
  if (r == 1 && p.k >= 3 && K == 0) {
    const int ua = p.order[p.k - 2], ub = p.order[p.k - 1];
    const int qa = p.parent[ua], qb = p.parent[ub];
    split = deg[ua] == 1 && !p.core[ua] && !p.virt[ua] && qa != qb && p.pos[qa] < p.k - 2 &&
            p.pos[qb] < p.k - 2 && literals_fit(2);
  }
  if (split) {
    r = 2;
  } else if (!literals_fit(r)) {
    return;
  }
  p.leaf_r = r;
  p.k_enum = p.k - r;
  p.leaf_par = p.parent[p.order[p.k - 1]];
  p.leaf_window = K > 0;
  if (split) {
    p.leaf_split = true;
    p.leaf_par2 = p.parent[p.order[p.k - 2]];
  }
  for (int t = 0; t < s.num_x + s.num_y; t++) p.lit_leaf[t] = lit_leaf[t];
}

// Capacities of one call: violation staging per job (vsmall), the bounded
// path's staging (vbig) and the frontier bytes of each deep job (fbytes).
struct Sizing {
  uint64_t vsmall, vbig;
  int64_t fbytes;
};
static Sizing call_sizing(int64_t budget, int64_t njobs, int64_t deep, int K, int64_t violation_cap) {
  Sizing z;
  njobs = std::max<int64_t>(1, njobs);
  // violation staging per job: a sixteenth of the budget over the batch, at
  // most 2^18 tuples.  Every radix-select pass reads what is staged, while a
  // threshold re-run skips the sources its bound rules out, so a small
  // sample and another re-run beat a large sample.
  const uint64_t vdef = (uint64_t)std::max<int64_t>(
      16384, std::min<int64_t>(budget / (16 * njobs) / (4 * MAXK), int64_t(1) << 18));
  z.vsmall = std::max<uint64_t>(violation_cap ? (uint64_t)violation_cap : vdef, (uint64_t)K + 1);
  // the bounded path's staging: an eighth of the budget, 2^16 to 2^22 tuples
  const uint64_t vb = (uint64_t)std::max<int64_t>(
      65536, std::min<int64_t>(budget / (8 * 4 * MAXK), int64_t(4) << 20));
  z.vbig = std::max<uint64_t>(violation_cap ? (uint64_t)violation_cap : vb, (uint64_t)K + 64);
  // half of the budget holds frontiers, shared evenly by the jobs of a batch
  // that have any (k > 2), each sized for its own pattern size
  z.fbytes = std::min<int64_t>(budget / (2 * std::max<int64_t>(1, deep)), int64_t(8) << 30);
  return z;
}

// Frontier capacity of one job (64 partial matches per data edge bounds what
// small graphs can need).
static uint64_t frontier_cap_of(const gfd_graph* g, const Plan& p, int64_t fbytes, int64_t forced) {
  if (forced) return (uint64_t)forced;
  return (uint64_t)std::max<int64_t>(
      4096, std::min<int64_t>(fbytes / (int64_t)per_slot_bytes(p.k), 64 * g->m));
}

// Default limit on a call's device memory: a quarter of what is free, at most
// 64 GiB.  A call allocates by need within it (candidate structures by label
// bucket, frontiers and CPI entries by what the batches ask for), not the
// limit itself.
static int64_t default_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return int64_t(4) << 30;
  const int64_t b = (int64_t)(fr / 4);
  return std::max<int64_t>(int64_t(256) << 20, std::min<int64_t>(b, int64_t(64) << 30));
}

// The fixed device buffers of a workspace, its host staging and its event;
// the selection histograms and the error word start at zero.
static void init_ws_buffers(Workspace* w, hipStream_t st) {
  w->misc = dalloc<unsigned long long>(w->al, 16);
  w->err = dalloc<uint32_t>(w->al, 1);
  w->sel_state = dalloc<uint32_t>(w->al, (size_t)MAX_JOBS * SEL_STATE_WORDS);
  w->sel_hist = dalloc<uint32_t>(w->al, (size_t)MAX_JOBS * RADIX_BINS);
  w->sel_out = dalloc<int32_t>(w->al, (size_t)SORT_MAX * MAXK);
  w->selrec = dalloc<uint8_t>(w->al, sizeof(SelJob) * MAX_JOBS);
  if (!w->hselrec) {
    w->hselrec = (uint8_t*)w->host_get(sizeof(SelJob) * MAX_JOBS, true);
    w->hselrec_dev = w->pageable ? nullptr : mapped_ptr(w->hselrec);
  }
  if (!w->hmisc) w->hmisc = (uint64_t*)w->host_get(sizeof(uint64_t) * 16, false);
  if (!w->pageable && !w->pack_ev) HIPCHK(hipEventCreateWithFlags(&w->pack_ev, hipEventDisableTiming));
  fill_u32(st, w->sel_hist, 0u, (uint64_t)MAX_JOBS * RADIX_BINS);
  fill_u32(st, w->err, 0u, 1);
  HIPCHK(hipStreamSynchronize(st));
}

// An idle workspace of g whose device memory comes from `alloc` (made if
// there is none); its buffers grow as calls need them.
static Workspace* acquire_ws(gfd_graph* g, int64_t budget, const gfd_allocator& alloc,
                             hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(g->mu);
    for (size_t i = 0; i < g->pool.size(); i++) {
      Workspace* w = g->pool[i];
      if (!w->al.same(alloc)) continue;
      g->pool.erase(g->pool.begin() + (ptrdiff_t)i);
      w->budget = budget;
      w->al.st = st;
      return w;
    }
  }
  Workspace* w = new Workspace();
  try {
    w->budget = budget;
    w->al.cb = alloc;
    w->al.st = st;
    init_ws_buffers(w, st);
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

// gfd_validate_ex on a workspace from the graph's pool (fixed == nullptr) or
// on the given one, whose budget is set.
static int32_t validate_impl(const gfd_graph* gc, const gfd_spec* specs, int32_t num_specs,
                             const gfd_validate_opts* opts, gfd_result* results, gfd_stats* stats,
                             Workspace* fixed) {
  const auto t_start = std::chrono::steady_clock::now();
  const Range whole("gfd_validate");
  gfd_graph* g = const_cast<gfd_graph*>(gc);
  if (!g) return set_error(GFD_EINVAL, "graph is NULL");
  if (num_specs < 0 || (num_specs > 0 && (!specs || !results)))
    return set_error(GFD_EINVAL, "specs/results");
  gfd_validate_opts o{};
  o.k_max = 1024;
  o.semantics = GFD_SEM_INDUCED;
  if (opts) o = *opts;
  if (o.k_max < 0 || o.k_max > SORT_MAX)
    return set_error(o.k_max < 0 ? GFD_EINVAL : GFD_EUNSUPPORTED, "k_max %d (max %d)", o.k_max, SORT_MAX);
  if (o.semantics != GFD_SEM_INDUCED && o.semantics != GFD_SEM_MONO) return set_error(GFD_EINVAL, "semantics");
  if (o.batched != 0 && o.batched != 1) return set_error(GFD_EINVAL, "batched must be 0 or 1");
  if (o.mem_budget_bytes < 0 || o.frontier_cap < 0 || o.violation_cap < 0) return set_error(GFD_EINVAL, "negative option");
  if (int32_t rc = check_allocator(o.allocator)) return rc;
  {
    const gfd_tuning& t = o.tuning;
    auto grid_ok = [](int32_t x) { return x == 0 || (x >= 64 && x <= 16384); };
    if (!grid_ok(t.flat_grid) || !grid_ok(t.scan_grid) || t.probe_ahead < 0 || t.probe_ahead > 2 ||
        t.ext_occupancy < 0 || t.ext_occupancy > 2 ||
        !(t.staging_log2 == 0 || (t.staging_log2 >= 10 && t.staging_log2 <= 24)))
      return set_error(GFD_EINVAL, "tuning out of range");
  }
  const bool count_only = (o.flags & GFD_FLAG_COUNT_ONLY) != 0;
  for (int32_t i = 0; i < num_specs; i++) {
    const int32_t rc = check_spec(g, specs[i], i);
    if (rc) return rc;
    if (o.k_max > 0 && !results[i].violations) return set_error(GFD_EINVAL, "result %d: violations buffer is NULL", i);
  }
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (num_specs == 0) return GFD_OK;
  if (o.mem_budget_bytes && o.mem_budget_bytes < (int64_t(64) << 20))
    return set_error(GFD_ENOMEM, "mem_budget_bytes below 64 MiB");
  const int K = o.k_max;
  Workspace* ws = nullptr;
  try {
    const int64_t budget =
        fixed ? fixed->budget : (o.mem_budget_bytes ? o.mem_budget_bytes : default_budget());
    ws = fixed ? fixed : acquire_ws(g, budget, o.allocator, (hipStream_t)o.hip_stream);
    if (ws->hitpool_dirty && ws->hitpool)  // an earlier call stopped midway
      fill_u32((hipStream_t)o.hip_stream, ws->hitpool, 0u, ws->hitpool_words);
    ws->hitpool_dirty = true;
    const int max_batch = o.batched ? MAX_JOBS : 1;
    const int64_t njobs_hint = std::min<int64_t>(num_specs, max_batch);
    int64_t deep = 0;
    for (int32_t i = 0; i < num_specs; i++) deep += specs[i].num_vertices > 2;
    Sizing sz = call_sizing(budget, njobs_hint, std::min<int64_t>(deep, max_batch), K, o.violation_cap);
    if (o.tuning.staging_log2 && !o.violation_cap)  // the tuned staging per GFD of a batch
      sz.vsmall = std::max<uint64_t>(uint64_t(1) << o.tuning.staging_log2, (uint64_t)K + 1);
    const uint64_t vsmall = sz.vsmall, vbig = sz.vbig;
    Ctx c{g, ws, (hipStream_t)o.hip_stream, o.semantics == GFD_SEM_INDUCED, K, (uint64_t)o.frontier_cap,
          Timer{}, stats, stats ? ws->misc + 8 : nullptr};
    c.tune = o.tuning;
    const uint32_t cls_mask = ((uint32_t)o.flags >> 8) & 0xFFu;
    c.tm.on = stats && ((o.flags & GFD_FLAG_TIMING) || cls_mask);
    c.tm.mask = cls_mask ? cls_mask : 0xFFu;
    c.tm.st = c.st;
    if (stats) {
      fill_u64(c.st, (uint64_t*)(ws->misc + 8), 0, 8);
      units_clear(c.st);
    }
    fill_u32(c.st, ws->err, 0u, 1);
    // plans, capacities and batches (those of the last call on this
    // workspace when it had the same GFDs and options)
    std::optional<Range> phase(std::in_place, "plan");
    const uint64_t mkey[6] = {(uint64_t)c.induced, (uint64_t)count_only, vsmall, (uint64_t)budget,
                              (uint64_t)max_batch, (uint64_t)c.K};
    PlanMemo* pm = ws->memo.get();
    if (!(pm && pm->specs.size() == (size_t)num_specs && !std::memcmp(pm->key, mkey, sizeof mkey) &&
          !std::memcmp(pm->specs.data(), specs, sizeof(gfd_spec) * (size_t)num_specs))) {
      auto m = std::make_shared<PlanMemo>();
      m->all.resize(num_specs);
      for (int32_t i = 0; i < num_specs; i++) {
        Job& J = m->all[i];
        J.spec = i;
        make_plan(g, specs[i], c.induced, J.plan);
        plan_leaves(specs[i], c.induced, count_only, c.K, J.plan);
        job_caps(g, J.plan, 0, vsmall, false, J.caps);
        m->est += (double)est_front_bytes(g, J.plan);
      }
      std::vector<int> cur;
      int64_t used = 0;
      for (int32_t i = 0; i < num_specs; i++) {
        const int64_t b = (int64_t)m->all[i].caps.bytes + 4096 * CTL_WORDS;
        if (!cur.empty() && ((int)cur.size() >= max_batch || used + b > budget)) {
          m->batches.push_back(cur);
          cur.clear();
          used = 0;
        }
        cur.push_back(i);
        used += b;
      }
      if (!cur.empty()) m->batches.push_back(cur);
      m->specs.assign(specs, specs + num_specs);
      std::memcpy(m->key, mkey, sizeof mkey);
      ws->memo = m;
      pm = m.get();
    }
    const std::vector<Job>& all = pm->all;
    {
      // a fresh pool is sized by the frontier estimate of the call's GFDs (at
      // most 1 GiB); it grows from there to what batches ask for
      const double cap = (double)std::min<int64_t>(budget / 4, int64_t(1) << 30);
      ws->front_want = std::max(ws->front_want, (size_t)std::min(pm->est * 1.25, cap));
    }
    std::vector<std::vector<int>> batches = pm->batches;
    const bool force_bounded = (o.flags & GFD_FLAG_FORCE_CHUNKED) != 0;
    std::vector<uint64_t> H((size_t)num_specs * CTL_WORDS);
    // first K of GFD i, straight into results[i].violations (counts come
    // from the control words)
    auto reported = [&](int32_t i) -> uint64_t {
      return std::min<uint64_t>((uint64_t)K, H[(size_t)i * CTL_WORDS + CTL_VIOL]);
    };
    uint64_t cpi_entries = 0;
    std::vector<char> retried(num_specs, 0);
    // 1: ran again in a smaller batch packed with other jobs that overflowed;
    // 2: ran again in a batch of its own
    std::vector<char> alone(num_specs, 0);
    bool moved = false;                         // a GFD left its batch: the pool was at its cap
    std::vector<char> went_bounded(num_specs, 0);
    // redo[x]: 1 the job runs again on the bounded path; 2 it runs again in a
    // later fast batch (the frontier pool or CPI arena it overflowed has grown)
    // the batches formed here run their main pass from captured graphs (not
    // the retries appended below, which follow a growth of the buffers)
    const bool use_graphs = !(o.flags & GFD_FLAG_NO_GRAPH) && !c.tm.on && !ws->al.area && !force_bounded;
    const size_t n_planned = batches.size();
    phase.reset();
    for (size_t bi = 0; bi < batches.size(); bi++) {
      const Range batch_range("batch");
      rewind_area(ws);
      const bool graph = use_graphs && bi < n_planned;
      // a batch whose main pass was captured replays it with the plans,
      // records and buffers it was captured with: no layout, no records
      GraphEntry* e = nullptr;
      std::string key;
      if (graph) {
        const Range lookup_range("graph lookup");
        key = graph_key(c, batches[bi], specs, count_only, vsmall);
        e = find_graph(ws, key);
      }
      std::vector<Job> jobs;
      size_t zero_bytes = 0;
      if (e) {
        jobs = e->jobs;
        for (size_t x = 0; x < jobs.size(); x++) jobs[x].spec = batches[bi][x];
        for (int j = 0; j < 8; j++) c.tm.launches[j] += e->launches[j];
        if (stats) stats->graph_replays++;
      } else {
        const Range layout_range("layout");
        for (int i : batches[bi]) jobs.push_back(all[i]);
        zero_bytes = layout_batch(c, jobs, !graph);
      }
      std::vector<char> redo(jobs.size(), force_bounded ? 1 : 0);
      if (!force_bounded) {
        if (graph && !e) {
          // a shape seen once before is captured now; one seen for the first
          // time runs eagerly (most shapes of a serving mix never repeat)
          {
            const size_t h = std::hash<std::string>()(key);
            if (std::find(ws->seen.begin(), ws->seen.end(), h) != ws->seen.end()) {
              e = capture_batch(c, jobs, zero_bytes, std::move(key));
              if (stats) stats->graph_captures++;
            } else {
              ws->seen.push_back(h);
              if (ws->seen.size() > 4 * GRAPHS_MAX) ws->seen.pop_front();
              batch_fills(c, zero_bytes);  // the eager pass below starts from them
            }
          }
        }
        {
          // filter, CPI, enumeration with the literal check, first K
          const Range main_pass(e ? "main pass (graph replay)" : "main pass");
          if (e) {
            c.recbase = e->recs;
            HIPCHK(hipGraphLaunch(e->exec, c.st));
          } else {
            Recs R;
            LaunchList L;
            plan_and_run_batch(c, jobs, R, L);
            read_back(c, jobs);
          }
          HIPCHK(hipStreamSynchronize(c.st));
        }
        uint8_t* const recbase = c.recbase ? c.recbase : ws->jobrec;  // where the main pass's records are
        c.recbase = nullptr;
        cpi_entries += std::min<uint64_t>(ws->hmisc[0], ws->cpi_cap);
        // what the batch asked of the frontier pool and the CPI arena (failed
        // reservations included): they grow to it for the next batch
        const bool grew_f = grow_front(ws, ws->hmisc[10]);
        const bool grew_c = grow_cpi(ws, ws->hmisc[0]);
        const bool grew = grew_f || grew_c;
        std::vector<int> over;  // only the violation staging overflowed
        std::vector<int> win;   // counted last leaf, violations to list: a first-K window
        std::vector<int> again, solo;
        std::vector<std::pair<uint64_t, int>> pack;  // (frontier bytes asked, GFD)
        const uint64_t pool_cap = front_usable(ws);
        for (size_t x = 0; x < jobs.size(); x++) {
          const uint64_t* h = ws->hctl + CTL_WORDS * x;
          const int sp = jobs[x].spec;
          std::memcpy(&H[(size_t)sp * CTL_WORDS], h, sizeof(uint64_t) * CTL_WORDS);
          if (h[CTL_FLAGS] & 5u) {  // frontier or CPI arena overflow
            // a job that failed at one level asks again at the next one, so
            // a few rounds of growth may be needed before its frontiers fit
            if (grew && retried[sp] < MAX_REGROW) {
              redo[x] = 2;
              retried[sp]++;
              again.push_back(sp);
            } else if (jobs.size() > 1 && alone[sp] < 2) {
              // the pool or arena is at its cap but was shared: in a smaller
              // batch, then alone, the job has more of it, which is usually
              // enough (and much faster than the bounded path). Only a
              // frontier overflow says what the job asks for.
              redo[x] = 2;
              moved = true;
              const uint64_t need = reached_front_bytes(jobs[x].plan, h, c.front_limit);
              if (alone[sp] == 0 && !(h[CTL_FLAGS] & 4u) && need < pool_cap) {
                alone[sp] = 1;
                pack.push_back({need, sp});
              } else {
                alone[sp] = 2;
                solo.push_back(sp);
              }
            } else {
              redo[x] = 1;
            }
          } else if (K > 0 && jobs[x].plan.leaf_window) {
            if (h[CTL_VIOL] > 0 && !(h[CTL_FLAGS] & FLAG_COUNTER_OVERFLOW)) win.push_back((int)x);
          } else if (K > 0 && h[CTL_VCOUNT] > vsmall) {
            over.push_back((int)x);
          }
        }
        if (!again.empty()) {
          batches.push_back(again);
          if (stats) stats->regrown_gfds += (int32_t)again.size();
        }
        if (!pack.empty()) {
          // first fit, largest first, into batches that ask at most the pool
          std::stable_sort(pack.begin(), pack.end(),
                           [](const std::pair<uint64_t, int>& u, const std::pair<uint64_t, int>& v) {
                             return u.first > v.first;
                           });
          std::vector<std::vector<int>> bins;
          std::vector<uint64_t> used;
          for (const auto& [need, sp] : pack) {
            size_t b = 0;
            while (b < bins.size() && used[b] + need > pool_cap) b++;
            if (b == bins.size()) {
              bins.emplace_back();
              used.push_back(0);
            }
            bins[b].push_back(sp);
            used[b] += need;
          }
          for (auto& bin : bins) {
            std::sort(bin.begin(), bin.end());
            batches.push_back(bin);
          }
          if (stats) stats->regrown_gfds += (int32_t)pack.size();
        }
        for (int sp : solo) batches.push_back({sp});
        if (stats) stats->regrown_gfds += (int32_t)solo.size();
        // the last-level records of the jobs to re-run, as the device holds
        // them (their sources were placed by the frontier reservations)
        // (and the leaf-count records of the window jobs)
        std::vector<ExtJob> lastrec(jobs.size());
        std::vector<LeafJob> leafrec(jobs.size());
        {
          std::vector<int> xs(over);
          xs.insert(xs.end(), win.begin(), win.end());
          read_recs(c, recbase, xs, [&](int x) { return jobs[x].last_rec; }, lastrec);
          read_recs(c, recbase, win, [&](int x) { return jobs[x].leaf_rec; }, leafrec);
        }
        // jobs whose first K the last level's sort already wrote go out now
        std::unique_ptr<ResultDrain> D;
        std::vector<char> done(jobs.size(), 0);
        if (K > 0) {
          D.reset(new ResultDrain(c, jobs, results, H, K));
          std::vector<char> isover(jobs.size(), 0);
          for (int x : over) isover[x] = 1;
          for (int x : win) isover[x] = 1;
          std::vector<int> fin;
          for (size_t x = 0; x < jobs.size(); x++)
            if (!redo[x] && !isover[x] && !H[(size_t)jobs[x].spec * CTL_WORDS + CTL_NEEDSEL]) {
              fin.push_back((int)x);
              done[x] = 1;
            }
          D->issue(fin);
        }
        if (!over.empty()) {
          if (stats) stats->threshold_gfds += (int32_t)over.size();
          const Range rerun("threshold re-run");
          rerun_last_levels(c, jobs, over, lastrec, vsmall, redo, [&] { if (D) D->drain(); });
          for (int x : over)
            if (!redo[x]) {
              H[(size_t)jobs[x].spec * CTL_WORDS + CTL_VCOUNT] = ws->hctl[CTL_WORDS * x + CTL_VCOUNT];
              H[(size_t)jobs[x].spec * CTL_WORDS + CTL_NEEDSEL] = ws->hctl[CTL_WORDS * x + CTL_NEEDSEL];
            }
        }
        if (!win.empty()) {
          const Range window("first-K window");
          run_windows(c, jobs, win, leafrec, lastrec, vsmall, redo, [&] { if (D) D->drain(); });
          for (int x : win)
            if (!redo[x]) {
              H[(size_t)jobs[x].spec * CTL_WORDS + CTL_VCOUNT] = ws->hctl[CTL_WORDS * x + CTL_VCOUNT];
              H[(size_t)jobs[x].spec * CTL_WORDS + CTL_NEEDSEL] = ws->hctl[CTL_WORDS * x + CTL_NEEDSEL];
            }
        }
        // staged violations beyond one workgroup's sort: batched radix select
        if (K > 0) {
          const Range sel("violation select");
          std::vector<SelJob> S;
          for (size_t x = 0; x < jobs.size(); x++) {
            if (redo[x] || !H[(size_t)jobs[x].spec * CTL_WORDS + CTL_NEEDSEL]) continue;
            S.push_back(sel_job(c, jobs[x].plan.k, jobs[x].mem.vbuf, jobs[x].mem.ctl, vsmall));
            S.back().out = jobs[x].mem.res;
          }
          run_select(c, S, false);
          D->drain();  // while the selection runs
          std::vector<int> rest;
          for (size_t x = 0; x < jobs.size(); x++)
            if (!redo[x] && !done[x]) rest.push_back((int)x);
          D->issue(rest);
        }
        HIPCHK(hipStreamSynchronize(c.st));
        if (D) D->drain();
        if (stats)
          for (size_t x = 0; x < jobs.size(); x++) {
            if (redo[x]) continue;
            const uint64_t* h = &H[(size_t)jobs[x].spec * CTL_WORDS];
            for (int l = 1; l < MAXK; l++) {
              stats->attempts += h[CTL_LEVEL_T + l];
              if (l >= 2) stats->partials += h[CTL_LEVEL_N + l];
            }
            for (int u = 0; u < jobs[x].plan.k; u++)
              stats->cpi_candidates += h[CTL_CAND + 2 * u + jobs[x].cur[u]];
            stats->leaf_gfds += jobs[x].plan.leaf_r > 0;
            stats->leaf_split_gfds += jobs[x].plan.leaf_split;
          }
      }
      for (size_t x = 0; x < jobs.size(); x++) {
        if (redo[x] != 1) continue;
        if (stats) stats->chunked_gfds++;
        went_bounded[jobs[x].spec] = 1;
        const Range bounded("bounded re-run");
        run_bounded(c, jobs[x], vbig);
        HIPCHK(hipMemcpyAsync(&H[(size_t)jobs[x].spec * CTL_WORDS], jobs[x].mem.ctl,
                              sizeof(uint64_t) * CTL_WORDS, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        const int32_t i = jobs[x].spec;
        const uint64_t n = reported(i);
        if (K > 0 && n) {
          HIPCHK(hipMemcpyAsync(results[i].violations, jobs[x].mem.res,
                                sizeof(int32_t) * n * jobs[x].plan.k, hipMemcpyDeviceToHost, c.st));
          HIPCHK(hipStreamSynchronize(c.st));
        }
      }
    }
    // the next call with these GFDs and options: when GFDs had to leave their
    // batches (the pool or arena was at its cap), every GFD's frontier bytes
    // and CPI entries are now known exactly from its control words, so its
    // batches are formed again from them, first fit, largest first by
    // frontier bytes, within the pool and the arena (less a sixteenth for the
    // levels that reserved without attempts), the budget and the batch
    // limit; a GFD that needed the bounded path runs alone (not under a
    // frontier cap, where a GFD overflows in any batch)
    if (moved && !c.front_limit) {
      const uint64_t cap = front_usable(ws) - front_usable(ws) / 16;
      const uint64_t cpi_cap = cpi_usable(ws) - cpi_usable(ws) / 16;
      std::vector<std::vector<int>> next;
      std::vector<std::pair<uint64_t, int>> order;
      for (int32_t i = 0; i < num_specs; i++) {
        if (went_bounded[i]) next.push_back({i});
        else order.push_back({reached_front_bytes(all[i].plan, &H[(size_t)i * CTL_WORDS], 0), i});
      }
      std::stable_sort(order.begin(), order.end(),
                       [](const std::pair<uint64_t, int>& u, const std::pair<uint64_t, int>& v) {
                         return u.first > v.first;
                       });
      std::vector<std::vector<int>> bins;
      std::vector<uint64_t> fb, cb;
      std::vector<int64_t> ab;
      for (const auto& [need, i] : order) {
        const int64_t b = (int64_t)all[i].caps.bytes + 4096 * CTL_WORDS;
        const uint64_t e = H[(size_t)i * CTL_WORDS + CTL_CPIASK];
        size_t x = 0;
        while (x < bins.size() && (fb[x] + need > cap || cb[x] + e > cpi_cap || ab[x] + b > budget ||
                                   (int)bins[x].size() >= max_batch))
          x++;
        if (x == bins.size()) {
          bins.emplace_back();
          fb.push_back(0);
          cb.push_back(0);
          ab.push_back(0);
        }
        bins[x].push_back(i);
        fb[x] += need;
        cb[x] += e;
        ab[x] += b;
      }
      for (auto& bin : bins) {
        std::sort(bin.begin(), bin.end());
        next.push_back(std::move(bin));
      }
      pm->batches = std::move(next);
    }
    // the error word and the per-class bytes, through pinned memory in one wait
    ws->hmisc[1] = 0;
    HIPCHK(hipMemcpyAsync(ws->hmisc + 1, ws->err, 4, hipMemcpyDeviceToHost, c.st));
    if (stats) HIPCHK(hipMemcpyAsync(ws->hmisc + 2, ws->misc + 8, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    if ((uint32_t)ws->hmisc[1] & 1u) throw GfdError{GFD_EDEVICE, "scan look-back did not complete"};
    if ((uint32_t)ws->hmisc[1] & 2u) throw GfdError{GFD_EDEVICE, "internal: a candidate list passed its bound"};
    int32_t rc = GFD_OK;
    for (int32_t i = 0; i < num_specs; i++) {
      const uint64_t* h = &H[(size_t)i * CTL_WORDS];
      gfd_result& r = results[i];
      r.match_count = h[CTL_MATCH];
      r.violation_count = h[CTL_VIOL];
      r.match_fp = count_only ? 0 : h[CTL_MFP];  // not computed for postponed leaves
      r.violation_fp = count_only ? 0 : h[CTL_VFP];
      r.satisfied = r.violation_count == 0;
      r.num_reported = (int32_t)reported(i);  // its tuples were copied with its batch
      if ((r.match_count >> 63) || (r.violation_count >> 63) || (h[CTL_FLAGS] & FLAG_COUNTER_OVERFLOW))
        rc = set_error(GFD_EOVERFLOW, "spec %d: counter passed 2^63", i);
    }
    if (stats) {
      for (int j = 0; j < 8; j++) stats->class_bytes[j] = ws->hmisc[2 + j];
      stats->cpi_entries = cpi_entries;
      stats->units_counted = units_counted() ? 1 : 0;
      units_read(c.st, stats->units);
      stats->batches = (int32_t)batches.size();
      stats->front_pool_bytes = (int64_t)ws->front_bytes;
      stats->cpi_arena_bytes = (int64_t)ws->cpi_cap * 4;
      if (c.tm.on) c.tm.collect(stats->class_ms);
      for (int j = 0; j < 8; j++) {
        stats->class_launches[j] = c.tm.launches[j];
        stats->launches += c.tm.launches[j];
      }
      stats->wall_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    ws->hitpool_dirty = false;
    if (!fixed) release_ws(g, ws);
    return rc;
  } catch (...) {
    if (ws && !fixed) release_ws(g, ws);
    return guarded([] () -> int32_t { throw; });
  }
}

extern "C" int32_t gfd_validate_ex(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                                   const gfd_validate_opts* opts, gfd_result* results,
                                   gfd_stats* stats) {
  return validate_impl(g, specs, num_specs, opts, results, stats, nullptr);
}

// ---------------------------------------------------------------------------
// the entry point that allocates nothing
// ---------------------------------------------------------------------------

// Every device byte of gfd_validate_noalloc's workspace is carved from this
// array (one copy per device the library runs on, held until the process
// ends).  Host code never uses its name as an address: the device address of
// each device's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[GFD_NOALLOC_SCRATCH_BYTES];

namespace {
struct NoAllocDevice {
  std::mutex mu;            // calls on one device share its scratch: one at a time
  uint8_t* ptr = nullptr;   // device address of this device's scratch
  Workspace* ws = nullptr;  // host state of those calls (pageable host staging)
};
std::mutex g_noalloc_mu;
std::unordered_map<int, NoAllocDevice*> g_noalloc;  // by device, never freed

NoAllocDevice* noalloc_device(int dev) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  NoAllocDevice*& d = g_noalloc[dev];
  if (!d) d = new NoAllocDevice();
  return d;
}
}  // namespace

extern "C" int32_t gfd_validate_noalloc(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                                        const gfd_validate_opts* opts, gfd_result* results) {
  if (!g) return set_error(GFD_EINVAL, "graph is NULL");
  gfd_validate_opts o{};
  o.k_max = 1024;
  o.semantics = GFD_SEM_INDUCED;
  if (opts) o = *opts;
  if (o.flags & ~(GFD_FLAG_FORCE_CHUNKED | GFD_FLAG_COUNT_ONLY))
    return set_error(GFD_EINVAL, "timing flags need events, which this entry point does not create");
  if (o.allocator.alloc) return set_error(GFD_EINVAL, "this entry point takes no allocator");
  if (o.mem_budget_bytes < 0) return set_error(GFD_EINVAL, "negative option");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GFD_EDEVICE, "no current device");
  }
  if (dev != g->device) return set_error(GFD_EINVAL, "the graph lives on device %d, not the current %d", g->device, dev);
  NoAllocDevice* d = noalloc_device(dev);
  std::lock_guard<std::mutex> lk(d->mu);
  return guarded([&] {
    if (!d->ptr) {  // once per device, with that device current
      void* p = nullptr;
      HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      d->ptr = (uint8_t*)p;
    }
    if (!d->ws) {
      d->ws = new Workspace();
      d->ws->pageable = true;
    }
    Workspace* w = d->ws;
    // every call carves the area again from its start; what must start at
    // zero is cleared on the call's stream
    w->forget_device_buffers();
    w->al.area = d->ptr;
    w->al.area_cap = (size_t)GFD_NOALLOC_SCRATCH_BYTES;
    w->al.st = (hipStream_t)o.hip_stream;
    // half of the area for the batches' candidate structures; the rest holds
    // the fixed buffers, records, frontier pool, CPI arena and staging
    const int64_t half = (int64_t)GFD_NOALLOC_SCRATCH_BYTES / 2;
    w->budget = o.mem_budget_bytes ? std::min<int64_t>(o.mem_budget_bytes, half) : half;
    init_ws_buffers(w, (hipStream_t)o.hip_stream);
    w->area_mark = w->al.area_top;
    return validate_impl(g, specs, num_specs, &o, results, nullptr, w);
  });
}

extern "C" int32_t gfd_validate(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                                const gfd_validate_opts* opts, gfd_result* results) {
  return gfd_validate_ex(g, specs, num_specs, opts, results, nullptr);
}

// ---------------------------------------------------------------------------
// serving: a resident graph, a request queue and worker threads that batch
// whatever is waiting whenever they are free (continuous batching)
// ---------------------------------------------------------------------------

struct gfd_server {
  gfd_graph* g = nullptr;
  gfd_server_opts o{};
  int64_t budget = 0;  // per worker
  ServeQueue q;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  void work(int w) {
    (void)hipSetDevice(g->device);
    std::vector<ServerReq*> batch;
    uint64_t bid = 0;
    while (q.take(o.max_batch_gfds, budget, batch, bid)) {
      const int64_t t_start = serve_now_ns();
      const Range batch_range("server batch");
      std::vector<gfd_spec> specs;
      std::vector<gfd_result> res;
      for (ServerReq* r : batch) {
        specs.insert(specs.end(), r->specs.begin(), r->specs.end());
        for (size_t i = 0; i < r->specs.size(); i++) {
          gfd_result x{};
          x.violations = r->viol.data() + i * (size_t)std::max(o.k_max, 1) * GFD_MAX_K;
          res.push_back(x);
        }
      }
      gfd_validate_opts vo{};
      vo.k_max = o.k_max;
      vo.semantics = o.semantics;
      vo.mem_budget_bytes = budget;
      vo.hip_stream = streams[w];
      vo.batched = 1;
      vo.allocator = o.allocator;
      vo.flags = GFD_FLAG_NO_GRAPH;  // a serving mix rarely repeats a batch's shape
      const int32_t rc = gfd_validate(g, specs.data(), (int32_t)specs.size(), &vo, res.data());
      std::vector<int32_t> st(batch.size(), rc);
      std::vector<std::string> msg(batch.size(), rc ? gfd_last_error() : "");
      if (rc && batch.size() > 1) {
        // the batch failed: each request alone, so only a failing one reports it
        size_t at = 0;
        for (size_t b = 0; b < batch.size(); b++) {
          const int32_t nb = (int32_t)batch[b]->specs.size();
          st[b] = gfd_validate(g, specs.data() + at, nb, &vo, res.data() + at);
          msg[b] = st[b] ? gfd_last_error() : "";
          at += (size_t)nb;
        }
      }
      const int64_t t_done = serve_now_ns();
      std::vector<size_t> first(batch.size(), 0);
      for (size_t b = 1; b < batch.size(); b++) first[b] = first[b - 1] + batch[b - 1]->specs.size();
      q.publish(batch, [&](size_t b, ServerReq& r) {
        for (size_t i = 0; i < r.specs.size(); i++) r.res[i] = res[first[b] + i];
        r.status = st[b];
        r.err = msg[b];
        r.info.start_ns = t_start;
        r.info.done_ns = t_done;
        r.info.batch_id = bid;
        r.info.batch_gfds = (int32_t)specs.size();
        r.info.batch_requests = (int32_t)batch.size();
        r.info.worker = w;
      });
    }
  }
};

extern "C" int32_t gfd_server_create(const gfd_graph* gc, const gfd_server_opts* opts,
                                     gfd_server** out) {
  if (!out) return set_error(GFD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!gc) return set_error(GFD_EINVAL, "graph is NULL");
  gfd_server_opts o{};
  o.workers = 2;
  o.max_batch_gfds = MAX_JOBS;
  o.k_max = 1024;
  o.semantics = GFD_SEM_INDUCED;
  if (opts) o = *opts;
  if (o.workers == 0) o.workers = 2;
  if (o.max_batch_gfds == 0) o.max_batch_gfds = MAX_JOBS;
  if (o.workers < 1 || o.workers > 8) return set_error(GFD_EINVAL, "workers must be 1..8");
  if (o.max_batch_gfds < 1 || o.max_batch_gfds > MAX_JOBS)
    return set_error(GFD_EINVAL, "max_batch_gfds must be 1..%d", MAX_JOBS);
  if (o.k_max < 0 || o.k_max > SORT_MAX) return set_error(GFD_EINVAL, "k_max");
  if (o.semantics != GFD_SEM_INDUCED && o.semantics != GFD_SEM_MONO) return set_error(GFD_EINVAL, "semantics");
  if (o.mem_budget_bytes < 0) return set_error(GFD_EINVAL, "negative budget");
  if (int32_t rc = check_allocator(o.allocator)) return rc;
  gfd_server* s = new gfd_server();
  s->g = const_cast<gfd_graph*>(gc);
  s->o = o;
  try {
    HIPCHK(hipSetDevice(s->g->device));
    if (o.mem_budget_bytes) {
      s->budget = o.mem_budget_bytes;
    } else {  // the workers share what the default budget of one call would take
      s->budget = std::max<int64_t>(int64_t(256) << 20, default_budget() / o.workers);
    }
    for (int w = 0; w < o.workers; w++) {
      hipStream_t st = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->streams.push_back(st);
    }
    // one workspace per worker, its batch arena reserved up front for a full
    // batch of the largest patterns (8 wildcard vertices on a path), within the
    // budget: growing it while serving would stall a batch for seconds
    int64_t reserve = 0;
    {
      gfd_spec path{};
      path.num_vertices = MAXK;
      for (int i = 0; i < MAXK; i++) path.vertex_labels[i] = GFD_WILDCARD;
      path.num_edges = MAXK - 1;
      for (int i = 0; i + 1 < MAXK; i++) path.edges[i] = gfd_edge{i, i + 1, GFD_WILDCARD};
      const Sizing sz = call_sizing(s->budget, o.max_batch_gfds, o.max_batch_gfds, o.k_max, 0);
      Plan p;
      make_plan(s->g, path, o.semantics == GFD_SEM_INDUCED, p);
      plan_leaves(path, o.semantics == GFD_SEM_INDUCED, false, 0, p);
      JobCaps caps;
      job_caps(s->g, p, 0, sz.vsmall, false, caps);
      reserve = std::min<int64_t>(s->budget, (int64_t)o.max_batch_gfds * (int64_t)align_up(caps.bytes) +
                                                 (int64_t(64) << 20));
    }
    std::vector<Workspace*> ws;
    try {
      for (int w = 0; w < o.workers; w++) {
        ws.push_back(acquire_ws(s->g, s->budget, o.allocator, s->streams[w]));
        ensure_arena(ws.back(), (size_t)reserve);
        // and a frontier pool of an eighth of the budget (at most 1 GiB)
        ws.back()->front_want =
            std::max(ws.back()->front_want, (size_t)std::min<int64_t>(s->budget / 8, int64_t(1) << 30));
        ensure_front(ws.back());
      }
    } catch (...) {
      for (Workspace* x : ws) release_ws(s->g, x);
      throw;
    }
    for (Workspace* x : ws) release_ws(s->g, x);
    for (int w = 0; w < o.workers; w++) s->workers.emplace_back([s, w] { s->work(w); });
  } catch (...) {
    // stop and join the workers already started, then report
    s->q.shutdown();
    for (auto& t : s->workers)
      if (t.joinable()) t.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return guarded([] () -> int32_t { throw; });
  }
  *out = s;
  return GFD_OK;
}

extern "C" int32_t gfd_server_submit(gfd_server* s, const gfd_spec* specs, int32_t num_specs,
                                     uint64_t* request_id) {
  if (!s || !request_id || num_specs < 1 || !specs) return set_error(GFD_EINVAL, "server/specs/id");
  if (num_specs > s->o.max_batch_gfds)
    return set_error(GFD_EINVAL, "request of %d GFDs exceeds max_batch_gfds", num_specs);
  std::unique_ptr<ServerReq> rp(new ServerReq());
  ServerReq* r = rp.get();
  try {
    const bool induced = s->o.semantics == GFD_SEM_INDUCED;
    // estimated device bytes of the request's jobs, sized as in a full batch
    const Sizing sz = call_sizing(s->budget, s->o.max_batch_gfds, s->o.max_batch_gfds, s->o.k_max, 0);
    for (int32_t i = 0; i < num_specs; i++) {
      const int32_t rc = check_spec(s->g, specs[i], i);
      if (rc) return rc;
      Plan p;
      make_plan(s->g, specs[i], induced, p);
      plan_leaves(specs[i], induced, false, 0, p);
      JobCaps caps;
      job_caps(s->g, p, 0, sz.vsmall, false, caps);
      // its candidate and CPI structures, staging and estimated frontiers
      r->est_bytes += (int64_t)caps.bytes +
                      (int64_t)std::min<uint64_t>(est_front_bytes(s->g, p), (uint64_t)s->budget / 4);
    }
    r->specs.assign(specs, specs + num_specs);
    r->res.resize(num_specs);
    r->viol.resize((size_t)num_specs * std::max(s->o.k_max, 1) * GFD_MAX_K);
    if (s->q.submit(r, request_id) != ServeQueue::OK) return set_error(GFD_EINVAL, "server is stopping");
    rp.release();
  } catch (...) {
    return guarded([] () -> int32_t { throw; });
  }
  return GFD_OK;
}

extern "C" int32_t gfd_server_wait(gfd_server* s, uint64_t request_id, int32_t timeout_ms,
                                   gfd_result* results, gfd_request_info* info) {
  if (!s) return set_error(GFD_EINVAL, "server is NULL");
  ServerReq* r = nullptr;
  switch (s->q.wait(request_id, timeout_ms, r)) {
    case ServeQueue::OK:
      break;
    case ServeQueue::UNKNOWN:
      return set_error(GFD_EINVAL, "unknown request %llu", (unsigned long long)request_id);
    case ServeQueue::CLAIMED:
      return set_error(GFD_EINVAL, "request %llu is being waited for", (unsigned long long)request_id);
    default:
      return set_error(GFD_EAGAIN, "request %llu not finished", (unsigned long long)request_id);
  }
  const int32_t rc = r->status;
  if (rc) set_error(rc, "%s", r->err.c_str());
  if (!rc && results) {
    const int K = s->o.k_max;
    for (size_t i = 0; i < r->specs.size(); i++) {
      int32_t* dst = results[i].violations;
      results[i] = r->res[i];
      results[i].violations = dst;
      if (K > 0 && dst && r->res[i].num_reported)
        std::memcpy(dst, r->res[i].violations,
                    sizeof(int32_t) * r->res[i].num_reported * r->specs[i].num_vertices);
    }
  }
  if (info) *info = r->info;
  delete r;
  return rc;
}

extern "C" void gfd_server_destroy(gfd_server* s) {
  if (!s) return;
  s->q.shutdown();
  for (auto& t : s->workers) t.join();
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;  // and the requests nobody waited for
}
