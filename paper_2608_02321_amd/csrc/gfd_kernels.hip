// HIP kernels (gfx950, wave64) for GFD validation:
//   - single-pass exclusive scans (decoupled look-back),
//   - candidate filtering with ballot/mbcnt stream compaction,
//   - Compact Path Index construction (top-down / bottom-up marking, CPI
//     adjacency lists per spanning-tree edge),
//   - level-synchronous embedding enumeration over the CPI with load-balanced
//     search over candidate lists, injectivity, non-tree edge and induced
//     non-edge probes, and the X -> Y literal check fused into the last level,
//   - exact lexicographic first-K selection of violating tuples.
// FastGFDs paper, Section IV-B (CPI, core-first matching) and Section II
// (definitions).  All arithmetic is integer.
#include "gfd_internal.h"

namespace gfd {

// ---------------------------------------------------------------------------
// wave and block helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Binary search in one sorted adjacency row: label of the edge to `v`, or NOEDGE.
__device__ __forceinline__ int32_t probe(const uint32_t* __restrict__ off,
                                         const int32_t* __restrict__ nbr,
                                         const int32_t* __restrict__ lab, int32_t u, int32_t v) {
  uint32_t lo = off[u], hi = off[u + 1];
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (nbr[mid] < v) lo = mid + 1; else hi = mid;
  }
  return (lo < off[u + 1] && nbr[lo] == v) ? lab[lo] : NOEDGE;
}

__device__ __forceinline__ bool constraint_ok(int32_t found, int32_t code) {
  if (code == PC_FREE) return true;
  if (code == PC_ABSENT) return found == NOEDGE;
  return found != NOEDGE && (code == ANY || found == code);
}

// ---------------------------------------------------------------------------
// single-pass exclusive scan of u32 items into u64 prefixes
// ---------------------------------------------------------------------------

constexpr uint64_t VAL_MASK = (1ull << 46) - 1;
__device__ __forceinline__ uint64_t pack_state(uint32_t ep, uint32_t flag, uint64_t v) {
  return ((uint64_t)(ep & 0xFFFFu) << 48) | ((uint64_t)flag << 46) | (v & VAL_MASK);
}

struct FnRowLen {
  const int32_t* list;
  const uint32_t* off;
  __device__ uint32_t operator()(uint64_t i) const {
    int32_t v = list[i];
    return off[v + 1] - off[v];
  }
};
struct FnPopc {
  const uint64_t* masks;
  __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)__popcll(masks[i]); }
};
struct FnSrc {
  const int32_t* par;
  const int32_t* pos;
  const uint32_t* cpi_off;
  uint32_t* beg;
  __device__ uint32_t operator()(uint64_t i) const {
    int32_t c = pos[par[i]];
    uint32_t b = cpi_off[c];
    beg[i] = b;
    return cpi_off[c + 1] - b;
  }
};

// Tiles are handed out by an atomic ticket, so a tile only ever waits on
// tiles already owned by running blocks; the waits are bounded and report an
// error instead of hanging.
template <class F>
__global__ __launch_bounds__(BS) void k_scan(F f, const uint64_t* __restrict__ d_n, uint64_t cap,
                                             int per_word, uint64_t* __restrict__ out,
                                             uint64_t* __restrict__ d_total,
                                             uint64_t* __restrict__ state, uint32_t* ticket,
                                             uint32_t epoch, uint32_t* err) {
  uint64_t N = *d_n < cap ? *d_n : cap;
  if (per_word) N = (N + 63) / 64;
  const uint64_t ntiles = (N + SCAN_TILE - 1) / SCAN_TILE;
  __shared__ uint32_t s_t;
  __shared__ uint64_t s_pre;
  __shared__ uint64_t s_w[BS / WAVE];
  const uint32_t ln = lane(), wv = threadIdx.x / WAVE;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint64_t t = s_t;
    if (t >= ntiles) {
      if (threadIdx.x == 0 && t == ntiles + gridDim.x - 1) {
        if (ntiles == 0) {
          out[0] = 0;
          *d_total = 0;
        }
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    const uint64_t base = t * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; j++) {
      v[j] = (base + j < N) ? f(base + j) : 0u;
      sum += v[j];
    }
    uint64_t x = sum;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      uint64_t y = __shfl_up(x, (unsigned)d);
      if (ln >= (uint32_t)d) x += y;
    }
    if (ln == WAVE - 1) s_w[wv] = x;
    __syncthreads();
    uint64_t wpre = 0, agg = 0;
#pragma unroll
    for (int w = 0; w < BS / WAVE; w++) {
      if ((uint32_t)w < wv) wpre += s_w[w];
      agg += s_w[w];
    }
    if (threadIdx.x == 0) {
      uint64_t prefix = 0;
      if (t == 0) {
        __hip_atomic_store(&state[0], pack_state(epoch, 2, agg), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&state[t], pack_state(epoch, 1, agg), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        int64_t j = (int64_t)t - 1;
        uint32_t spins = 0;
        while (j >= 0) {
          uint64_t w = __hip_atomic_load(&state[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          uint32_t ep = (uint32_t)(w >> 48), fl = (uint32_t)(w >> 46) & 3u;
          if (ep != (epoch & 0xFFFFu) || fl == 0) {
            if (++spins > (1u << 24)) {
              atomicOr(err, 1u);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          prefix += w & VAL_MASK;
          if (fl == 2) break;
          j--;
        }
        __hip_atomic_store(&state[t], pack_state(epoch, 2, prefix + agg), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      s_pre = prefix;
    }
    __syncthreads();
    uint64_t run = s_pre + wpre + x - sum;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; j++) {
      if (base + j < N) {
        out[base + j] = run;
        run += v[j];
      }
    }
    if (t == ntiles - 1 && threadIdx.x == BS - 1) {
      out[N] = s_pre + agg;
      *d_total = s_pre + agg;
    }
  }
}

template <class F>
static void launch_scan(hipStream_t st, ScanWs& ws, F f, const uint64_t* d_n, uint64_t cap,
                        int per_word, uint64_t* out, uint64_t* d_total) {
  uint64_t items = per_word ? (cap + 63) / 64 : cap;
  uint64_t tiles = (items + SCAN_TILE - 1) / SCAN_TILE;
  int grid = (int)(tiles < 1 ? 1 : (tiles > 512 ? 512 : tiles));
  ws.epoch = (ws.epoch + 1) & 0xFFFFu;
  if (ws.epoch == 0) {  // wrapped: stale tile states could alias the new epoch
    fill_u64(st, ws.tile_state, 0, ws.max_tiles);
    ws.epoch = 1;
  }
  hipLaunchKernelGGL(k_scan<F>, dim3(grid), dim3(BS), 0, st, f, d_n, cap, per_word, out, d_total,
                     ws.tile_state, ws.ticket, ws.epoch, ws.err);
}

void scan_row_lengths(hipStream_t st, ScanWs& ws, const int32_t* list, const uint64_t* d_n,
                      uint64_t cap, const uint32_t* off, uint64_t* P, uint64_t* d_total) {
  launch_scan(st, ws, FnRowLen{list, off}, d_n, cap, 0, P, d_total);
}
void scan_popcounts(hipStream_t st, ScanWs& ws, const uint64_t* masks, const uint64_t* d_n,
                    uint64_t cap, uint64_t* pre, uint64_t* d_total) {
  launch_scan(st, ws, FnPopc{masks}, d_n, cap, 1, pre, d_total);
}
void scan_sources(hipStream_t st, ScanWs& ws, const int32_t* par_col, const uint64_t* d_n,
                  uint64_t cap, const int32_t* pos_map, const uint32_t* cpi_off, uint32_t* beg,
                  uint64_t* P, uint64_t* d_total) {
  launch_scan(st, ws, FnSrc{par_col, pos_map, cpi_off, beg}, d_n, cap, 0, P, d_total);
}

// ---------------------------------------------------------------------------
// load-balanced search: map a tile of flat work positions to (source, offset)
// ---------------------------------------------------------------------------

constexpr int LBS_SLOTS = BS + 1 + 63;
struct LbsShared {
  uint64_t p[LBS_SLOTS];
  uint64_t lo, hi;
};

// largest s in [lo, hi] with P[s] <= a (P non-decreasing, P[lo] <= a)
__device__ __forceinline__ uint64_t last_le(const uint64_t* __restrict__ P, uint64_t lo,
                                            uint64_t hi, uint64_t a) {
  while (lo < hi) {
    uint64_t mid = (lo + hi + 1) >> 1;
    if (P[mid] <= a) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Every thread of the block must call this with the same (t0, t1), t0 < t1.
__device__ __forceinline__ bool lbs_tile(const uint64_t* __restrict__ P, uint64_t N, uint64_t t0,
                                         uint64_t t1, LbsShared& sh, uint64_t& s, uint64_t& off) {
  if (threadIdx.x == 0) sh.lo = last_le(P, 0, N - 1, t0);
  if (threadIdx.x == 1) sh.hi = last_le(P, 0, N - 1, t1 - 1);
  __syncthreads();
  const uint64_t lo = sh.lo, hi = sh.hi;
  const uint64_t span = hi - lo + 2;  // P[lo .. hi+1]
  const bool in_lds = span <= (uint64_t)LBS_SLOTS;
  if (in_lds)
    for (uint64_t j = threadIdx.x; j < span; j += BS) sh.p[j] = P[lo + j];
  __syncthreads();
  const uint64_t a = t0 + threadIdx.x;
  bool valid = a < t1;
  if (valid) {
    if (in_lds) {
      uint32_t l = 0, h = (uint32_t)(span - 2);
      while (l < h) {
        uint32_t mid = (l + h + 1) >> 1;
        if (sh.p[mid] <= a) l = mid; else h = mid - 1;
      }
      s = lo + l;
      off = a - sh.p[l];
    } else {
      s = last_le(P, lo, hi, a);
      off = a - P[s];
    }
  }
  __syncthreads();
  return valid;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_fill(T* p, T v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BS)
    p[i] = v;
}
template <class T>
static void fill(hipStream_t st, T* p, T v, uint64_t n) {
  if (n == 0) return;
  uint64_t b = (n + BS - 1) / BS;
  int grid = (int)(b > 2048 ? 2048 : b);
  hipLaunchKernelGGL(k_fill<T>, dim3(grid), dim3(BS), 0, st, p, v, n);
}
void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, uint64_t n) { fill(st, p, v, n); }
void fill_u64(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n) { fill(st, p, v, n); }
void fill_u32(hipStream_t st, uint32_t* p, uint32_t v, uint64_t n) { fill(st, p, v, n); }

// ---------------------------------------------------------------------------
// candidate filter: label bucket (or list) -> flags -> compaction
// (Section IV-B: label candidates and the degree filter)
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool filter_pass(const FilterArgs& a, int32_t v) {
  if (a.min_out > 0 && (int64_t)(a.g.out_off[v + 1] - a.g.out_off[v]) < a.min_out) return false;
  if (a.min_in > 0 && (int64_t)(a.g.in_off[v + 1] - a.g.in_off[v]) < a.min_in) return false;
  for (int j = 0; j < a.nmarks; j++)
    if (a.marks[j][v] != a.mark_ep[j]) return false;
  return true;
}

__global__ __launch_bounds__(BS) void k_filter_flags(FilterArgs a) {
  const uint64_t N = a.d_n ? (*a.d_n < a.cap ? *a.d_n : a.cap) : a.n_host;
  const uint64_t nw = (N + 63) / 64;
  const uint64_t wid = ((uint64_t)blockIdx.x * BS + threadIdx.x) / WAVE;
  const uint64_t nwv = (uint64_t)gridDim.x * BS / WAVE;
  for (uint64_t w = wid; w < nw; w += nwv) {
    const uint64_t i = w * 64 + lane();
    bool f = false;
    if (i < N) f = filter_pass(a, a.list ? a.list[i] : (int32_t)i);
    const uint64_t m = __ballot(f);
    if (lane() == 0) a.masks[w] = m;
  }
}

__global__ __launch_bounds__(BS) void k_filter_emit(FilterArgs a, const uint64_t* __restrict__ pre,
                                                    int32_t* __restrict__ out, uint8_t* mem,
                                                    uint8_t mem_ep) {
  const uint64_t N = a.d_n ? (*a.d_n < a.cap ? *a.d_n : a.cap) : a.n_host;
  const uint64_t nw = (N + 63) / 64;
  const uint64_t wid = ((uint64_t)blockIdx.x * BS + threadIdx.x) / WAVE;
  const uint64_t nwv = (uint64_t)gridDim.x * BS / WAVE;
  for (uint64_t w = wid; w < nw; w += nwv) {
    const uint64_t i = w * 64 + lane();
    const uint64_t m = a.masks[w];
    if (i < N && ((m >> lane()) & 1ull)) {
      const int32_t v = a.list ? a.list[i] : (int32_t)i;
      out[pre[w] + rank_below(m)] = v;
      if (mem) mem[v] = mem_ep;
    }
  }
}

void filter_flags(hipStream_t st, const FilterArgs& a, int grid) {
  hipLaunchKernelGGL(k_filter_flags, dim3(grid), dim3(BS), 0, st, a);
}
void filter_emit(hipStream_t st, const FilterArgs& a, const uint64_t* pre, int32_t* out,
                 uint8_t* mem, uint8_t mem_ep, int grid) {
  hipLaunchKernelGGL(k_filter_emit, dim3(grid), dim3(BS), 0, st, a, pre, out, mem, mem_ep);
}

// ---------------------------------------------------------------------------
// CPI marking (Section IV-B: BFS candidate subgraph and dead-end removal)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BS) void k_mark(DevGraph g, int dir, const int32_t* __restrict__ list,
                                             const uint64_t* __restrict__ d_n, uint64_t cap,
                                             const uint64_t* __restrict__ P,
                                             const uint64_t* __restrict__ d_total,
                                             uint64_t total_cap, int32_t elab, int32_t vlab,
                                             uint8_t* __restrict__ mark, uint8_t ep) {
  __shared__ LbsShared sh;
  const uint64_t N = *d_n < cap ? *d_n : cap;
  const uint64_t T = *d_total < total_cap ? *d_total : total_cap;
  const uint32_t* off = dir ? g.in_off : g.out_off;
  const int32_t* nbr = dir ? g.in_nbr : g.out_nbr;
  const int32_t* lab = dir ? g.in_lab : g.out_lab;
  for (uint64_t t0 = (uint64_t)blockIdx.x * BS; t0 < T; t0 += (uint64_t)gridDim.x * BS) {
    const uint64_t t1 = t0 + BS < T ? t0 + BS : T;
    uint64_t s, o;
    if (lbs_tile(P, N, t0, t1, sh, s, o)) {
      const uint32_t e = off[list[s]] + (uint32_t)o;
      const int32_t v = nbr[e];
      if ((elab == ANY || lab[e] == elab) && (vlab == ANY || g.vlab[v] == vlab)) mark[v] = ep;
    }
  }
}

void mark_rows(hipStream_t st, const DevGraph& g, int dir, const int32_t* list,
               const uint64_t* d_n, uint64_t cap, const uint64_t* P, const uint64_t* d_total,
               uint64_t total_cap, int32_t elab, int32_t vlab, uint8_t* mark, uint8_t ep,
               int grid) {
  hipLaunchKernelGGL(k_mark, dim3(grid), dim3(BS), 0, st, g, dir, list, d_n, cap, P, d_total,
                     total_cap, elab, vlab, mark, ep);
}

// ---------------------------------------------------------------------------
// CPI adjacency N_u^p(v_p) for a spanning-tree edge (p, u)
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool adj_keep(const AdjArgs& a, uint64_t s, uint64_t o, int32_t& v) {
  const DevGraph& g = a.g;
  const int32_t vp = a.list[s];
  const uint32_t* off = a.dir ? g.in_off : g.out_off;
  const int32_t* nbr = a.dir ? g.in_nbr : g.out_nbr;
  const int32_t* lab = a.dir ? g.in_lab : g.out_lab;
  const uint32_t e = off[vp] + (uint32_t)o;
  v = nbr[e];
  if (a.mem[v] != a.ep) return false;
  if (a.prim != ANY && lab[e] != a.prim) return false;
  if (a.other == PC_FREE) return true;
  // reverse direction: scanned out-row (vp -> v) => look for v in vp's in-row
  const int32_t r = a.dir ? probe(g.out_off, g.out_nbr, g.out_lab, vp, v)
                          : probe(g.in_off, g.in_nbr, g.in_lab, vp, v);
  return constraint_ok(r, a.other);
}

__global__ __launch_bounds__(BS) void k_adj_flags(AdjArgs a) {
  __shared__ LbsShared sh;
  const uint64_t N = *a.d_n < a.cap ? *a.d_n : a.cap;
  const uint64_t T = *a.d_total < a.total_cap ? *a.d_total : a.total_cap;
  for (uint64_t t0 = (uint64_t)blockIdx.x * BS; t0 < T; t0 += (uint64_t)gridDim.x * BS) {
    const uint64_t t1 = t0 + BS < T ? t0 + BS : T;
    uint64_t s, o;
    int32_t v;
    bool f = false;
    if (lbs_tile(a.P, N, t0, t1, sh, s, o)) f = adj_keep(a, s, o, v);
    const uint64_t m = __ballot(f);
    const uint64_t w = (t0 + threadIdx.x) / 64;
    if (lane() == 0 && t0 + threadIdx.x < T) a.masks[w] = m;
  }
}

__global__ __launch_bounds__(BS) void k_adj_emit(AdjArgs a, const uint64_t* __restrict__ pre,
                                                 int32_t* __restrict__ ent) {
  __shared__ LbsShared sh;
  const uint64_t N = *a.d_n < a.cap ? *a.d_n : a.cap;
  const uint64_t T = *a.d_total < a.total_cap ? *a.d_total : a.total_cap;
  const DevGraph& g = a.g;
  const uint32_t* off = a.dir ? g.in_off : g.out_off;
  const int32_t* nbr = a.dir ? g.in_nbr : g.out_nbr;
  for (uint64_t t0 = (uint64_t)blockIdx.x * BS; t0 < T; t0 += (uint64_t)gridDim.x * BS) {
    const uint64_t t1 = t0 + BS < T ? t0 + BS : T;
    uint64_t s, o;
    if (lbs_tile(a.P, N, t0, t1, sh, s, o)) {
      const uint64_t pos = t0 + threadIdx.x, w = pos / 64;
      const uint64_t m = a.masks[w];
      if ((m >> lane()) & 1ull) ent[pre[w] + rank_below(m)] = nbr[off[a.list[s]] + (uint32_t)o];
    }
  }
}

__global__ __launch_bounds__(BS) void k_adj_offsets(AdjArgs a, const uint64_t* __restrict__ pre,
                                                    uint32_t* __restrict__ cpi_off) {
  const uint64_t N = *a.d_n < a.cap ? *a.d_n : a.cap;
  for (uint64_t s = (uint64_t)blockIdx.x * BS + threadIdx.x; s <= N;
       s += (uint64_t)gridDim.x * BS) {
    const uint64_t p = a.P[s], w = p / 64, b = p % 64;
    uint64_t r = pre[w];
    if (b) r += (uint64_t)__popcll(a.masks[w] & ((1ull << b) - 1));
    cpi_off[s] = (uint32_t)r;
  }
}

__global__ __launch_bounds__(BS) void k_pos_map(const int32_t* __restrict__ list,
                                                const uint64_t* __restrict__ d_n, uint64_t cap,
                                                int32_t* __restrict__ pos) {
  const uint64_t N = *d_n < cap ? *d_n : cap;
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < N; i += (uint64_t)gridDim.x * BS)
    pos[list[i]] = (int32_t)i;
}

void adj_flags(hipStream_t st, const AdjArgs& a, int grid) {
  hipLaunchKernelGGL(k_adj_flags, dim3(grid), dim3(BS), 0, st, a);
}
void adj_emit(hipStream_t st, const AdjArgs& a, const uint64_t* pre, int32_t* ent, int grid) {
  hipLaunchKernelGGL(k_adj_emit, dim3(grid), dim3(BS), 0, st, a, pre, ent);
}
void adj_offsets(hipStream_t st, const AdjArgs& a, const uint64_t* pre, uint32_t* cpi_off,
                 int grid) {
  hipLaunchKernelGGL(k_adj_offsets, dim3(grid), dim3(BS), 0, st, a, pre, cpi_off);
}
void pos_map(hipStream_t st, const int32_t* list, const uint64_t* d_n, uint64_t cap, int32_t* pos,
             int grid) {
  hipLaunchKernelGGL(k_pos_map, dim3(grid), dim3(BS), 0, st, list, d_n, cap, pos);
}

// ---------------------------------------------------------------------------
// enumeration (Section IV-B matching over the CPI) with the fused literal
// check (Section II: h |= X implies h |= Y)
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ int32_t pick(const int32_t (&h)[N], int idx) {
  int32_t r = h[0];
#pragma unroll
  for (int j = 1; j < N; j++)
    if (j == idx) r = h[j];
  return r;
}

__device__ __forceinline__ bool literal_holds(const ExtArgs& a, const DevLit& l,
                                              const int32_t (&h)[MAXK]) {
  const int32_t x = a.g.attr[(int64_t)l.attr * a.g.n + pick(h, l.pos)];
  if (l.kind == 0) return x != ABSENT && x == l.value;
  const int32_t y = a.g.attr[(int64_t)l.attr2 * a.g.n + pick(h, l.pos2)];
  return x != ABSENT && y != ABSENT && x == y;
}

struct FinalAcc {
  unsigned long long match, viol, mfp, vfp;
};

// One complete match h (matching order).  Counts it, checks X -> Y, and stages
// a violation if it precedes the current threshold.  Returns whether a tuple
// must be staged; `t` then holds it in variable order.
__device__ __forceinline__ bool finalize(const ExtArgs& a, const int32_t (&h)[MAXK],
                                         int32_t (&t)[MAXK], FinalAcc& acc, bool thr_on,
                                         const int32_t (&thr)[MAXK]) {
  uint64_t hs = 0x9E3779B97F4A7C15ull * (uint64_t)a.k;
#pragma unroll
  for (int v = 0; v < MAXK; v++) {
    t[v] = pick(h, a.var_pos[v]);
    if (v < a.k) hs = mix64(hs ^ (uint64_t)(uint32_t)t[v]);
  }
  bool X = true, Y = !a.y_false;
  for (int j = 0; j < a.nx; j++) X = X && literal_holds(a, a.lit[j], h);
  if (X && Y)
    for (int j = 0; j < a.ny; j++) Y = Y && literal_holds(a, a.lit[a.nx + j], h);
  acc.match += 1;
  acc.mfp += hs;
  if (!(X && !Y)) return false;
  acc.viol += 1;
  acc.vfp += hs;
  if (a.vcap == 0) return false;
  if (thr_on) {
    // stage only if t < thr lexicographically (unsigned ids)
    int c = 0;
#pragma unroll
    for (int v = 0; v < MAXK; v++)
      if (c == 0 && v < a.k) {
        uint32_t x = (uint32_t)t[v], y = (uint32_t)thr[v];
        c = x < y ? -1 : (x > y ? 1 : 0);
      }
    if (c >= 0) return false;
  }
  return true;
}

__device__ __forceinline__ void stage(const ExtArgs& a, bool want, const int32_t (&t)[MAXK]) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if ((int)lane() == leader) base = atomicAdd((unsigned long long*)a.d_vcount, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (want) {
    const uint64_t slot = base + rank_below(m);
    if (slot < a.vcap) {
      int32_t* dst = a.vbuf + slot * (uint64_t)a.k;
#pragma unroll
      for (int v = 0; v < MAXK; v++)
        if (v < a.k) dst[v] = t[v];
    } else {
      atomicOr(a.d_flags, 2u);
    }
  }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

__device__ __forceinline__ void flush_acc(const ExtArgs& a, FinalAcc acc) {
  __shared__ unsigned long long s_acc[4][BS / WAVE];
  acc.match = wave_sum(acc.match);
  acc.viol = wave_sum(acc.viol);
  acc.mfp = wave_sum(acc.mfp);
  acc.vfp = wave_sum(acc.vfp);
  const uint32_t wv = threadIdx.x / WAVE;
  if (lane() == 0) {
    s_acc[0][wv] = acc.match;
    s_acc[1][wv] = acc.viol;
    s_acc[2][wv] = acc.mfp;
    s_acc[3][wv] = acc.vfp;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long s = 0;
    for (int w = 0; w < BS / WAVE; w++) s += s_acc[threadIdx.x][w];
    if (s) atomicAdd(&a.counters[threadIdx.x], s);
  }
}

template <bool LAST>
__global__ __launch_bounds__(BS) void k_extend(ExtArgs a) {
  __shared__ LbsShared sh;
  __shared__ unsigned long long s_wcnt[BS / WAVE];
  __shared__ unsigned long long s_base;
  const uint64_t N = *a.d_nsrc < a.src_cap ? *a.d_nsrc : a.src_cap;
  FinalAcc acc{0, 0, 0, 0};
  int32_t thr[MAXK];
  bool thr_on = false;
  if (LAST) {
    thr_on = a.thr != nullptr && *a.d_thr_valid != 0;
#pragma unroll
    for (int v = 0; v < MAXK; v++) thr[v] = thr_on && v < a.k ? a.thr[v] : 0;
  }
  if (N > 0) {
    const uint64_t T = a.P[N];
    const uint64_t A1 = a.a_end < T ? a.a_end : T;
    const uint32_t wv = threadIdx.x / WAVE;
    for (uint64_t t0 = a.a_begin + (uint64_t)blockIdx.x * BS; t0 < A1;
         t0 += (uint64_t)gridDim.x * BS) {
      const uint64_t t1 = t0 + BS < A1 ? t0 + BS : A1;
      uint64_t s = 0, o = 0;
      const bool valid = lbs_tile(a.P, N, t0, t1, sh, s, o);
      int32_t h[MAXK];
      bool ok = false;
      if (valid) {
        const int32_t v = a.cpi_ent[a.beg[s] + o];
        ok = true;
#pragma unroll
        for (int j = 0; j < MAXK; j++) {
          h[j] = (j < a.i) ? a.src_cols[(uint64_t)j * a.src_stride + s] : v;
          if (j < a.i && h[j] == v) ok = false;
        }
        for (int c = 0; c < a.nchk && ok; c++) {
          const int32_t hw = pick(h, a.chk_pos[c]);
          if (a.chk_fwd[c] != PC_FREE)
            ok = constraint_ok(probe(a.g.out_off, a.g.out_nbr, a.g.out_lab, hw, v), a.chk_fwd[c]);
          if (ok && a.chk_bwd[c] != PC_FREE)
            ok = constraint_ok(probe(a.g.in_off, a.g.in_nbr, a.g.in_lab, hw, v), a.chk_bwd[c]);
        }
      }
      if (!LAST) {
        // block-aggregated append to the next frontier
        const uint64_t m = __ballot(ok);
        if (lane() == 0) s_wcnt[wv] = (unsigned long long)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
          unsigned long long tot = 0;
          for (int w = 0; w < BS / WAVE; w++) tot += s_wcnt[w];
          s_base = tot ? atomicAdd((unsigned long long*)a.d_ndst, tot) : 0ull;
        }
        __syncthreads();
        if (ok) {
          unsigned long long slot = s_base + rank_below(m);
          for (uint32_t w = 0; w < wv; w++) slot += s_wcnt[w];
          if (slot < a.dst_cap) {
#pragma unroll
            for (int j = 0; j < MAXK; j++)
              if (j <= a.i) a.dst_cols[(uint64_t)j * a.dst_cap + slot] = h[j];
          } else {
            atomicOr(a.d_flags, 1u);
          }
        }
      } else {
        int32_t t[MAXK];
        bool want = false;
        if (ok) {
          FinalAcc one{0, 0, 0, 0};
          want = finalize(a, h, t, one, thr_on, thr);
          if (!a.collect_only) {
            acc.match += one.match;
            acc.viol += one.viol;
            acc.mfp += one.mfp;
            acc.vfp += one.vfp;
          }
        }
        stage(a, want, t);
      }
    }
  }
  if (LAST && !a.collect_only) flush_acc(a, acc);
}

// k == 1: every candidate of the single pattern vertex is a match.
__global__ __launch_bounds__(BS) void k_single(ExtArgs a, const int32_t* __restrict__ list,
                                               const uint64_t* __restrict__ d_n, uint64_t cap) {
  uint64_t N = *d_n < cap ? *d_n : cap;
  if (a.a_end < N) N = a.a_end;
  const uint64_t I0 = a.a_begin < N ? a.a_begin : N;
  FinalAcc acc{0, 0, 0, 0};
  int32_t thr[MAXK];
  const bool thr_on = a.thr != nullptr && *a.d_thr_valid != 0;
#pragma unroll
  for (int v = 0; v < MAXK; v++) thr[v] = thr_on && v < a.k ? a.thr[v] : 0;
  const uint64_t stride = (uint64_t)gridDim.x * BS;
  const uint64_t rounds = (N - I0 + stride - 1) / stride;  // uniform trip count for the ballot
  for (uint64_t r = 0; r < rounds; r++) {
    const uint64_t i = I0 + r * stride + (uint64_t)blockIdx.x * BS + threadIdx.x;
    int32_t h[MAXK], t[MAXK];
    bool want = false;
    if (i < N) {
      const int32_t v = list[i];
#pragma unroll
      for (int j = 0; j < MAXK; j++) h[j] = v;
      FinalAcc one{0, 0, 0, 0};
      want = finalize(a, h, t, one, thr_on, thr);
      if (!a.collect_only) {
        acc.match += one.match;
        acc.viol += one.viol;
        acc.mfp += one.mfp;
        acc.vfp += one.vfp;
      }
    }
    stage(a, want, t);
  }
  if (!a.collect_only) flush_acc(a, acc);
}

void extend(hipStream_t st, const ExtArgs& a, bool last, int grid) {
  if (last)
    hipLaunchKernelGGL(k_extend<true>, dim3(grid), dim3(BS), 0, st, a);
  else
    hipLaunchKernelGGL(k_extend<false>, dim3(grid), dim3(BS), 0, st, a);
}
void single_vertex(hipStream_t st, const ExtArgs& a, const int32_t* list, const uint64_t* d_n,
                   uint64_t cap, int grid) {
  hipLaunchKernelGGL(k_single, dim3(grid), dim3(BS), 0, st, a, list, d_n, cap);
}

// ---------------------------------------------------------------------------
// lexicographic first-K of the staged violations
// ---------------------------------------------------------------------------

constexpr int SORT_THREADS = 1024;

__device__ __forceinline__ int cmp_lds(const uint32_t* s, uint32_t x, uint32_t y, int k) {
  for (int w = 0; w < k; w++) {
    uint32_t a = s[x * k + w], b = s[y * k + w];
    if (a != b) return a < b ? -1 : 1;
  }
  return 0;
}

// Bitonic sort of p2 (power of two) tuples held in LDS, ascending.
__device__ void bitonic_lds(uint32_t* s, uint32_t p2, int k) {
  for (uint32_t size = 2; size <= p2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
        const uint32_t lo = (i / stride) * 2 * stride + (i % stride), hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const int c = cmp_lds(s, lo, hi, k);
        if ((c > 0) == asc && c != 0) {
          for (int w = 0; w < k; w++) {
            uint32_t tmp = s[lo * k + w];
            s[lo * k + w] = s[hi * k + w];
            s[hi * k + w] = tmp;
          }
        }
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(SORT_THREADS) void k_topk_small(const int32_t* __restrict__ vbuf,
                                                             const uint64_t* __restrict__ d_vcount,
                                                             uint64_t vcap, int k, int K,
                                                             int32_t* __restrict__ res,
                                                             uint32_t* d_need_select) {
  __shared__ uint32_t s[SORT_MAX * MAXK];
  const uint64_t cnt = *d_vcount < vcap ? *d_vcount : vcap;
  if (cnt > (uint64_t)SORT_MAX) {
    if (threadIdx.x == 0) *d_need_select = 1;
    return;
  }
  if (threadIdx.x == 0) *d_need_select = 0;
  uint32_t p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  for (uint32_t i = threadIdx.x; i < p2 * (uint32_t)k; i += blockDim.x)
    s[i] = (i / k < cnt) ? (uint32_t)vbuf[i] : 0xFFFFFFFFu;
  bitonic_lds(s, p2, k);
  const uint64_t out = cnt < (uint64_t)K ? cnt : (uint64_t)K;
  for (uint32_t i = threadIdx.x; i < out * (uint32_t)k; i += blockDim.x) res[i] = (int32_t)s[i];
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_tuples(int32_t* buf,
                                                              const uint64_t* __restrict__ d_n,
                                                              int k) {
  __shared__ uint32_t s[SORT_MAX * MAXK];
  const uint64_t cnt = *d_n < (uint64_t)SORT_MAX ? *d_n : (uint64_t)SORT_MAX;
  uint32_t p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  for (uint32_t i = threadIdx.x; i < p2 * (uint32_t)k; i += blockDim.x)
    s[i] = (i / k < cnt) ? (uint32_t)buf[i] : 0xFFFFFFFFu;
  bitonic_lds(s, p2, k);
  for (uint32_t i = threadIdx.x; i < cnt * (uint32_t)k; i += blockDim.x) buf[i] = (int32_t)s[i];
}

void topk_small(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap, int k,
                int K, int32_t* res, uint32_t* d_need_select) {
  hipLaunchKernelGGL(k_topk_small, dim3(1), dim3(SORT_THREADS), 0, st, vbuf, d_vcount, vcap, k, K,
                     res, d_need_select);
}
void sort_tuples(hipStream_t st, int32_t* buf, const uint64_t* d_n, int k) {
  hipLaunchKernelGGL(k_sort_tuples, dim3(1), dim3(SORT_THREADS), 0, st, buf, d_n, k);
}

// Radix select state words: [0..MAXK) prefix tuple being decided,
// [MAXK] remaining rank (1-based) among tuples that match the prefix so far.
__global__ void k_select_begin(uint32_t* state, int K) {
  if (threadIdx.x < MAXK) state[threadIdx.x] = 0;
  if (threadIdx.x == 0) state[MAXK] = (uint32_t)K;
}

// Tuples that agree with the prefix on words < word and on the already
// decided high bits of `word` vote for the next digit.
__global__ __launch_bounds__(BS) void k_select_hist(const int32_t* __restrict__ vbuf,
                                                    const uint64_t* __restrict__ d_vcount,
                                                    uint64_t vcap, int k, int word, int shift,
                                                    int bits, const uint32_t* __restrict__ state,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[RADIX_BINS];
  for (int b = threadIdx.x; b < RADIX_BINS; b += BS) sh[b] = 0;
  __syncthreads();
  const uint64_t cnt = *d_vcount < vcap ? *d_vcount : vcap;
  const uint32_t hi_mask = (shift + bits >= 32) ? 0u : (0xFFFFFFFFu << (shift + bits));
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * BS) {
    const uint32_t* t = (const uint32_t*)vbuf + i * (uint64_t)k;
    bool match = true;
    for (int w = 0; w < word && match; w++) match = t[w] == state[w];
    if (!match) continue;
    const uint32_t x = t[word];
    if ((x & hi_mask) != (state[word] & hi_mask)) continue;
    atomicAdd(&sh[(x >> shift) & ((1u << bits) - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < RADIX_BINS; b += BS)
    if (sh[b]) atomicAdd(&hist[b], sh[b]);
}

__global__ void k_select_pick(int word, int shift, int bits, uint32_t* state, uint32_t* hist) {
  if (threadIdx.x == 0) {
    uint32_t r = state[MAXK], cum = 0;
    const uint32_t nb = 1u << bits;
    uint32_t d = nb - 1;
    for (uint32_t b = 0; b < nb; b++) {
      if (cum + hist[b] >= r) {
        d = b;
        break;
      }
      cum += hist[b];
    }
    state[MAXK] = r - cum;
    state[word] |= d << shift;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < RADIX_BINS; b += blockDim.x) hist[b] = 0;
}

__global__ __launch_bounds__(BS) void k_select_compact(const int32_t* __restrict__ vbuf,
                                                       const uint64_t* __restrict__ d_vcount,
                                                       uint64_t vcap, int k,
                                                       const uint32_t* __restrict__ state,
                                                       int32_t* __restrict__ out,
                                                       unsigned long long* d_outcount) {
  const uint64_t cnt = *d_vcount < vcap ? *d_vcount : vcap;
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * BS) {
    const uint32_t* t = (const uint32_t*)vbuf + i * (uint64_t)k;
    int c = 0;
    for (int w = 0; w < k && c == 0; w++) c = t[w] < state[w] ? -1 : (t[w] > state[w] ? 1 : 0);
    if (c <= 0) {
      const unsigned long long slot = atomicAdd(d_outcount, 1ull);
      if (slot < (unsigned long long)SORT_MAX)
        for (int w = 0; w < k; w++) out[slot * k + w] = (int32_t)t[w];
    }
  }
}

void select_begin(hipStream_t st, uint32_t* state, int K) {
  hipLaunchKernelGGL(k_select_begin, dim3(1), dim3(64), 0, st, state, K);
}
void select_pass(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap,
                 int k, int word, int shift, int bits, uint32_t* state, uint32_t* hist, int grid) {
  hipLaunchKernelGGL(k_select_hist, dim3(grid), dim3(BS), 0, st, vbuf, d_vcount, vcap, k, word,
                     shift, bits, state, hist);
  hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(BS), 0, st, word, shift, bits, state, hist);
}
void select_compact(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap,
                    int k, const uint32_t* state, int32_t* out, uint64_t* d_outcount, int grid) {
  hipLaunchKernelGGL(k_select_compact, dim3(grid), dim3(BS), 0, st, vbuf, d_vcount, vcap, k, state,
                     out, (unsigned long long*)d_outcount);
}

}  // namespace gfd
