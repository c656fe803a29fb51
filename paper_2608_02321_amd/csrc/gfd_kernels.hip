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



// Label of data edge a -> b, or NOEDGE: binary search of the shorter of
// out-row(a) (for b) and in-row(b) (for a).  Power-law hubs make the two
// lengths differ by orders of magnitude.
__device__ __forceinline__ int32_t edge_label(const DevGraph& g, int32_t a, int32_t b,
                                              unsigned long long& by) {
  const uint32_t oa = g.out_off[a], oa1 = g.out_off[a + 1];
  const uint32_t ib = g.in_off[b], ib1 = g.in_off[b + 1];
  by += 16;
  const bool use_out = (oa1 - oa) <= (ib1 - ib);
  const int32_t* nbr = use_out ? g.out_nbr : g.in_nbr;
  const int32_t* lab = use_out ? g.out_lab : g.in_lab;
  const int32_t key = use_out ? b : a;
  uint32_t lo = use_out ? oa : ib, hi = use_out ? oa1 : ib1;
  const uint32_t end = hi;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    by += 4;
    if (nbr[mid] < key) lo = mid + 1; else hi = mid;
  }
  if (lo < end && nbr[lo] == key) {
    by += 8;
    return lab[lo];
  }
  return NOEDGE;
}

__device__ __forceinline__ bool constraint_ok(int32_t found, int32_t code) {
  if (code == PC_FREE) return true;
  if (code == PC_ABSENT) return found == NOEDGE;
  return found != NOEDGE && (code == ANY || found == code);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// ---------------------------------------------------------------------------
// single-pass exclusive scan of u32 items into u64 prefixes
// ---------------------------------------------------------------------------

constexpr uint64_t VAL_MASK = (1ull << 46) - 1;
__device__ __forceinline__ uint64_t pack_state(uint32_t ep, uint32_t flag, uint64_t v) {
  return ((uint64_t)(ep & 0xFFFFu) << 48) | ((uint64_t)flag << 46) | (v & VAL_MASK);
}

struct FnSrc {
  const int32_t* par;
  const int32_t* pos;
  const uint32_t* cpi_beg;
  const uint32_t* cpi_len;
  uint32_t* beg;
  __device__ uint32_t operator()(uint64_t i) const {
    const int32_t c = pos[par[i]];
    beg[i] = cpi_beg[c];
    return cpi_len[c];
  }
};

// Exclusive prefix of tile aggregates in ticket order, computed by the 64
// lanes of wave 0 together: each round loads the states of the 64 nearest
// predecessors at once and sums back to the closest one that already holds its
// inclusive prefix.  Tile t waits only on tiles with smaller tickets, which
// running blocks own; the wait is bounded and reports an error instead of
// hanging.  Each state word carries its whole message (epoch, flag, value), so
// relaxed agent-scope atomics are enough: they are coherent across XCDs
// without the L2 write-back/invalidate that release/acquire ordering costs.
__device__ uint64_t tile_prefix_wave(const TileScan& ts, uint64_t t, uint64_t agg) {
  if (t == 0) {
    if (lane() == 0)
      __hip_atomic_store(&ts.state[0], pack_state(ts.epoch, 2, agg), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane() == 0)
    __hip_atomic_store(&ts.state[t], pack_state(ts.epoch, 1, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint64_t prefix = 0;
  int64_t end = (int64_t)t;
  uint32_t spins = 0;
  for (;;) {
    const int64_t j = end - 1 - (int64_t)lane();  // lane 0: nearest predecessor
    uint32_t fl = 2;
    uint64_t val = 0;
    if (j >= 0) {
      const uint64_t w = __hip_atomic_load(&ts.state[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      fl = ((uint32_t)(w >> 48) == (ts.epoch & 0xFFFFu)) ? ((uint32_t)(w >> 46) & 3u) : 0u;
      val = w & VAL_MASK;
    }
    const uint64_t incl = __ballot(fl == 2);
    const uint64_t waiting = __ballot(fl == 0);
    const int first = incl ? __ffsll((long long)incl) - 1 : WAVE;  // closest inclusive
    const uint64_t need = first >= WAVE - 1 ? ~0ull : ((2ull << first) - 1);
    if (waiting & need) {
      if (++spins > (1u << 22)) {
        if (lane() == 0) atomicOr(ts.err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    prefix += wave_sum((int)lane() <= first ? val : 0ull);
    if (first < WAVE) break;
    end -= WAVE;
  }
  if (lane() == 0)
    __hip_atomic_store(&ts.state[t], pack_state(ts.epoch, 2, prefix + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return prefix;
}

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
    if (threadIdx.x < WAVE) {
      const TileScan ts{state, ticket, err, epoch};
      const uint64_t pb = tile_prefix_wave(ts, t, agg);
      if (threadIdx.x == 0) s_pre = pb;
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
  int grid = (int)(tiles < 1 ? 1 : (tiles > 64 ? 64 : tiles));
  ws.epoch = (ws.epoch + 1) & 0xFFFFu;
  if (ws.epoch == 0) {  // wrapped: stale tile states could alias the new epoch
    fill_u64(st, ws.tile_state, 0, ws.max_tiles);
    ws.epoch = 1;
  }
  hipLaunchKernelGGL(k_scan<F>, dim3(grid), dim3(BS), 0, st, f, d_n, cap, per_word, out, d_total,
                     ws.tile_state, ws.ticket, ws.epoch, ws.err);
}

void scan_sources(hipStream_t st, ScanWs& ws, const int32_t* par_col, const uint64_t* d_n,
                  uint64_t cap, const int32_t* pos_map, const uint32_t* cpi_beg,
                  const uint32_t* cpi_len, uint32_t* beg, uint64_t* P, uint64_t* d_total) {
  launch_scan(st, ws, FnSrc{par_col, pos_map, cpi_beg, cpi_len, beg}, d_n, cap, 0, P, d_total);
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
// block-level helpers
// ---------------------------------------------------------------------------

// Adds every thread's x into *dst once per block (all threads must call).
__device__ __forceinline__ void block_add(unsigned long long* dst, unsigned long long x) {
  __shared__ unsigned long long s_part[BS / WAVE];
  x = wave_sum(x);
  __syncthreads();
  if (lane() == 0) s_part[threadIdx.x / WAVE] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < BS / WAVE; w++) t += s_part[w];
    if (t) atomicAdd(dst, t);
  }
}

// Block-wide exclusive scan of one u32 per thread; returns the thread's prefix
// and sets `total`.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total) {
  __shared__ uint32_t s_w[BS / WAVE];
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint32_t y = __shfl_up(inc, (unsigned)d);
    if (lane() >= (uint32_t)d) inc += y;
  }
  __syncthreads();
  if (lane() == WAVE - 1) s_w[threadIdx.x / WAVE] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  const uint32_t wv = threadIdx.x / WAVE;
#pragma unroll
  for (int w = 0; w < BS / WAVE; w++) {
    if ((uint32_t)w < wv) pre += s_w[w];
    tot += s_w[w];
  }
  total = tot;
  return pre + inc - x;
}

// Block-wide walk over the concatenation of BS rows (one row per thread, given
// as start and length): every round maps BS consecutive entries to their rows
// with a binary search in LDS, so each thread does a short chain of loads for
// one entry instead of walking a whole row.  All threads must call it.
struct FlatShared {
  uint32_t pre[BS];
  uint32_t beg[BS];
};
template <class F>
__device__ __forceinline__ void block_flat(FlatShared& sh, uint32_t beg, uint32_t len, F f) {
  uint32_t total;
  const uint32_t pre = block_excl_scan(len, total);
  sh.pre[threadIdx.x] = pre;
  sh.beg[threadIdx.x] = beg;
  __syncthreads();
  for (uint32_t base = 0; base < total; base += BS) {
    const uint32_t ai = base + threadIdx.x;
    if (ai < total) {
      uint32_t lo = 0, hi = BS - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (sh.pre[mid] <= ai) lo = mid; else hi = mid - 1;
      }
      f(lo, sh.beg[lo] + (ai - sh.pre[lo]));
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// candidate filter (Section IV-B: label candidates, degree filter, BFS
// candidate subgraph with dead-end removal as pull constraints)
// ---------------------------------------------------------------------------

// Output order is not fixed: each tile reserves its slots with one atomic add,
// so no tile waits on another.  Candidate sets are sets; every later step
// reads them through the position map or by scanning them whole.
__global__ __launch_bounds__(BS) void k_cand(CandArgs a) {
  const uint64_t N = a.d_n ? (*a.d_n < a.cap ? *a.d_n : a.cap) : a.n_host;
  const uint64_t ntiles = (N + BS - 1) / BS;
  __shared__ unsigned long long s_base;
  __shared__ FlatShared fs;
  __shared__ uint32_t s_found[BS];
  unsigned long long by = 0;
  const DevGraph& g = a.g;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t i = t * BS + threadIdx.x;
    bool ok = i < N;
    int32_t v = 0;
    if (ok) {
      v = a.list ? a.list[i] : (int32_t)i;
      by += a.list ? 4 : 0;
      if (a.min_out > 0) {
        by += 8;
        ok = (int32_t)(g.out_off[v + 1] - g.out_off[v]) >= a.min_out;
      }
      if (ok && a.min_in > 0) {
        by += 8;
        ok = (int32_t)(g.in_off[v + 1] - g.in_off[v]) >= a.min_in;
      }
    }
    for (int c = 0; c < a.ncons; c++) {  // uniform loop: every thread takes part
      const PullCons cs = a.cons[c];
      const uint32_t* off = cs.dir ? g.in_off : g.out_off;
      const int32_t* nbr = cs.dir ? g.in_nbr : g.out_nbr;
      const int32_t* lab = cs.dir ? g.in_lab : g.out_lab;
      uint32_t rb = 0, rl = 0;
      if (ok) {
        rb = off[v];
        rl = off[v + 1] - rb;
        by += 8;
      }
      s_found[threadIdx.x] = 0;
      block_flat(fs, rb, rl, [&](uint32_t item, uint32_t x) {
        if (s_found[item]) return;  // some neighbour already qualified
        if (cs.elab != ANY) {
          by += 4;
          if (lab[x] != cs.elab) return;
        }
        by += 5;
        if (cs.mem[nbr[x]] == (uint8_t)cs.ep) s_found[item] = 1;
      });
      ok = ok && s_found[threadIdx.x] != 0;
      __syncthreads();
    }
    uint32_t total;
    const uint32_t rank = block_excl_scan(ok ? 1u : 0u, total);
    if (threadIdx.x == 0)
      s_base = total ? atomicAdd((unsigned long long*)a.d_out_n, (unsigned long long)total) : 0ull;
    __syncthreads();
    if (ok) {
      const uint64_t idx = s_base + rank;
      a.out[idx] = v;
      a.mem[v] = (uint8_t)a.mem_ep;
      by += 5;
      if (a.posmap) {
        a.posmap[v] = (int32_t)idx;
        by += 4;
      }
    }
    __syncthreads();
  }
  if (a.bytes) block_add(a.bytes, by);
}

void cand_filter(hipStream_t st, const CandArgs& a, int grid) {
  hipLaunchKernelGGL(k_cand, dim3(grid), dim3(BS), 0, st, a);
}

// ---------------------------------------------------------------------------
// CPI adjacency lists for one spanning-tree edge (p, u)
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool cpi_keep(const CpiArgs& a, int32_t vp, uint32_t x,
                                         unsigned long long& by) {
  const DevGraph& g = a.g;
  const int32_t* nbr = a.dir ? g.in_nbr : g.out_nbr;
  const int32_t* lab = a.dir ? g.in_lab : g.out_lab;
  const int32_t v = nbr[x];
  by += 5;
  if (a.mem[v] != (uint8_t)a.ep) return false;
  if (a.prim != ANY) {
    by += 4;
    if (lab[x] != a.prim) return false;
  }
  if (a.other == PC_FREE) return true;
  // the reverse direction of the scanned edge: dir 0 scanned vp -> v, so the
  // reverse is v -> vp; dir 1 scanned v -> vp, so the reverse is vp -> v
  const int32_t r = a.dir ? edge_label(g, vp, v, by) : edge_label(g, v, vp, by);
  return constraint_ok(r, a.other);
}

// Two walks over each tile's rows: count the kept entries per row, reserve
// the tile's entries with one atomic add, then write them.  A list is
// (begin, length) per parent candidate; lists of one tile are contiguous.  The
// order of entries inside one list is not fixed; nothing downstream needs it.
__global__ __launch_bounds__(BS) void k_cpi(CpiArgs a) {
  const uint64_t N = *a.d_n < a.cap ? *a.d_n : a.cap;
  const uint64_t ntiles = (N + BS - 1) / BS;
  __shared__ unsigned long long s_base;
  __shared__ FlatShared fs;
  __shared__ uint32_t s_cnt[BS];
  __shared__ int32_t s_vp[BS];
  unsigned long long by = 0, dummy = 0;
  const uint32_t* off = a.dir ? a.g.in_off : a.g.out_off;
  const int32_t* nbr = a.dir ? a.g.in_nbr : a.g.out_nbr;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t s = t * BS + threadIdx.x;
    const bool valid = s < N;
    int32_t vp = 0;
    uint32_t b = 0, len = 0;
    if (valid) {
      vp = a.list[s];
      b = off[vp];
      len = off[vp + 1] - b;
      by += 12;
    }
    s_vp[threadIdx.x] = vp;
    s_cnt[threadIdx.x] = 0;
    __syncthreads();
    block_flat(fs, b, len, [&](uint32_t item, uint32_t x) {
      if (cpi_keep(a, s_vp[item], x, by)) atomicAdd(&s_cnt[item], 1u);
    });
    const uint32_t cnt = s_cnt[threadIdx.x];
    uint32_t total;
    const uint32_t pre = block_excl_scan(cnt, total);
    if (threadIdx.x == 0)
      s_base = total ? atomicAdd((unsigned long long*)a.d_entries, (unsigned long long)total) : 0ull;
    __syncthreads();
    const uint64_t base = s_base;
    if (valid) {
      a.cpi_beg[s] = (uint32_t)(base + pre);
      a.cpi_len[s] = cnt;
      by += 8;
    }
    s_cnt[threadIdx.x] = pre;  // becomes the running write position of each row
    __syncthreads();
    block_flat(fs, b, len, [&](uint32_t item, uint32_t x) {
      if (cpi_keep(a, s_vp[item], x, dummy)) {
        const uint32_t at = atomicAdd(&s_cnt[item], 1u);
        a.cpi_ent[base + at] = nbr[x];
        by += 4;
      }
    });
  }
  if (a.bytes) block_add(a.bytes, by);
}

void cpi_adjacency(hipStream_t st, const CpiArgs& a, int grid) {
  hipLaunchKernelGGL(k_cpi, dim3(grid), dim3(BS), 0, st, a);
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
  unsigned long long by = 0;
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
        // CPI entry, plus the source's list start, prefix and partial once per source
        by += 4 + (o == 0 ? 12ull + 4ull * (uint64_t)a.i : 0ull);
        ok = true;
#pragma unroll
        for (int j = 0; j < MAXK; j++) {
          h[j] = (j < a.i) ? a.src_cols[(uint64_t)j * a.src_stride + s] : v;
          if (j < a.i && h[j] == v) ok = false;
        }
        for (int c = 0; c < a.nchk && ok; c++) {
          const int32_t hw = pick(h, a.chk_pos[c]);
          if (a.chk_fwd[c] != PC_FREE)
            ok = constraint_ok(edge_label(a.g, hw, v, by), a.chk_fwd[c]);
          if (ok && a.chk_bwd[c] != PC_FREE)
            ok = constraint_ok(edge_label(a.g, v, hw, by), a.chk_bwd[c]);
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
            by += 4ull * (uint64_t)(a.i + 1);
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
          by += 4ull * (uint64_t)(2 * a.nx + 2 * a.ny);
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
  if (a.bytes) block_add(a.bytes, by);
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

// Finds the bin holding the remaining rank with a block-wide scan of the
// histogram (BS threads x RADIX_BINS / BS bins each), then clears it.
__global__ __launch_bounds__(BS) void k_select_pick(int word, int shift, int bits,
                                                    uint32_t* state, uint32_t* hist) {
  constexpr int PER = RADIX_BINS / BS;
  const uint32_t nb = 1u << bits;
  const uint32_t r = state[MAXK];  // read before the scan's barriers; one thread rewrites it
  uint32_t h[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t bin = threadIdx.x * PER + j;
    h[j] = bin < nb ? hist[bin] : 0u;
    sum += h[j];
  }
  uint32_t total;
  const uint32_t pre = block_excl_scan(sum, total);
  if (pre < r && r <= pre + sum) {  // exactly one thread
    uint32_t cum = pre, d = threadIdx.x * PER;
    for (int j = 0; j < PER; j++) {
      if (cum + h[j] >= r) {
        d = threadIdx.x * PER + j;
        break;
      }
      cum += h[j];
    }
    state[MAXK] = r - cum;
    state[word] |= d << shift;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; j++) hist[threadIdx.x * PER + j] = 0;
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
