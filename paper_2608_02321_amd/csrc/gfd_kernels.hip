// HIP kernels (gfx950, wave64) for GFD validation, batched over jobs (GFDs):
//   - single-pass exclusive scans with a wave-parallel decoupled look-back,
//   - candidate filtering: label bucket + degree filter, pull constraints
//     (adjacency to the candidates of neighbouring pattern vertices), sparse-set
//     compaction with one atomic reservation per tile,
//   - Compact Path Index adjacency lists per spanning-tree edge,
//   - level-synchronous embedding enumeration over the CPI, every extension
//     attempt mapped to its source by load-balanced search; injectivity,
//     non-tree edge and induced non-edge probes; the X -> Y literal check fused
//     into the last level,
//   - exact lexicographic first-K selection of violating tuples.
// FastGFDs paper, Section IV-B (CPI, core-first matching) and Section II
// (definitions).  All arithmetic is integer.
#include "gfd_internal.h"

namespace gfd {

// ---------------------------------------------------------------------------
// wave and block helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

#ifdef GFD_COUNT_UNITS
extern __device__ unsigned long long unit_counts[UNIT_KINDS];
#endif

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

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// Block-wide exclusive scan of one u32 per thread; returns the thread's prefix
// and sets `total`.  All threads must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total) {
  __shared__ uint32_t s_w[BS / WAVE];
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t y = __shfl_up(inc, (unsigned)d);
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

// The same scan over one u64 per thread.
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t x, uint64_t& total) {
  __shared__ uint64_t s_w64[BS / WAVE];
  uint64_t inc = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t y = __shfl_up(inc, (unsigned)d);
    if (lane() >= (uint32_t)d) inc += y;
  }
  __syncthreads();
  if (lane() == WAVE - 1) s_w64[threadIdx.x / WAVE] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  const uint32_t wv = threadIdx.x / WAVE;
#pragma unroll
  for (int w = 0; w < BS / WAVE; w++) {
    if ((uint32_t)w < wv) pre += s_w64[w];
    tot += s_w64[w];
  }
  total = tot;
  return pre + inc - x;
}

// Adds every thread's x into *dst once per block.  All threads must call it.
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

__device__ __forceinline__ bool constraint_ok(int32_t found, int32_t code) {
  if (code == PC_FREE) return true;
  if (code == PC_ABSENT) return found == NOEDGE;
  return found != NOEDGE && (code == ANY || found == code);
}

// Label of data edge a -> b, or NOEDGE, searching the row of `anchor` (a's
// out-row when anchor == a, else b's in-row).  Enumeration and CPI probes
// anchor on the vertex that neighbouring threads share (the earlier matched
// vertex, the CPI source), so the searched row stays in cache across the
// wave instead of each thread fetching its own candidate's row.
// ceil(log2 d) for d >= 1 (0 for d <= 1)
__device__ __forceinline__ uint32_t clog2(uint64_t d) {
  return d <= 1 ? 0u : 64u - (uint32_t)__clzll((long long)(d - 1));
}

__device__ __forceinline__ int32_t edge_label_at(const DevGraph& g, int32_t a, int32_t b,
                                                 bool anchor_a, unsigned long long& by,
                                                 Units* U = nullptr) {
  const uint32_t* off = anchor_a ? g.out_off : g.in_off;
  const int32_t* nbr = anchor_a ? g.out_nbr : g.in_nbr;
  const int32_t* lab = anchor_a ? g.out_lab : g.in_lab;
  const int32_t row = anchor_a ? a : b, key = anchor_a ? b : a;
  uint32_t lo = off[row], hi = off[row + 1];
  const uint32_t end = hi;
  by += 8;
  if (U) {
    U->c[U_CHK_ONE]++;
    U->c[U_ONE_LOG2D] += clog2(hi - lo);
  }
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    by += 4;
    if (U) U->c[U_ONE_STEPS]++;
    if (nbr[mid] < key) lo = mid + 1; else hi = mid;
  }
  if (lo < end && nbr[lo] == key) {
    by += 4;
    return lab[lo];
  }
  return NOEDGE;
}

// Labels of both data edges between a and b, (a -> b, b -> a), NOEDGE where
// absent: one search of a's combined row instead of one in each direction.
// A long row is first looked up in its fingerprint table, which settles the
// common case (not adjacent) in about one access; the row search then runs
// only for neighbours (to read their labels) and for the rare fingerprint
// that matches by chance.
__device__ __forceinline__ int2 edge_labels_both(const DevGraph& g, int32_t a, int32_t b,
                                                 unsigned long long& by, Units* U = nullptr) {
  const uint64_t t0 = g.hub_off[a], t1 = g.hub_off[a + 1];
  by += 16;
  if (U) U->c[U_BOTH_LOG2D] += clog2(g.sym_off[a + 1] - g.sym_off[a]);
  if (t1 > t0) {
    const uint64_t mask = t1 - t0 - 1;
    const uint8_t f = hub_fp(b);
    // at least half the slots are free, so the probe sequence ends
    for (uint64_t i = hub_slot(b, t1 - t0);; i = (i + 1) & mask) {
      const uint8_t e = g.hub_tab[t0 + i];
      by += 1;
      if (e == f) break;
      if (e == 0) {
        if (U) U->c[U_TABLE_FREE]++;
        return make_int2(NOEDGE, NOEDGE);
      }
    }
    if (U) U->c[U_TABLE_HIT]++;
  } else if (U) {
    U->c[U_SHORT_ROW]++;
  }
  uint64_t lo = g.sym_off[a], hi = g.sym_off[a + 1];
  const uint64_t end = hi;
  by += 16;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    by += 4;
    if (U) U->c[U_BOTH_STEPS]++;
    if (g.sym_nbr[mid] < b) lo = mid + 1; else hi = mid;
  }
  if (lo < end && g.sym_nbr[lo] == b) {
    by += 8;
    return g.sym_lab[lo];
  }
  return make_int2(NOEDGE, NOEDGE);
}

// Constraint `code` on data edge a -> b, probed in the anchor's row.
__device__ __forceinline__ bool pair_ok(const DevGraph& g, int32_t a, int32_t b, bool anchor_a,
                                        int32_t code, unsigned long long& by, Units* U = nullptr) {
  if (code == PC_FREE) return true;
  return constraint_ok(edge_label_at(g, a, b, anchor_a, by, U), code);
}

// Membership bitmaps (n bits, 512 KB at 4M vertices) stay in L2: their probes
// count no algorithmic HBM bytes.
__device__ __forceinline__ bool member(const CandSet& c, int32_t x) {
  return (c.bits[(uint32_t)x >> 5] >> ((uint32_t)x & 31u)) & 1u;
}

// ---------------------------------------------------------------------------
// per-job single-pass exclusive scan (decoupled look-back)
// ---------------------------------------------------------------------------

constexpr uint64_t VAL_MASK = (1ull << 46) - 1;
__device__ __forceinline__ uint64_t pack_state(uint32_t ep, uint32_t flag, uint64_t v) {
  return ((uint64_t)(ep & 0xFFFFu) << 48) | ((uint64_t)flag << 46) | (v & VAL_MASK);
}

// Exclusive prefix of tile aggregates in ticket order, computed by the 64
// lanes of wave 0 together: each round loads the states of the 64 nearest
// predecessors at once and sums back to the closest one that already holds its
// inclusive prefix.  Tile t waits only on tiles with smaller tickets, which
// running blocks own; the wait is bounded and reports an error instead of
// hanging.  Each state word carries its whole message (epoch, flag, value), so
// relaxed agent-scope atomics are enough: they are coherent across XCDs
// without the L2 write-back/invalidate that release/acquire ordering costs.
__device__ uint64_t tile_prefix_wave(const JobScan& sc, uint64_t t, uint64_t agg) {
  if (t == 0) {
    if (lane() == 0)
      __hip_atomic_store(&sc.tstate[0], pack_state(sc.epoch, 2, agg), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane() == 0)
    __hip_atomic_store(&sc.tstate[t], pack_state(sc.epoch, 1, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint64_t prefix = 0;
  int64_t end = (int64_t)t;
  uint32_t spins = 0;
  for (;;) {
    const int64_t j = end - 1 - (int64_t)lane();  // lane 0: nearest predecessor
    uint32_t fl = 2;
    uint64_t val = 0;
    if (j >= 0) {
      const uint64_t w =
          __hip_atomic_load(&sc.tstate[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      fl = ((uint32_t)(w >> 48) == (sc.epoch & 0xFFFFu)) ? ((uint32_t)(w >> 46) & 3u) : 0u;
      val = w & VAL_MASK;
    }
    const uint64_t incl = __ballot(fl == 2);
    const uint64_t waiting = __ballot(fl == 0);
    const int first = incl ? __ffsll((long long)incl) - 1 : WAVE;  // closest inclusive
    const uint64_t need = first >= WAVE - 1 ? ~0ull : ((2ull << first) - 1);
    if (waiting & need) {
      if (++spins > (1u << 22)) {
        if (lane() == 0) atomicOr(sc.err, 1u);
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
    __hip_atomic_store(&sc.tstate[t], pack_state(sc.epoch, 2, prefix + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return prefix;
}

// Exclusive scan of f(0..N-1) into sc.P[0..N] and *sc.d_total, by the nb
// blocks given to one job (each calls it once).  Tiles are handed out by the
// job's ticket; the block taking the last ticket resets it.  All threads of
// the block must call it.
template <class F>
__device__ void job_scan(uint64_t N, F f, const JobScan& sc, uint64_t nb) {
  const uint64_t ntiles = (N + SCAN_TILE - 1) / SCAN_TILE;
  __shared__ uint32_t s_t;
  __shared__ uint64_t s_pre;
  __shared__ uint64_t s_w[BS / WAVE];
  const uint32_t ln = lane(), wv = threadIdx.x / WAVE;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_t = atomicAdd(sc.ticket, 1u);
    __syncthreads();
    const uint64_t t = s_t;
    if (t >= ntiles) {
      if (threadIdx.x == 0 && t == ntiles + nb - 1) {
        if (ntiles == 0) {
          sc.P[0] = 0;
          *sc.d_total = 0;
        }
        __hip_atomic_store(sc.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
      const uint64_t y = __shfl_up(x, (unsigned)d);
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
      const uint64_t pb = tile_prefix_wave(sc, t, agg);
      if (threadIdx.x == 0) s_pre = pb;
    }
    __syncthreads();
    uint64_t run = s_pre + wpre + x - sum;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; j++) {
      if (base + j < N) {
        sc.P[base + j] = run;
        run += v[j];
      }
    }
    if (t == ntiles - 1 && threadIdx.x == BS - 1) {
      sc.P[N] = s_pre + agg;
      *sc.d_total = s_pre + agg;
    }
  }
}

// ---------------------------------------------------------------------------
// load-balanced search: map a tile of flat work positions to (source, offset)
// ---------------------------------------------------------------------------

constexpr int LBS_SLOTS = (int)LBS_CHUNK + 2;  // prefix entries staged in LDS
struct LbsShared {
  uint64_t p[LBS_SLOTS];
  uint64_t lo, hi;
};

// largest s in [lo, hi] with P[s] <= a (P non-decreasing, P[lo] <= a)
template <class T>
__device__ __forceinline__ uint64_t last_le(const T* __restrict__ P, uint64_t lo, uint64_t hi,
                                            uint64_t a) {
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) >> 1;
    if (P[mid] <= a) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The same search done by one whole wave: every round samples 64 evenly spaced
// prefix values at once and keeps the stretch that holds the answer, so a
// search over N sources costs about log64(N) dependent loads.
template <class T>
__device__ __forceinline__ uint64_t wave_last_le(const T* __restrict__ P, uint64_t lo, uint64_t hi,
                                                 uint64_t a) {
  while (hi - lo >= WAVE) {
    const uint64_t step = (hi - lo) / WAVE + 1;
    uint64_t idx = lo + (uint64_t)(lane() + 1) * step;
    if (idx > hi) idx = hi;
    // lanes past hi all sample P[hi]; the votes form a prefix of the lanes
    const uint64_t cnt = (uint64_t)__popcll(__ballot(P[idx] <= a));
    const uint64_t nlo = lo + cnt * step;
    const uint64_t nhi = lo + (cnt + 1) * step - 1;
    lo = nlo < hi ? nlo : hi;
    hi = nhi < hi ? nhi : hi;
  }
  const bool le = lo + lane() <= hi && P[lo + lane()] <= a;
  return lo + (uint64_t)__popcll(__ballot(le)) - 1;
}

// Maps the flat positions [c0, c1) of one job row (P[0] <= c0 < c1 <= P[N],
// at most LBS_CHUNK of them) to (source, offset).  The chunk's first and last
// source come from two wave-parallel searches and their prefix values are
// staged in LDS.  SERIAL: thread t takes the LBS_ROUNDS consecutive
// positions c0 + t*LBS_ROUNDS ..; one binary search places the first and the
// rest walk forward, so short rows (most of a power-law graph) cost no search
// each.  Otherwise round r gives thread t position c0 + r*BS + t (coalesced
// loads across the wave), each placed by its own binary search.
// f(valid, s, o, a) -- position a = P[s] + o -- is called by every thread
// LBS_ROUNDS times (uniform trip count); the call ends with a barrier.
template <bool SERIAL, class T, class F>
__device__ __forceinline__ void flat_chunk(const T* __restrict__ P, uint64_t N, uint64_t c0,
                                           uint64_t c1, LbsShared& sh, F f) {
  if (threadIdx.x < WAVE) {
    const uint64_t lo = wave_last_le(P, 0, N - 1, c0);
    if (threadIdx.x == 0) sh.lo = lo;
  } else if (threadIdx.x < 2 * WAVE) {
    const uint64_t hi = wave_last_le(P, 0, N - 1, c1 - 1);
    if (threadIdx.x == WAVE) sh.hi = hi;
  }
  __syncthreads();
  const uint64_t lo = sh.lo, hi = sh.hi;
  const uint64_t span = hi - lo + 2;  // P[lo .. hi+1]
  const bool in_lds = span <= (uint64_t)LBS_SLOTS;
  if (in_lds)
    for (uint64_t j = threadIdx.x; j < span; j += BS) sh.p[j] = P[lo + j];
  __syncthreads();
  // largest l in [from, span-2] with sh.p[l] <= a
  auto lds_search = [&](uint32_t from, uint64_t a) -> uint32_t {
    uint32_t l = from, h = (uint32_t)(span - 2);
    while (l < h) {
      const uint32_t mid = (l + h + 1) >> 1;
      if (sh.p[mid] <= a) l = mid; else h = mid - 1;
    }
    return l;
  };
  const uint64_t a0 = SERIAL ? c0 + (uint64_t)threadIdx.x * LBS_ROUNDS : c0 + threadIdx.x;
  uint32_t l = (SERIAL && in_lds && a0 < c1) ? lds_search(0, a0) : 0u;  // source lo + l
  for (int r = 0; r < LBS_ROUNDS; r++) {
    const uint64_t a = SERIAL ? a0 + (uint64_t)r : a0 + (uint64_t)r * BS;
    const bool valid = a < c1;
    uint64_t s = 0, o = 0;
    if (valid) {
      if (in_lds) {
        if (SERIAL)
          while (sh.p[l + 1] <= a) l++;  // a < P[hi+1], so this stops inside the slice
        else
          l = lds_search(l, a);  // positions only grow: search from the last source
        s = lo + l;
        o = a - sh.p[l];
      } else {
        s = last_le(P, lo, hi, a);
        o = a - P[s];
      }
    }
    f(valid, s, o, a);
  }
  __syncthreads();
}

// flat_chunk<false> split in phases: every round's position is placed and
// its value loaded by pre(s, o) first -- LBS_ROUNDS independent loads in
// flight per thread --, then mid(s, value) per round (more independent
// loads), and only then f(valid, s, first, value, mid's bit) runs per round.
template <class T, class Pre, class Mid, class F>
__device__ __forceinline__ void flat_chunk_pre(const T* __restrict__ P, uint64_t N, uint64_t c0,
                                               uint64_t c1, LbsShared& sh, Pre pre, Mid mid, F f) {
  if (threadIdx.x < WAVE) {
    const uint64_t lo = wave_last_le(P, 0, N - 1, c0);
    if (threadIdx.x == 0) sh.lo = lo;
  } else if (threadIdx.x < 2 * WAVE) {
    const uint64_t hi = wave_last_le(P, 0, N - 1, c1 - 1);
    if (threadIdx.x == WAVE) sh.hi = hi;
  }
  __syncthreads();
  const uint64_t lo = sh.lo, hi = sh.hi;
  const uint64_t span = hi - lo + 2;  // P[lo .. hi+1]
  const bool in_lds = span <= (uint64_t)LBS_SLOTS;
  if (in_lds)
    for (uint64_t j = threadIdx.x; j < span; j += BS) sh.p[j] = P[lo + j];
  __syncthreads();
  // per round only the source is kept; its offset is recomputed from the
  // staged prefix when the value is loaded, and f learns only whether it is
  // the source's first position
  uint32_t ss[LBS_ROUNDS];
  int32_t pv[LBS_ROUNDS];
  uint32_t valid = 0, first = 0;
  uint32_t l = 0;  // in_lds: source lo + l
#pragma unroll
  for (int r = 0; r < LBS_ROUNDS; r++) {
    const uint64_t a = c0 + (uint64_t)r * BS + threadIdx.x;
    ss[r] = 0;
    if (a < c1) {
      valid |= 1u << r;
      uint64_t sx;
      if (in_lds) {
        uint32_t h = (uint32_t)(span - 2);
        while (l < h) {  // positions only grow: search from the last source
          const uint32_t mid = (l + h + 1) >> 1;
          if (sh.p[mid] <= a) l = mid; else h = mid - 1;
        }
        sx = lo + l;
      } else {
        sx = last_le(P, lo, hi, a);
      }
      ss[r] = (uint32_t)sx;
    }
  }
#pragma unroll
  for (int r = 0; r < LBS_ROUNDS; r++) {
    pv[r] = 0;
    if ((valid >> r) & 1u) {
      const uint64_t a = c0 + (uint64_t)r * BS + threadIdx.x;
      const uint32_t o = (uint32_t)(a - (in_lds ? sh.p[ss[r] - lo] : (uint64_t)P[ss[r]]));
      first |= (o == 0 ? 1u : 0u) << r;
      pv[r] = pre(ss[r], o);
    }
  }
  // a second batch of independent loads per round, issued before any round
  // runs: mid(s, value) gives one bit that f receives
  uint32_t known = 0;
#pragma unroll
  for (int r = 0; r < LBS_ROUNDS; r++)
    if ((valid >> r) & 1u) known |= (mid(ss[r], pv[r]) & 1u) << r;
#pragma unroll
  for (int r = 0; r < LBS_ROUNDS; r++)
    f(((valid >> r) & 1u) != 0, (uint64_t)ss[r], ((first >> r) & 1u) != 0, pv[r],
      ((known >> r) & 1u) != 0);
  __syncthreads();
}

// The flat work of every job of a launch shares one chunk space: job j owns
// ceil(width_j / LBS_CHUNK) consecutive chunks and the 1-D grid strides over
// all of them, so the blocks keep working on whichever jobs still have chunks
// and one large job never runs on a fixed slice of the chip.
struct ChunkMap {
  uint64_t cs[MAX_JOBS + 1];  // first chunk of every job; cs[njobs] = total
};

__device__ __forceinline__ uint64_t chunks_of(uint64_t positions) {
  return (positions + LBS_CHUNK - 1) / LBS_CHUNK;
}

// Thread j evaluates chunks(j), the chunk count of job j, and the block scans
// them into m.cs; ends with a barrier.  njobs <= MAX_JOBS = BS.
template <class W>
__device__ __forceinline__ void chunk_map_build(ChunkMap& m, int njobs, W chunks) {
  __shared__ uint64_t s_wtot[BS / WAVE];
  const int j = (int)threadIdx.x;
  uint64_t c = j < njobs ? chunks(j) : 0ull;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t y = __shfl_up(c, (unsigned)d);
    if ((int)lane() >= d) c += y;
  }
  const uint32_t wv = threadIdx.x / WAVE;
  if (lane() == WAVE - 1) s_wtot[wv] = c;
  __syncthreads();
  for (uint32_t w = 0; w < wv; w++) c += s_wtot[w];
  m.cs[j + 1] = c;
  if (j == 0) m.cs[0] = 0;
  __syncthreads();
}

// Chunk order with L2 locality.  The workgroups of a 1-D launch are handed
// round-robin to the NXCD dies (workgroup b to die b % NXCD).  Every pass of
// the grid over the chunk space covers gridDim.x consecutive chunks; when the
// grid is a multiple of NXCD, die x takes the x-th contiguous part of each
// pass, so the per-job data those chunks read at random (candidate bitmaps,
// CPI lists) is held in one die's L2 rather than in all of them, while the
// passes keep all dies on the same region of the chunk space.
__device__ __forceinline__ uint64_t first_chunk() {
  if (gridDim.x % NXCD) return blockIdx.x;
  return (uint64_t)(blockIdx.x % NXCD) * (gridDim.x / NXCD) + blockIdx.x / NXCD;
}

// The job owning chunk c (< cs[njobs]): the largest j with cs[j] <= c.
__device__ __forceinline__ int chunk_job(const ChunkMap& m, int njobs, uint64_t c) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (m.cs[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The blocks of a scan launch shared among its jobs in proportion to their
// scan tiles: job j, scanning items(j) positions (UINT64_MAX: it does not
// scan), gets at least one virtual block (so an empty scan still writes its
// zero total), the grid walks the virtual blocks, and body(j, nb) runs on each
// of job j's nb virtual blocks.  One large job thus gets most of the chip
// instead of a fixed row of blocks.
template <class Items, class Body>
__device__ __forceinline__ void shared_scan_blocks(int njobs, Items items, Body body) {
  __shared__ ChunkMap tm;  // tiles per job, prefix
  __shared__ ChunkMap vm;  // virtual blocks per job, prefix
  chunk_map_build(tm, njobs, [&](int j) -> uint64_t {
    const uint64_t n = items(j);
    return n == ~0ull ? 0ull : (n + SCAN_TILE - 1) / SCAN_TILE;
  });
  const uint64_t T = tm.cs[njobs], G = gridDim.x;
  chunk_map_build(vm, njobs, [&](int j) -> uint64_t {
    if (items(j) == ~0ull) return 0ull;
    const uint64_t t = tm.cs[j + 1] - tm.cs[j];
    uint64_t nb = T ? (G * t + T - 1) / T : 1;
    if (nb > t) nb = t;
    return nb ? nb : 1;
  });
  for (uint64_t vb = blockIdx.x; vb < vm.cs[njobs]; vb += gridDim.x) {
    const int jb = chunk_job(vm, njobs, vb);
    body(jb, vm.cs[jb + 1] - vm.cs[jb]);
  }
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
  const uint64_t b = (n + BS - 1) / BS;
  const int grid = (int)(b > 2048 ? 2048 : b);
  hipLaunchKernelGGL(k_fill<T>, dim3(grid), dim3(BS), 0, st, p, v, n);
}
void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, uint64_t n) { fill(st, p, v, n); }
void fill_u64(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n) { fill(st, p, v, n); }
void fill_u32(hipStream_t st, uint32_t* p, uint32_t v, uint64_t n) { fill(st, p, v, n); }

// ---------------------------------------------------------------------------
// candidate filter (Section IV-B: label candidates, degree filter, BFS
// candidate subgraph with dead-end removal as pull constraints)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t filter_items(const FilterJob& J) {
  return J.d_n ? (*J.d_n < J.cap ? *J.d_n : J.cap) : J.n_host;
}
__device__ __forceinline__ int32_t filter_item(const FilterJob& J, uint64_t i) {
  return J.list ? J.list[i] : (int32_t)i;
}

// Adjacency rows of one direction.
struct Rows {
  const uint32_t* off;
  const int32_t* nbr;
  const int32_t* lab;
};
__device__ __forceinline__ Rows plain_rows(const DevGraph& g, int dir) {
  return dir ? Rows{g.in_off, g.in_nbr, g.in_lab} : Rows{g.out_off, g.out_nbr, g.out_lab};
}
// Rows of a direct job's items, indexed base + i.
__device__ __forceinline__ Rows direct_rows(const DevGraph& g, const FilterJob& J, int dir) {
  if (!J.list) return plain_rows(g, dir);
  return dir ? Rows{g.lv_in_off, g.lv_in_nbr, g.lv_in_lab}
             : Rows{g.lv_out_off, g.lv_out_nbr, g.lv_out_lab};
}

// Degree filter of item i (vertex v): for a direct job the row offsets are
// read in item order (coalesced), otherwise gathered by vertex id.
__device__ __forceinline__ bool degree_ok(const DevGraph& g, const FilterJob& J, uint64_t i,
                                          int32_t v, unsigned long long& by) {
  const uint64_t r = J.direct ? J.base + i : (uint64_t)v;
  if (J.min_out > 0) {
    const uint32_t* off = J.direct ? direct_rows(g, J, 0).off : g.out_off;
    by += 8;
    if ((int32_t)(off[r + 1] - off[r]) < J.min_out) return false;
  }
  if (J.min_in > 0) {
    const uint32_t* off = J.direct ? direct_rows(g, J, 1).off : g.in_off;
    by += 8;
    if ((int32_t)(off[r + 1] - off[r]) < J.min_in) return false;
  }
  return true;
}

// Arrays of the edge-label blocks a job uses (blk 1: keyed by vertex and edge
// label; 2: by the far end's label too).
struct BlockArrays {
  const uint32_t* row;
  const uint32_t* start;
  const int32_t* nbr;
};
__device__ __forceinline__ BlockArrays block_arrays(const DevGraph& g, int blk, int dir) {
  return blk == 2 ? BlockArrays{g.elt_row[dir], g.elt_start[dir], g.elt_nbr[dir]}
                  : BlockArrays{g.elb_row[dir], g.elb_start[dir], g.elb_nbr[dir]};
}

// Row of bucket position p in rows [rb, re) of a block (rows ascending by
// position), or re when the bucket row has no entries there.
__device__ __forceinline__ uint32_t block_row_of(const uint32_t* rows, uint32_t rb, uint32_t re,
                                                 uint32_t p, unsigned long long& by) {
  uint32_t lo = rb, hi = re;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    by += 4;
    if (rows[mid] < p) lo = mid + 1; else hi = mid;
  }
  return (lo < re && rows[lo] == p) ? lo : re;
}

// Row lengths of (item, constraint) pairs, item-major.  A direct job needs no
// scan: its rows are contiguous.
// Algorithmic bytes (COUNT: the timing form): per pair, the item, what the
// degree filter and the row lookup read, the row's two bounds and the
// prefix written.
template <bool COUNT>
__global__ __launch_bounds__(BS) void k_filter_scan(DevGraph g, const FilterJob* __restrict__ jobs,
                                                    int njobs, unsigned long long* bytes) {
  unsigned long long by = 0;
  shared_scan_blocks(njobs, [&](int j) -> uint64_t {
    const FilterJob& J = jobs[j];
    if (!J.active || J.ncons == 0 || J.direct) return ~0ull;
    return filter_items(J) * (uint64_t)J.ncons;
  }, [&](int jb, uint64_t nb) {
    const FilterJob& J = jobs[jb];
    const uint32_t nc = (uint32_t)J.ncons;
    job_scan(filter_items(J) * nc, [&](uint64_t q) -> uint32_t {
      const uint64_t i = q / nc;
      const uint32_t c = (uint32_t)(q - i * nc);
      const int32_t v = filter_item(J, i);
      if (COUNT) by += 4 + 8;  // the item, the prefix
      if (!degree_ok(g, J, i, v, by)) return 0u;
      const PullC& cs = J.cons[c];
      if (COUNT) by += 8;  // the row's bounds
      if (cs.blk) {  // the item's run in the edge-label block
        const BlockArrays ba = block_arrays(g, cs.blk, cs.dir);
        const uint32_t r = block_row_of(ba.row, cs.rb, cs.re, g.lab_pos[v], by);
        return r < cs.re ? ba.start[r + 1] - ba.start[r] : 0u;
      }
      const uint32_t* off = cs.dir ? g.in_off : g.out_off;
      return off[v + 1] - off[v];
    }, J.sc, nb);
  });
  if (COUNT) block_add(bytes, by);
}

// Flat entries of constraint c of a direct job: its items' rows in one slice
// (the prefix P has N + 1 entries), or the rows of its edge-label block.
__device__ __forceinline__ uint64_t direct_span(const DevGraph& g, const FilterJob& J, int c,
                                                const uint32_t*& P, uint64_t& N) {
  const PullC& cs = J.cons[c];
  if (cs.blk) {
    P = block_arrays(g, cs.blk, cs.dir).start + cs.rb;
    N = cs.re - cs.rb;
  } else {
    P = direct_rows(g, J, cs.dir).off + J.base;
    N = J.n_host;
  }
  return (uint64_t)(P[N] - P[0]);
}

// Hits found by one thread, gathered per bitmap word.  A thread's positions
// are consecutive, so the words it sets (per bitmap) never decrease: it keeps
// its two latest words and masks, writing an older one out when a third
// appears.  At the end of a chunk (a point all lanes reach) the wave merges
// equal words across lanes, which hold neighbouring positions, so one lane
// per word issues the atomic instead of every lane that hit it.
__device__ __forceinline__ void wave_or_flush(uint32_t* p, uint32_t m) {
  // key of an empty slot: unique per lane, so it merges with nothing
  const uint64_t key = (p && m) ? (uint64_t)p : ~(uint64_t)lane();
  uint32_t acc = m;
  for (int off = 1; off < WAVE; off <<= 1) {
    const uint64_t k2 = __shfl_down(key, off);
    const uint32_t m2 = __shfl_down(acc, off);
    if ((int)lane() + off < WAVE && k2 == key) acc |= m2;
  }
  const uint64_t kp = __shfl_up(key, 1);
  // the first lane of a run of equal words writes the run's bits (a lane that
  // follows an empty slot may write bits already written: OR is idempotent)
  if (p && m && (lane() == 0 || kp != key)) atomicOr(p, acc);
}

struct HitRun {
  uint32_t* at[2] = {nullptr, nullptr};
  uint32_t mask[2] = {0, 0};
  // item t meets the constraint whose bitmap is hb
  __device__ void set(uint32_t* hb, uint64_t t) {
    uint32_t* w = hb + (t >> 5);
    const uint32_t bit = 1u << (t & 31u);
    if (w == at[1]) {
      mask[1] |= bit;
    } else if (w == at[0]) {
      mask[0] |= bit;
    } else {
      if (at[0] && mask[0]) atomicOr(at[0], mask[0]);
      at[0] = at[1];
      mask[0] = mask[1];
      at[1] = w;
      mask[1] = bit;
    }
  }
  // called by every lane of the wave
  __device__ void flush_wave() {
    wave_or_flush(at[0], mask[0]);
    wave_or_flush(at[1], mask[1]);
    at[0] = at[1] = nullptr;
    mask[0] = mask[1] = 0;
  }
};

// Hit bytes (hitmode 0): byte c * hit_bytes + i of hits is set to 1 by a
// plain store, once per run of a thread's positions on one (constraint, item).
__device__ __forceinline__ uint8_t* hit_bytes(const FilterJob& J, int c) {
  return (uint8_t*)J.hits + (uint64_t)c * 32 * J.hit_words;
}
struct ItemRun {
  uint8_t* last = nullptr;
  __device__ void set(uint8_t* b) {
    if (b != last) {
      *b = 1;
      last = b;
    }
  }
};

// One thread per adjacency entry: mark constraint c of item i as met.
// BITMAPS: every job of the launch records hits in bitmaps (hitmode 1), else
// in bytes (hitmode 0); one instantiation per form keeps each lean.  Both
// forms keep 8 waves per SIMD (the bitmap form spills one value for it):
// the pulls wait on scattered row and bitmap reads.
template <bool BITMAPS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8))) void k_filter_pull(DevGraph g, const FilterJob* __restrict__ jobs,
                                                    int njobs, unsigned long long* bytes) {
  __shared__ LbsShared sh;
  __shared__ ChunkMap cm;
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t {
    const FilterJob& J = jobs[j];
    if (!J.active || !J.ncons) return 0ull;
    if (!J.direct) return chunks_of(*J.sc.d_total);
    uint64_t ch = 0, N;
    const uint32_t* P;
    for (int c = 0; c < J.ncons; c++) ch += chunks_of(direct_span(g, J, c, P, N));
    return ch;
  });
  unsigned long long by = 0;
  for (uint64_t ch = first_chunk(); ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = chunk_job(cm, njobs, ch);
    const FilterJob& J = jobs[jb];
    uint64_t r = ch - cm.cs[jb];
    if (J.direct) {
      // constraint c, chunk r of its slice; positions are entries of the view
      int c = 0;
      const uint32_t* P;
      uint64_t N;
      uint64_t T = direct_span(g, J, 0, P, N);
      while (r >= chunks_of(T)) {
        r -= chunks_of(T);
        T = direct_span(g, J, ++c, P, N);
      }
      const PullC& cs = J.cons[c];
      const uint64_t c0 = P[0] + r * LBS_CHUNK;
      const uint64_t c1 = c0 + LBS_CHUNK < P[0] + T ? c0 + LBS_CHUNK : P[0] + T;
      // the job's fields in registers: the hit stores below cannot make the
      // compiler reload them
      constexpr bool bitmaps = BITMAPS;
      uint32_t* const hb = J.hits + (uint64_t)c * J.hit_words;
      uint8_t* const hb8 = hit_bytes(J, c);
      const CandSet w = cs.w;
      const int32_t elab = cs.elab;
      HitRun run;
      ItemRun irun;
      auto hit = [&](uint64_t item) {
        if constexpr (bitmaps) run.set(hb, item);
        else irun.set(hb8 + item);
      };
      if (cs.blk) {  // only e-labelled entries; the block names each row's item
        const BlockArrays ba = block_arrays(g, cs.blk, cs.dir);
        const uint32_t* rows = ba.row + cs.rb;
        const int32_t* nbr = ba.nbr;
        flat_chunk<true>(P, N, c0, c1, sh, [&](bool valid, uint64_t s, uint64_t o, uint64_t x) {
          if (!valid) return;
          by += (o == 0 ? 8 : 0) + 4;  // per row: item and start; per entry: neighbour
          if (member(w, nbr[x])) hit(rows[s]);
        });
      } else {
        const Rows rw = direct_rows(g, J, cs.dir);
        flat_chunk<true>(P, N, c0, c1, sh, [&](bool valid, uint64_t i, uint64_t o, uint64_t x) {
          if (!valid) return;
          // per entry: neighbour (+ label); the items' offsets stream once
          by += (o == 0 ? 4 : 0) + 4 + (elab != ANY ? 4 : 0);
          if (elab != ANY && rw.lab[x] != elab) return;
          if (member(w, rw.nbr[x])) hit(i);
        });
      }
      if constexpr (bitmaps) run.flush_wave();
    } else {
      const uint32_t nc = (uint32_t)J.ncons;
      const uint64_t NP = filter_items(J) * (uint64_t)nc;
      const uint64_t T = *J.sc.d_total;
      const uint64_t c0 = r * LBS_CHUNK;
      const uint64_t c1 = c0 + LBS_CHUNK < T ? c0 + LBS_CHUNK : T;
      constexpr bool bitmaps = BITMAPS;
      uint32_t* const hits = J.hits;
      const uint64_t hwords = J.hit_words;
      const int32_t* const list = J.list;
      HitRun run;
      ItemRun irun;
      uint64_t run_q = ~0ull;  // the (item, constraint) pair whose block row is run_x
      uint32_t run_x = 0;
      flat_chunk<true>(J.sc.P, NP, c0, c1, sh, [&](bool valid, uint64_t q, uint64_t o, uint64_t) {
        if (!valid) return;
        const uint64_t i = q / nc;
        const uint32_t c = (uint32_t)(q - i * nc);
        const PullC& cs = J.cons[c];
        const int32_t v = list ? list[i] : (int32_t)i;
        int32_t w;
        if (cs.blk) {  // only the item's run in the edge-label block
          const BlockArrays ba = block_arrays(g, cs.blk, cs.dir);
          if (q != run_q) {  // found once per run of this thread's positions
            run_q = q;
            run_x = ba.start[block_row_of(ba.row, cs.rb, cs.re, g.lab_pos[v], by)];
            by += 12;  // item, bucket position, start
          }
          w = ba.nbr[run_x + (uint32_t)o];
          by += 4;
        } else {
          const Rows rw = plain_rows(g, cs.dir);
          const uint32_t x = rw.off[v] + (uint32_t)o;
          // per row: item and its two offsets; per entry: neighbour (+ label)
          by += (o == 0 ? 12 : 0) + 4 + (cs.elab != ANY ? 4 : 0);
          if (cs.elab != ANY && rw.lab[x] != cs.elab) return;
          w = rw.nbr[x];
        }
        if (!member(cs.w, w)) return;
        if constexpr (bitmaps) run.set(hits + (uint64_t)c * hwords, i);
        else irun.set((uint8_t*)hits + (uint64_t)c * 32 * hwords + i);
      });
      if constexpr (bitmaps) run.flush_wave();
    }
  }
  if (bytes) block_add(bytes, by);
}

// Items meeting the degree filter and every constraint join C(u) (a set: no
// fixed order).  The items of all jobs share one chunk space: a chunk is
// LBS_CHUNK items with hit bytes (8 consecutive items per thread), or 32 * BS
// items when the launch's jobs have hit bitmaps (one 32-item word per thread,
// whose constraint words, ANDed, pick the items to examine, so items no
// constraint touched cost a bit, not a load).  Hit bytes and words are
// cleared as they are read.  A block reserves its output with one atomic add, and runs of
// members in one bitmap word are set with one atomic.
// BITMAPS: every job of the launch has hit bitmaps (hitmode 1).
template <bool BITMAPS>
__global__ __launch_bounds__(BS) void k_filter_compact(DevGraph g,
                                                       const FilterJob* __restrict__ jobs,
                                                       int njobs, unsigned long long* bytes) {
  constexpr int IPT = (int)(LBS_CHUNK / BS);
  static_assert(IPT == 8, "hit bytes are read as one 8-byte word per thread and constraint");
  __shared__ ChunkMap cm;
  __shared__ unsigned long long s_base;
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t {
    const FilterJob& J = jobs[j];
    if (!J.active) return 0ull;
    constexpr uint64_t per = BITMAPS ? 32ull * BS : LBS_CHUNK;
    return (filter_items(J) + per - 1) / per;
  });
  unsigned long long by = 0;
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(chunk_job(cm, njobs, ch));
    const FilterJob& J = jobs[jb];
    const uint64_t N = filter_items(J);
    // candidates of this thread: items i0 + r for the set bits r of m
    uint64_t i0;
    uint32_t m = 0;
    if constexpr (BITMAPS) {
      const uint64_t wi = (ch - cm.cs[jb]) * BS + threadIdx.x;
      i0 = 32 * wi;
      if (i0 < N) m = N - i0 >= 32 ? ~0u : ((1u << (N - i0)) - 1u);
      if (m)
        for (int c = 0; c < J.ncons; c++) {
          uint32_t* hw = J.hits + (uint64_t)c * J.hit_words + wi;
          const uint32_t x = *hw;
          by += 4;
          if (x) *hw = 0;
          m &= x;
        }
    } else {
      // IPT == 8 items: one aligned 8-byte word of hit bytes per constraint
      i0 = (ch - cm.cs[jb]) * LBS_CHUNK + (uint64_t)threadIdx.x * IPT;
      if (i0 < N) m = N - i0 >= IPT ? (1u << IPT) - 1u : ((1u << (N - i0)) - 1u);
      if (m)
        for (int c = 0; c < J.ncons; c++) {
          uint64_t* hw = (uint64_t*)(hit_bytes(J, c) + i0);
          const uint64_t x = *hw;
          by += 8;
          if (x) *hw = 0;
          uint32_t nz = 0;
#pragma unroll
          for (int r = 0; r < IPT; r++) nz |= (((x >> (8 * r)) & 0xFFu) != 0 ? 1u : 0u) << r;
          m &= nz;
        }
    }
    uint32_t keep = 0;  // bit r: item i0 + r joins
    for (uint32_t q = m; q; q &= q - 1) {
      const int r = __ffs(q) - 1;
      const uint64_t i = i0 + r;
      const int32_t v = filter_item(J, i);
      by += J.list ? 4 : 0;
      bool ok = !J.keep || ((J.keep[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u);
      ok = ok && degree_ok(g, J, i, v, by);
      keep |= (ok ? 1u : 0u) << r;
    }
    uint32_t total;
    const uint32_t rank = block_excl_scan((uint32_t)__popc(keep), total);
    if (threadIdx.x == 0)
      s_base = total ? atomicAdd((unsigned long long*)J.d_out_n, (unsigned long long)total) : 0ull;
    __syncthreads();
    uint64_t idx = s_base + rank;
    uint32_t word = 0xFFFFFFFFu, mask = 0;
    for (uint32_t q = keep; q; q &= q - 1) {
      const int r = __ffs(q) - 1;
      const int32_t v = filter_item(J, i0 + r);
      if (idx < J.out_cap) {
        J.out[idx] = v;
        // a direct labelled filter's item index is the bucket position itself
        if (J.pos) J.pos[J.pos_by_bucket && J.direct && J.list ? (uint32_t)(i0 + r)
                                                                : pos_index(g, J.pos_by_bucket, v)] = (int32_t)idx;
      } else {  // the host's bound on |C(u)| does not hold: reported, nothing written
        atomicOr(J.sc.err, 2u);
      }
      idx++;
      by += 12;
      const uint32_t w = (uint32_t)v >> 5;
      if (w != word) {
        if (mask) atomicOr(&J.bits[word], mask);
        word = w;
        mask = 0;
      }
      mask |= 1u << ((uint32_t)v & 31u);
    }
    if (mask) atomicOr(&J.bits[word], mask);
    __syncthreads();
  }
  if (bytes) block_add(bytes, by);
}

__global__ __launch_bounds__(BS) void k_filter_clear(const FilterJob* __restrict__ jobs) {
  const FilterJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  for (uint64_t w = (uint64_t)blockIdx.x * BS + threadIdx.x; w < J.nwords;
       w += (uint64_t)gridDim.x * BS)
    J.bits[w] = 0;
}

void filter_scan(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                 unsigned long long* bytes) {
  if (bytes) hipLaunchKernelGGL(k_filter_scan<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else hipLaunchKernelGGL(k_filter_scan<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}
void filter_pull(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                 bool bitmaps, unsigned long long* bytes) {
  if (bitmaps)
    hipLaunchKernelGGL(k_filter_pull<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else
    hipLaunchKernelGGL(k_filter_pull<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}
void filter_compact(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                    bool bitmaps, unsigned long long* bytes) {
  if (bitmaps)
    hipLaunchKernelGGL(k_filter_compact<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else
    hipLaunchKernelGGL(k_filter_compact<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}
void filter_clear(hipStream_t st, const FilterJob* jobs, int njobs, int gx) {
  hipLaunchKernelGGL(k_filter_clear, dim3(gx, njobs), dim3(BS), 0, st, jobs);
}

// ---------------------------------------------------------------------------
// CPI adjacency lists for one spanning-tree edge (p, u) per job
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t cpi_sources(const CpiJob& J) {
  return *J.p.cnt < J.cap_p ? *J.p.cnt : J.cap_p;
}

// Entry x of the row of v_p: kept when its far end is in C(u), its label is
// `prim` and the reverse direction meets `other`.
__device__ __forceinline__ bool cpi_keep(const DevGraph& g, const CpiJob& J, int32_t vp,
                                         uint32_t x, int32_t& v, unsigned long long& by) {
  v = (J.dir ? g.in_nbr : g.out_nbr)[x];
  by += 4;
  if (J.prim != ANY) {
    by += 4;
    if ((J.dir ? g.in_lab : g.out_lab)[x] != J.prim) return false;
  }
  if (!member(J.u, v)) return false;
  if (J.other == PC_FREE) return true;
  // dir 0 scanned vp -> v, so the reverse is v -> vp; dir 1 the opposite
  // in the row of the source vp, shared by the threads of its entries
  return J.dir ? pair_ok(g, vp, v, true, J.other, by) : pair_ok(g, v, vp, false, J.other, by);
}

// Row lengths of the members of C(p); clears the per-source counters.
// Algorithmic bytes (COUNT): per parent candidate, the candidate, its row's
// bounds, the two list heads cleared and the prefix written (28).
template <bool COUNT>
__global__ __launch_bounds__(BS) void k_cpi_scan(DevGraph g, const CpiJob* __restrict__ jobs,
                                                 int njobs, unsigned long long* bytes) {
  unsigned long long by = 0;
  shared_scan_blocks(njobs, [&](int j) -> uint64_t {
    return jobs[j].active ? cpi_sources(jobs[j]) : ~0ull;
  }, [&](int jb, uint64_t nb) {
    const CpiJob& J = jobs[jb];
    const uint32_t* off = J.dir ? g.in_off : g.out_off;
    job_scan(cpi_sources(J), [&](uint64_t s) -> uint32_t {
      const int32_t vp = J.p.list[s];
      J.len[s] = 0;
      J.cur[s] = 0;
      if (COUNT) by += 28;
      return off[vp + 1] - off[vp];
    }, J.sc, nb);
  });
  if (COUNT) block_add(bytes, by);
}

// Entry v (far end, label already prim) of the row of v_p in an edge-label
// block: kept when v is in C(u) and the reverse direction meets `other`.
__device__ __forceinline__ bool cpi_keep_v(const DevGraph& g, const CpiJob& J, int32_t vp,
                                           int32_t v, unsigned long long& by) {
  if (!member(J.u, v)) return false;
  if (J.other == PC_FREE) return true;
  return J.dir ? pair_ok(g, vp, v, true, J.other, by) : pair_ok(g, v, vp, false, J.other, by);
}

// Whether the job streams the edge-label block of p's bucket (entries labelled
// prim only, members of C(p) picked out by its bitmap) instead of the whole
// rows of C(p)'s members: when the block is at most twice those rows.
__device__ __forceinline__ bool cpi_direct(const DevGraph& g, const CpiJob& J) {
  if (!J.blk) return false;
  const uint32_t* P = block_arrays(g, J.blk, J.dir).start;
  return (uint64_t)(P[J.re] - P[J.rb]) <= 2ull * *J.sc.d_total;
}

// Chunk space of the CPI kernels: the block's entries, or every adjacency
// entry of every member of C(p).
__device__ __forceinline__ uint64_t cpi_chunks(const DevGraph& g, const CpiJob& J) {
  if (!J.active) return 0ull;
  if (cpi_direct(g, J)) {
    const uint32_t* P = block_arrays(g, J.blk, J.dir).start;
    return chunks_of(P[J.re] - P[J.rb]);
  }
  return chunks_of(*J.sc.d_total);
}

// Runs f(valid, s, v) over chunk r of job J: s the member's index in C(p), v
// a kept entry of its list (valid false for positions outside the job or
// entries that are not kept; uniform call count).
template <class F>
__device__ __forceinline__ void cpi_chunk(const DevGraph& g, const CpiJob& J, uint64_t r,
                                          LbsShared& sh, unsigned long long& by, F f) {
  if (cpi_direct(g, J)) {
    const BlockArrays ba = block_arrays(g, J.blk, J.dir);
    const uint32_t* P = ba.start + J.rb;
    const uint64_t N = J.re - J.rb, T = P[N] - P[0];
    const uint64_t c0 = P[0] + r * LBS_CHUNK;
    const uint64_t c1 = c0 + LBS_CHUNK < P[0] + T ? c0 + LBS_CHUNK : P[0] + T;
    const uint32_t* rows = ba.row + J.rb;
    const int32_t* nbr = ba.nbr;
    flat_chunk<true>(P, N, c0, c1, sh, [&](bool valid, uint64_t s, uint64_t o, uint64_t x) {
      if (!valid) return;
      const int32_t vp = g.lab_vtx[J.base + rows[s]];
      by += (o == 0 ? 12 : 0);  // per row: position, start, vertex
      if (!member(J.p, vp)) return;
      const int32_t v = nbr[x];
      by += 4;
      // the block's rows are bucket positions of p's label
      if (cpi_keep_v(g, J, vp, v, by)) f((uint64_t)J.p.pos[J.p.by_bucket ? rows[s] : (uint32_t)vp], v);
    });
  } else {
    const uint32_t* off = J.dir ? g.in_off : g.out_off;
    const uint64_t T = *J.sc.d_total;
    const uint64_t c0 = r * LBS_CHUNK;
    const uint64_t c1 = c0 + LBS_CHUNK < T ? c0 + LBS_CHUNK : T;
    flat_chunk<true>(J.sc.P, cpi_sources(J), c0, c1, sh, [&](bool valid, uint64_t s, uint64_t o, uint64_t) {
      if (!valid) return;
      const int32_t vp = J.p.list[s];
      int32_t v;
      by += 8;
      if (cpi_keep(g, J, vp, off[vp] + (uint32_t)o, v, by)) f(s, v);
    });
  }
}

// Two passes per tree edge (the bounded path, whose job may not fit its
// members' rows in the arena): count the kept entries of every member, give
// each member a list of that length, then fill.
__global__ __launch_bounds__(BS) void k_cpi_count(DevGraph g, const CpiJob* __restrict__ jobs,
                                                  int njobs, unsigned long long* bytes) {
  __shared__ LbsShared sh;
  __shared__ ChunkMap cm;
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t { return cpi_chunks(g, jobs[j]); });
  unsigned long long by = 0;
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = chunk_job(cm, njobs, ch);
    const CpiJob& J = jobs[jb];
    cpi_chunk(g, J, ch - cm.cs[jb], sh, by, [&](uint64_t s, int32_t) { atomicAdd(&J.len[s], 1u); });
  }
  if (bytes) block_add(bytes, by);
}

// Each tile of members reserves their lists in the arena with one atomic add.
__global__ __launch_bounds__(BS) void k_cpi_alloc(DevGraph g, const CpiJob* __restrict__ jobs) {
  __shared__ unsigned long long s_base;
  const CpiJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  const uint64_t N = cpi_sources(J);
  for (uint64_t t0 = (uint64_t)blockIdx.x * BS; t0 < N; t0 += (uint64_t)gridDim.x * BS) {
    const uint64_t s = t0 + threadIdx.x;
    const uint32_t len = s < N ? J.len[s] : 0u;
    uint32_t total;
    const uint32_t pre = block_excl_scan(len, total);
    if (threadIdx.x == 0)
      s_base = total ? atomicAdd(J.arena_cursor, (unsigned long long)total) : 0ull;
    __syncthreads();
    if (s < N) {
      if (s_base + total > J.arena_cap) {  // out of arena: the job is redone in bounded mode
        J.len[s] = 0;
        J.beg[s] = 0;
        if (threadIdx.x == 0) atomicOr(J.flags, 4u);
      } else {
        J.beg[s] = (uint32_t)(s_base + pre);
      }
    }
    __syncthreads();
  }
}

// One pass per tree edge: the job reserves, in one atomic add, a region of
// the arena as large as the rows of C(p)'s members (the scan's total), and
// member s's list starts at the region's base plus the row prefix P[s] -- its
// row bounds its list.  A job past the arena is redone in bounded mode.
__global__ void k_cpi_reserve(const CpiJob* __restrict__ jobs) {
  const CpiJob& J = jobs[blockIdx.y];
  if (!J.active || threadIdx.x != 0) return;
  const uint64_t total = cpi_sources(J) ? *J.sc.d_total : 0ull;
  const uint64_t base = total ? atomicAdd(J.arena_cursor, (unsigned long long)total) : 0ull;
  *J.d_asked += total;  // one thread per job; the job's edges reserve one launch after another
  if (base + total > J.arena_cap) {
    atomicOr(J.flags, 4u);
    *J.d_base = ~0ull;
  } else {
    *J.d_base = base;
  }
}

// Kept entries go to their member's list.  ONEPASS: at the member's row
// prefix in the job's reserved region, the list length being the member's
// cursor, and the first entry also records the list's start; otherwise into
// the list the counting pass sized.
template <bool ONEPASS>
__global__ __launch_bounds__(BS) void k_cpi_fill(DevGraph g, const CpiJob* __restrict__ jobs,
                                                 int njobs, unsigned long long* bytes) {
  __shared__ LbsShared sh;
  __shared__ ChunkMap cm;
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t { return cpi_chunks(g, jobs[j]); });
  unsigned long long by = 0, dummy = 0;
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = chunk_job(cm, njobs, ch);
    const CpiJob& J = jobs[jb];
    if constexpr (ONEPASS) {
      const uint64_t base = *J.d_base;
      if (base == ~0ull) continue;  // out of arena (uniform per chunk)
      cpi_chunk(g, J, ch - cm.cs[jb], sh, by, [&](uint64_t s, int32_t v) {
        const uint64_t start = base + J.sc.P[s];
        const uint32_t at = atomicAdd(&J.len[s], 1u);
        J.arena[start + at] = v;
        if (at == 0) J.beg[s] = (uint32_t)start;
        by += 4 + (at == 0 ? 12 : 0);  // the entry; per list: prefix, start
      });
    } else {
      cpi_chunk(g, J, ch - cm.cs[jb], sh, dummy, [&](uint64_t s, int32_t v) {
        const uint32_t at = atomicAdd(&J.cur[s], 1u);
        if (at < J.len[s]) {
          J.arena[(uint64_t)J.beg[s] + at] = v;
          by += 4;
        }
      });
    }
  }
  if (bytes) block_add(bytes, by);
}

void cpi_scan(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
              unsigned long long* bytes) {
  if (bytes) hipLaunchKernelGGL(k_cpi_scan<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else hipLaunchKernelGGL(k_cpi_scan<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}
void cpi_reserve(hipStream_t st, const CpiJob* jobs, int njobs) {
  hipLaunchKernelGGL(k_cpi_reserve, dim3(1, njobs), dim3(64), 0, st, jobs);
}
void cpi_count(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
               unsigned long long* bytes) {
  hipLaunchKernelGGL(k_cpi_count, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}
void cpi_alloc(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int gx) {
  hipLaunchKernelGGL(k_cpi_alloc, dim3(gx, njobs), dim3(BS), 0, st, g, jobs);
}
void cpi_fill(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
              bool onepass, unsigned long long* bytes) {
  if (onepass)
    hipLaunchKernelGGL(k_cpi_fill<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else
    hipLaunchKernelGGL(k_cpi_fill<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}

// ---------------------------------------------------------------------------
// enumeration (Section IV-B matching over the CPI) with the fused literal
// check (Section II: h |= X implies h |= Y)
// ---------------------------------------------------------------------------

template <class T, int N>
__device__ __forceinline__ T pick(const T (&h)[N], int idx) {
  // masks, not selects: a select chain over a runtime index is turned back
  // into an indexed private array, which lives in scratch memory
  T r = 0;
#pragma unroll
  for (int j = 0; j < N; j++) r |= h[j] & (T)(0 - (T)(j == idx));
  return r;
}

template <class Col>
__device__ __forceinline__ bool literal_holds(const DevGraph& g, const DevLit& l, Col col) {
  const int32_t x = g.attr[(int64_t)l.attr * g.n + col(l.pos)];
  if (l.kind == 0) return x != ABSENT && x == l.value;
  const int32_t y = g.attr[(int64_t)l.attr2 * g.n + col(l.pos2)];
  return x != ABSENT && y != ABSENT && x == y;
}

// Whether the complete match h (matching order) orders after the staging
// threshold in variable order (or equals it when the threshold is exclusive).
__device__ __forceinline__ bool past_threshold(const ExtJob& J, const int32_t (&h)[MAXK],
                                               const int32_t* thr) {
  int c = 0;
#pragma unroll
  for (int v = 0; v < MAXK; v++)
    if (c == 0 && v < J.k) {
      const uint32_t x = (uint32_t)pick(h, J.var_pos[v]), y = (uint32_t)thr[v];
      c = x < y ? -1 : (x > y ? 1 : 0);
    }
  return c > 0 || (c == 0 && !J.thr_incl);
}

// The same on the tuple already in variable order.
__device__ __forceinline__ bool past_threshold_t(const ExtJob& J, const int32_t (&t)[MAXK],
                                                 const int32_t* thr) {
  int c = 0;
#pragma unroll
  for (int v = 0; v < MAXK; v++)
    if (c == 0 && v < J.k) {
      const uint32_t x = (uint32_t)t[v], y = (uint32_t)thr[v];
      c = x < y ? -1 : (x > y ? 1 : 0);
    }
  return c > 0 || (c == 0 && !J.thr_incl);
}

struct FinalAcc {
  unsigned long long match, viol, mfp, vfp;
};

// One complete match h (matching order): count it, fingerprint it in variable
// order, check X -> Y; returns whether a violation must be staged (it
// precedes the current threshold); `t` then holds it in variable order.
// col(p) reads the match at matching-order position p again (p is the
// same for the whole wave): a cached load or a register, cheaper than
// selecting the entry out of h.
template <class Col>
__device__ __forceinline__ bool finalize(const DevGraph& g, const ExtJob& J,
                                         const int32_t (&h)[MAXK], int32_t (&t)[MAXK],
                                         FinalAcc& acc, bool count, bool thr_on,
                                         const int32_t* thr, unsigned long long& by, Col col,
                                         Units* U = nullptr) {
  uint64_t hs = 0x9E3779B97F4A7C15ull * (uint64_t)J.k;
#pragma unroll
  for (int v = 0; v < MAXK; v++) {
    t[v] = v < J.k ? col(J.var_pos[v]) : 0;
    if (v < J.k) hs = mix64(hs ^ (uint64_t)(uint32_t)t[v]);
  }
  bool X = true, Y = !J.y_false;
  for (int j = 0; j < J.nx && X; j++) {
    X = literal_holds(g, J.lit[j], col);
    by += J.lit[j].kind == 0 ? 4 : 8;  // the attribute values read
    if (U) U->c[U_LIT_READS] += J.lit[j].kind == 0 ? 1 : 2;
  }
  if (X && Y)
    for (int j = 0; j < J.ny && Y; j++) {
      Y = literal_holds(g, J.lit[J.nx + j], col);
      by += J.lit[J.nx + j].kind == 0 ? 4 : 8;
      if (U) U->c[U_LIT_READS] += J.lit[J.nx + j].kind == 0 ? 1 : 2;
    }
  if (count) {
    acc.match += 1;
    acc.mfp += hs;
    if (U) U->c[U_MATCHES]++;
  }
  if (!(X && !Y)) return false;
  if (count) {
    acc.viol += 1;
    acc.vfp += hs;
    if (U) U->c[U_VIOLATIONS]++;
  }
  if (J.vcap == 0) return false;
  // stage only if t < thr (t <= thr when thr_incl), lexicographically on unsigned ids
  return !(thr_on && past_threshold_t(J, t, thr));
}

// Whether a job's staging is already past its capacity: a wave that starts
// work on such a job drops its tuples without touching the counter (the
// count already shows the overflow).  A stale read only costs one more
// atomic add.
__device__ __forceinline__ bool staging_past_cap(const ExtJob& J) {
  return __hip_atomic_load(J.d_vcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > J.vcap;
}

// Wave-aggregated append of violating tuples to the job's staging buffer.
// `full` (wave-uniform) becomes true once this wave's append has pushed the
// count past vcap; from then on the wave drops its tuples without touching
// the counter, so a GFD with millions of violations does not keep hammering
// one address.  The host detects the overflow as count > vcap, which holds
// from the first dropped tuple on (an exactly full buffer is not an overflow).
__device__ __forceinline__ void stage(const ExtJob& J, bool want, const int32_t (&t)[MAXK],
                                      bool& full) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  if (full) return;
  const int leader = __ffsll((long long)m) - 1;
  const unsigned long long cnt = (unsigned long long)__popcll(m);
  unsigned long long base = 0;
  if ((int)lane() == leader) base = atomicAdd((unsigned long long*)J.d_vcount, cnt);
  base = __shfl(base, leader);
  // only once the count is past vcap: the host then sees the overflow
  if (base + cnt > J.vcap) full = true;
  if (want) {
    const uint64_t slot = base + rank_below(m);
    if (slot < J.vcap) {
      int32_t* dst = J.vbuf + slot * (uint64_t)J.k;
#pragma unroll
      for (int v = 0; v < MAXK; v++)
        if (v < J.k) dst[v] = t[v];
    }
  }
}


__device__ __forceinline__ void flush_acc(unsigned long long* counters, FinalAcc acc) {
  __shared__ unsigned long long s_acc[4][BS / WAVE];
  acc.match = wave_sum(acc.match);
  acc.viol = wave_sum(acc.viol);
  acc.mfp = wave_sum(acc.mfp);
  acc.vfp = wave_sum(acc.vfp);
  const uint32_t wv = threadIdx.x / WAVE;
  __syncthreads();
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
    if (s) atomicAdd(&counters[threadIdx.x], s);
  }
}

__device__ __forceinline__ uint64_t ext_sources(const ExtJob& J) {
  return *J.d_nsrc < J.src_cap ? *J.d_nsrc : J.src_cap;
}

// Whether every extension of source s orders past the threshold: its bound
// variables, read in variable order up to the first unbound one, already
// exceed thr.
__device__ __forceinline__ bool source_past(const ExtJob& J, uint64_t s,
                                            const int32_t (&thr)[MAXK], unsigned long long& by) {
  for (int v = 0; v < J.k; v++) {
    const int p = J.var_pos[v];
    if (p >= J.i) return false;  // unbound: undecided
    by += 4;
    const uint32_t x = (uint32_t)J.src_cols[(uint64_t)p * J.src_stride + s];
    const uint32_t y = (uint32_t)thr[v];
    if (x != y) return x > y;
  }
  return false;
}

// CPI list length of every partial match's spanning-tree parent.
// Algorithmic bytes (COUNT): per source, the prefix written, the bound words
// the threshold test reads, and (when it gets attempts) the parent's vertex
// and position, its list's bounds and the list start written.
template <bool COUNT>
__global__ __launch_bounds__(BS) void k_ext_scan(DevGraph g, const ExtJob* __restrict__ jobs,
                                                 int njobs, unsigned long long* bytes) {
  unsigned long long by = 0;
  shared_scan_blocks(njobs, [&](int j) -> uint64_t {
    return jobs[j].active && !jobs[j].deferred ? ext_sources(jobs[j]) : ~0ull;
  }, [&](int jb, uint64_t nb) {
    const ExtJob& J = jobs[jb];
    const int32_t* par = J.src_cols + (uint64_t)J.par_pos * J.src_stride;
    const bool prune = J.prune && J.thr != nullptr && *J.d_thr_valid != 0;
    int32_t thr[MAXK];
#pragma unroll
    for (int v = 0; v < MAXK; v++) thr[v] = prune && v < J.k ? J.thr[v] : 0;
    const uint64_t xn = J.cross ? (*J.cross_n < J.cross_cap ? *J.cross_n : J.cross_cap) : 0ull;
    job_scan(ext_sources(J), [&](uint64_t s) -> uint32_t {
      if (COUNT) by += 8;  // the prefix
      // a source the threshold rules out gets no attempts, so its list start
      // is never read: decided first, it skips the parent's row lookups
      if (prune && source_past(J, s, thr, by)) return 0u;
      if (J.cross) {  // all of the new component root's candidates
        J.begs[s] = 0;
        if (COUNT) by += 4;
        return (uint32_t)xn;
      }
      const int32_t c = J.par_posmap[pos_index(g, J.par_by_bucket, par[s])];
      J.begs[s] = J.cpi_beg[c];
      if (COUNT) by += 20;
      return J.cpi_len[c];
    }, J.sc, nb);
  });
  if (COUNT) block_add(bytes, by);
}

// Attempt window of one job in the launch's chunk space (0 for a job of the
// other variant: a job at its last level has no next frontier, and the
// inner-level variant skips it, and the other way round).
template <bool LAST>
__device__ __forceinline__ uint64_t ext_width(const ExtJob& J) {
  if (!J.active || J.deferred || (J.last != 0) != LAST) return 0;
  const uint64_t T = ext_sources(J) ? *J.sc.d_total : 0ull;
  const uint64_t A1 = J.a_end < T ? J.a_end : T;
  return A1 > J.a_begin ? A1 - J.a_begin : 0ull;
}

// WAVES: the least number of waves per SIMD the register allocation must
// allow (1: the compiler's own choice; 8: at most 64 VGPRs per lane, the rest
// spilled).  The last level waits on chains of dependent loads; where they go
// to HBM, more waves in flight pay for the spills.
template <bool LAST, bool AHEAD, int WAVES>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WAVES)))
void k_ext_run(DevGraph g, const ExtJob* __restrict__ jobs, int njobs, unsigned long long* bytes) {
  __shared__ LbsShared sh;
  __shared__ ChunkMap cm;
  __shared__ unsigned long long s_wcnt[BS / WAVE];
  __shared__ unsigned long long s_woff[BS / WAVE];
  __shared__ int32_t s_thr[MAXK];
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t { return chunks_of(ext_width<LAST>(jobs[j])); });
  const uint32_t wv = threadIdx.x / WAVE;
  unsigned long long by = 0;
#ifdef GFD_COUNT_UNITS
  Units units{};
  Units* U = &units;
#else
  Units* U = nullptr;
#endif
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = chunk_job(cm, njobs, ch);
    const ExtJob& J = jobs[jb];
    const uint64_t N = ext_sources(J);
    const uint64_t T = *J.sc.d_total;  // N > 0: the job owns chunks
    const uint64_t A1 = J.a_end < T ? J.a_end : T;
    const uint64_t c0 = J.a_begin + (ch - cm.cs[jb]) * LBS_CHUNK;
    const uint64_t c1 = c0 + LBS_CHUNK < A1 ? c0 + LBS_CHUNK : A1;
    const int i = J.i;
    FinalAcc acc{0, 0, 0, 0};
    bool thr_on = false, full = LAST && staging_past_cap(J);
    if (LAST) {
      // the staging threshold, shared through LDS: written before the first
      // barrier of the chunk (the previous chunk ended on one), read after it
      thr_on = J.thr != nullptr && *J.d_thr_valid != 0;
      if (threadIdx.x < MAXK)
        s_thr[threadIdx.x] = thr_on && (int)threadIdx.x < J.k ? J.thr[threadIdx.x] : 0;
    }
    const int32_t* thr = s_thr;
    auto cpi_entry = [&](uint32_t s, uint32_t o) -> int32_t {
      return J.cpi_ent[(uint64_t)J.begs[s] + o];
    };
    // AHEAD: the first probe's table slot for every round at once; a free
    // slot settles that probe (the pair is not adjacent), and the eight
    // lookups overlap instead of waiting one round each.  It costs registers
    // (4 waves per SIMD instead of 5), which pays where the graph sits in
    // cache and the kernel waits on issue and cache latency, not on HBM.
    auto first_probe_free = [&](uint32_t s, int32_t v) -> uint32_t {
      if (!AHEAD || J.nchk == 0 || J.chk_fwd[0] == PC_FREE || J.chk_bwd[0] == PC_FREE) return 0u;
      const int32_t hw = J.src_cols[(uint64_t)J.chk_pos[0] * J.src_stride + s];
      const uint64_t t0 = g.hub_off[hw], t1 = g.hub_off[hw + 1];
      if (t1 <= t0) return 0u;
      return g.hub_tab[t0 + hub_slot(v, t1 - t0)] == 0 ? 1u : 0u;
    };
    flat_chunk_pre(J.sc.P, N, c0, c1, sh, cpi_entry, first_probe_free,
                   [&](bool valid, uint64_t s, bool first, int32_t v, bool free0) {
      int32_t h[MAXK];
      bool ok = false;
      if (valid) {
        // the CPI entry; the source's list start, prefix and partial once per source
        by += 4 + (first ? 12ull + 4ull * (uint64_t)i : 0ull);
        if (U) {
          U->c[LAST ? U_ATTEMPTS : U_INNER_ATTEMPTS]++;
          if (LAST && first) U->c[U_SOURCES]++;
        }
        ok = true;
#pragma unroll
        for (int j = 0; j < MAXK; j++) {
          h[j] = (j < i) ? J.src_cols[(uint64_t)j * J.src_stride + s] : v;
          if (j < i && h[j] == v) ok = false;
        }
        if (U && LAST && ok) U->c[U_INJECTIVE]++;
        // a collect-only pass keeps nothing past its threshold: such tuples
        // skip the edge probes and the literal check
        if (LAST && ok && thr_on && J.collect_only) ok = !past_threshold(J, h, thr);
        for (int c = 0; c < J.nchk && ok; c++) {
          const int32_t hw = pick(h, J.chk_pos[c]);
          const int32_t cf = J.chk_fwd[c], cb = J.chk_bwd[c];
          // rows of hw, which the wave's threads share: the combined row when
          // both directions are constrained, else the one direction's row
          Units* UL = LAST ? U : nullptr;  // units of the last level only
          if (cf != PC_FREE && cb != PC_FREE) {
            int2 l;
            if (UL) UL->c[U_CHK_BOTH]++;
            if (c == 0 && free0) {
              l = make_int2(NOEDGE, NOEDGE);
              by += 17;  // what the probe reads: the table bounds and one slot
              if (UL) {
                UL->c[U_TABLE_FREE]++;
                UL->c[U_BOTH_LOG2D] += clog2(g.sym_off[hw + 1] - g.sym_off[hw]);
              }
            } else {
              l = edge_labels_both(g, hw, v, by, UL);
            }
            ok = constraint_ok(l.x, cf) && constraint_ok(l.y, cb);
          } else {
            ok = pair_ok(g, hw, v, true, cf, by, UL) && pair_ok(g, v, hw, false, cb, by, UL);
          }
        }
      }
      if (!LAST) {  // block-aggregated append to the next frontier
        // s_wcnt is read only by thread 0 before the second barrier and s_woff
        // only written by it between the barriers, so a wave running ahead
        // into the next round cannot overwrite what a slower wave still reads
        const uint64_t m = __ballot(ok);
        if (lane() == 0) s_wcnt[wv] = (unsigned long long)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
          unsigned long long tot = 0;
          for (int w = 0; w < BS / WAVE; w++) tot += s_wcnt[w];
          unsigned long long base = tot ? atomicAdd((unsigned long long*)J.d_ndst, tot) : 0ull;
          if (tot && base + tot > J.dst_cap) atomicOr(J.flags, 1u);  // the job is redone bounded
          for (int w = 0; w < BS / WAVE; w++) {
            s_woff[w] = base;
            base += s_wcnt[w];
          }
        }
        __syncthreads();
        if (ok) {
          const unsigned long long slot = s_woff[wv] + rank_below(m);
          if (slot < J.dst_cap) {
#pragma unroll
            for (int j = 0; j < MAXK; j++)
              if (j <= i) J.dst_cols[(uint64_t)j * J.dst_cap + slot] = h[j];
            by += 4ull * (uint64_t)(i + 1);
          }
        }
      } else {
        int32_t t[MAXK];
        bool want = false;
        if (ok)
          want = finalize(g, J, h, t, acc, !J.collect_only, thr_on, thr, by, [&](int p) -> int32_t {
            return p < i ? J.src_cols[(uint64_t)p * J.src_stride + s] : v;
          }, U);
        stage(J, want, t, full);
      }
    });
    if (LAST && !J.collect_only) flush_acc(J.counters, acc);
  }
  if (bytes) block_add(bytes, by);
#ifdef GFD_COUNT_UNITS
  for (int u = 0; u < UNIT_KINDS; u++) block_add(&unit_counts[u], units.c[u]);
#endif
}

// Unit counts of a counting build (see Units); nothing in a normal build.
#ifdef GFD_COUNT_UNITS
__device__ unsigned long long unit_counts[UNIT_KINDS];
bool units_counted() { return true; }
static unsigned long long* unit_counts_ptr() {
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(unit_counts)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return (unsigned long long*)p;
}
void units_clear(hipStream_t st) {
  if (unsigned long long* p = unit_counts_ptr()) fill_u64(st, (uint64_t*)p, 0, UNIT_KINDS);
}
void units_read(hipStream_t st, uint64_t* host) {
  unsigned long long* p = unit_counts_ptr();
  if (!p || hipMemcpyAsync(host, p, sizeof(uint64_t) * UNIT_KINDS, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    (void)hipGetLastError();
}
#else
bool units_counted() { return false; }
void units_clear(hipStream_t) {}
void units_read(hipStream_t, uint64_t* host) {
  for (int u = 0; u < UNIT_KINDS; u++) host[u] = 0;
}
#endif

// Job records from the mapped pinned staging into device memory.
__global__ __launch_bounds__(BS) void k_copy_words(const uint64_t* __restrict__ src,
                                                   uint64_t* __restrict__ dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BS)
    dst[i] = src[i];
}

void copy_words(hipStream_t st, const uint64_t* src, uint64_t* dst, uint64_t n) {
  if (n == 0) return;
  const uint64_t b = (n + BS - 1) / BS;
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)(b > 64 ? 64 : b)), dim3(BS), 0, st, src, dst, n);
}

__global__ __launch_bounds__(BS) void k_gather_recs(const uint8_t* __restrict__ base, RecGather g,
                                                    uint64_t* __restrict__ dst) {
  for (int r = blockIdx.x; r < g.n; r += gridDim.x) {
    const uint64_t* src = (const uint64_t*)(base + g.off[r]);
    for (uint32_t w = threadIdx.x; w < g.words; w += BS) dst[(uint64_t)r * g.words + w] = src[w];
  }
}

void gather_recs(hipStream_t st, const uint8_t* base, const RecGather& g, uint64_t* dst) {
  if (g.n <= 0) return;
  hipLaunchKernelGGL(k_gather_recs, dim3((unsigned)g.n), dim3(BS), 0, st, base, g, dst);
}

// Reported tuples of a batch's jobs, back to back, for one copy to the host.
__global__ __launch_bounds__(BS) void k_pack_results(const PackJob* __restrict__ jobs,
                                                     int32_t* __restrict__ out) {
  const PackJob J = jobs[blockIdx.x];
  for (uint64_t w = threadIdx.x; w < J.words; w += BS) out[J.dst + w] = J.src[w];
}

void pack_results(hipStream_t st, const PackJob* jobs, int njobs, int32_t* out) {
  if (njobs > 0) hipLaunchKernelGGL(k_pack_results, dim3(njobs), dim3(BS), 0, st, jobs, out);
}

// k == 1: every member of C(root) is a match; the window is over list indices.
__global__ __launch_bounds__(BS) void k_ext_single(DevGraph g, const ExtJob* __restrict__ jobs,
                                                   unsigned long long* bytes) {
  const ExtJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  uint64_t N = ext_sources(J);
  if (J.a_end < N) N = J.a_end;
  const uint64_t I0 = J.a_begin < N ? J.a_begin : N;
  FinalAcc acc{0, 0, 0, 0};
  unsigned long long by = 0;
  int32_t thr[MAXK];
  const bool thr_on = J.thr != nullptr && *J.d_thr_valid != 0;
#pragma unroll
  for (int v = 0; v < MAXK; v++) thr[v] = thr_on && v < J.k ? J.thr[v] : 0;
  bool full = staging_past_cap(J);
  const uint64_t stride = (uint64_t)gridDim.x * BS;
  const uint64_t rounds = (N - I0 + stride - 1) / stride;  // uniform trip count for the ballot
  for (uint64_t r = 0; r < rounds; r++) {
    const uint64_t i = I0 + r * stride + (uint64_t)blockIdx.x * BS + threadIdx.x;
    int32_t h[MAXK], t[MAXK];
    bool want = false;
    if (i < N) {
      const int32_t v = J.src_cols[i];
      by += 4;
#pragma unroll
      for (int j = 0; j < MAXK; j++) h[j] = v;
      want = finalize(g, J, h, t, acc, !J.collect_only, thr_on, thr, by, [&](int) { return v; });
    }
    stage(J, want, t, full);
  }
  if (!J.collect_only) flush_acc(J.counters, acc);
  if (bytes) block_add(bytes, by);
}

void ext_scan(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int grid,
              unsigned long long* bytes) {
  if (bytes) hipLaunchKernelGGL(k_ext_scan<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else hipLaunchKernelGGL(k_ext_scan<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}

// Next-frontier reservation (see front_reserve): one thread per job takes
// its slots from the pool with one atomic add, then the block zeroes the tile
// states of every reserved scan (the scan's look-back reads them before any
// tile writes its own).
__global__ __launch_bounds__(BS) void k_front_reserve(ExtJob* __restrict__ cur, ExtJob* __restrict__ next,
                                                      LeafJob* __restrict__ leaf, int njobs,
                                                      uint8_t* __restrict__ pool, uint64_t pool_bytes,
                                                      unsigned long long* cursor) {
  __shared__ uint64_t* s_ts[MAX_JOBS];
  __shared__ uint64_t s_tw[MAX_JOBS];
  const int x = (int)threadIdx.x;
  uint64_t* ts = nullptr;
  uint64_t tw = 0;
  if (x < njobs && cur[x].active && !cur[x].last) {
    ExtJob& E = cur[x];
    uint64_t T = *E.sc.d_total;  // attempts: the level keeps at most this many
    if (E.front_limit && T > E.front_limit) T = E.front_limit;
    const int w = E.i + 1;  // matched vertices per partial match of the next level
    auto al = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    const uint64_t cb = al(4ull * (uint64_t)w * T), pb = al(8ull * (T + 1)), bb = al(4ull * T + 4),
                   tws = T / SCAN_TILE + 2, tb = al(8ull * tws);
    const uint64_t need = cb + pb + bb + tb;
    const unsigned long long base = atomicAdd(cursor, (unsigned long long)need);
    if (base + need <= pool_bytes) {
      uint8_t* p = pool + base;
      int32_t* cols = (int32_t*)p;
      E.dst_cols = cols;
      E.dst_cap = T;
      ts = (uint64_t*)(p + cb + pb + bb);
      tw = tws;
      if (next && next[x].active && next[x].i == w) {
        ExtJob& N = next[x];
        N.src_cols = cols;
        N.src_stride = T;
        N.src_cap = T;
        N.sc.P = (uint64_t*)(p + cb);
        N.begs = (uint32_t*)(p + cb + pb);
        N.sc.tstate = ts;
      }
      if (leaf && leaf[x].active && leaf[x].i == w) {
        LeafJob& F = leaf[x];
        F.src_cols = cols;
        F.src_stride = T;
        F.src_cap = T;
      }
    } else {
      // no slots: this level's kept matches flag an overflow and the next
      // level (or leaf count) has no sources -- also when a replayed graph
      // finds the records as an earlier replay left them
      E.dst_cols = nullptr;
      E.dst_cap = 0;
      if (next && next[x].active && next[x].i == w) {
        next[x].src_cap = 0;
        next[x].sc.P = next[x].home_P;
      }
      if (leaf && leaf[x].active && leaf[x].i == w) leaf[x].src_cap = 0;
    }
  }
  if (x < MAX_JOBS) {
    s_ts[x] = ts;
    s_tw[x] = tw;
  }
  __syncthreads();
  for (int j = 0; j < njobs; j++) {
    uint64_t* t = s_ts[j];
    for (uint64_t q = threadIdx.x; q < s_tw[j]; q += BS) t[q] = 0;
  }
}

void front_reserve(hipStream_t st, ExtJob* cur, ExtJob* next, LeafJob* leaf, int njobs,
                   uint8_t* pool, uint64_t pool_bytes, unsigned long long* cursor) {
  hipLaunchKernelGGL(k_front_reserve, dim3(1), dim3(BS), 0, st, cur, next, leaf, njobs, pool, pool_bytes,
                     cursor);
}
template <int WAVES>
static void ext_run_w(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int grid,
                      bool last, bool ahead, unsigned long long* bytes) {
  if (last && ahead)
    hipLaunchKernelGGL((k_ext_run<true, true, WAVES>), dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else if (last)
    hipLaunchKernelGGL((k_ext_run<true, false, WAVES>), dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else
    hipLaunchKernelGGL((k_ext_run<false, false, WAVES>), dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}

void ext_run(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int grid, bool last,
             bool ahead, bool occ8, unsigned long long* bytes) {
  if (occ8)
    ext_run_w<8>(st, g, jobs, njobs, grid, last, ahead, bytes);
  else
    ext_run_w<1>(st, g, jobs, njobs, grid, last, ahead, bytes);
}
void ext_single(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int gx,
                unsigned long long* bytes) {
  hipLaunchKernelGGL(k_ext_single, dim3(gx, njobs), dim3(BS), 0, st, g, jobs, bytes);
}

// ---------------------------------------------------------------------------
// leaf postponement (count-only): completions by leaves counted, not enumerated
// ---------------------------------------------------------------------------

// A literal whose variables are all one leaf, evaluated at vertex x.
__device__ __forceinline__ bool leaf_literal(const DevGraph& g, const DevLit& l, int32_t x) {
  const int32_t a = g.attr[(int64_t)l.attr * g.n + x];
  if (l.kind == 0) return a != ABSENT && a == l.value;
  const int32_t b = g.attr[(int64_t)l.attr2 * g.n + x];
  return a != ABSENT && b != ABSENT && a == b;
}

// Predicate masks of vertex x over the leaf slots: bit j of mx when leaf j's X
// literals hold at x, of mxy when its X and Y literals do.
__device__ __forceinline__ void leaf_masks_of(const DevGraph& g, const LeafJob& J,
                                              const int32_t* lit_leaf, int r, int32_t x,
                                              uint32_t& mx, uint32_t& mxy) {
  const uint32_t all = (1u << r) - 1;
  uint32_t failx = 0, faily = 0;
  for (int t = 0; t < J.nx + J.ny; t++) {
    const int j = lit_leaf[t];
    if (j < 0) continue;
    if (!leaf_literal(g, J.lit[t], x)) {
      if (t < J.nx) failx |= 1u << j;
      else faily |= 1u << j;
    }
  }
  mx = all & ~failx;
  mxy = all & ~(failx | faily);
}

__device__ __forceinline__ void leaf_masks(const DevGraph& g, const LeafJob& J, int32_t x,
                                           uint32_t& mx, uint32_t& mxy) {
  leaf_masks_of(g, J, J.lit_leaf, J.r, x, mx, mxy);
}

// Whether x is in the leaf list of parent image vp: the list holds the
// candidates x != vp for which the tree edge and its reverse constraint hold.
__device__ __forceinline__ bool in_leaf_list(const DevGraph& g, const CandSet& u, int32_t dir,
                                             int32_t prim, int32_t other, int32_t x, int32_t vp,
                                             unsigned long long& by) {
  if (x == vp || !member(u, x)) return false;
  return dir ? (constraint_ok(edge_label_at(g, x, vp, false, by), prim) &&
                pair_ok(g, vp, x, true, other, by))
             : (constraint_ok(edge_label_at(g, vp, x, true, by), prim) &&
                pair_ok(g, x, vp, false, other, by));
}

// One thread per member c of C(p): cnt[c][f][B] = members of c's leaf list
// whose family-f masks contain B (f = 0: every member, 1: X, 2: X and Y).
__device__ __forceinline__ uint64_t leaf_members(const LeafJob& J) {
  return !J.active ? 0ull : (*J.d_np < J.cap_p ? *J.d_np : J.cap_p);
}

// The members of every job's C(p) share one space of BS-member chunks (one
// job per chunk).  With no literal on the leaves a member's counts are its
// list's length and the list is not read.  Otherwise the lists of a chunk's
// members are walked by the whole block: their entries form one index space
// (a block scan of the lengths), so a hub's long list does not hold up its
// wave, and each entry adds to its member's counts in LDS.
__global__ __launch_bounds__(BS) void k_leaf_prep(DevGraph g, const LeafJob* __restrict__ jobs,
                                                  int njobs) {
  __shared__ ChunkMap cm;
  __shared__ uint64_t s_pre[BS];
  __shared__ uint32_t s_beg[BS];
  __shared__ uint32_t s_cx[LEAF_SUBSETS][BS], s_cxy[LEAF_SUBSETS][BS];
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t { return (leaf_members(jobs[j]) + BS - 1) / BS; });
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
    const int jb = chunk_job(cm, njobs, ch);
    const LeafJob& J = jobs[jb];
    const uint64_t np = leaf_members(J);
    const uint32_t nsub = 1u << J.r;
    const uint64_t c = (ch - cm.cs[jb]) * BS + threadIdx.x;
    const bool act = c < np;
    const uint32_t b = act ? J.cpi_beg[c] : 0u, len = act ? J.cpi_len[c] : 0u;
    bool leaf_lits = false;  // the same for the whole block
    for (int t = 0; t < J.nx + J.ny; t++) leaf_lits |= J.lit_leaf[t] >= 0;
    if (leaf_lits) {
      uint64_t total;
      const uint64_t pre = block_excl_scan64(len, total);
      s_pre[threadIdx.x] = pre;
      s_beg[threadIdx.x] = b;
#pragma unroll
      for (int B = 0; B < LEAF_SUBSETS; B++) s_cx[B][threadIdx.x] = s_cxy[B][threadIdx.x] = 0u;
      __syncthreads();
      for (uint64_t it = threadIdx.x; it < total; it += BS) {
        // the member whose entries hold `it`: the last t with s_pre[t] <= it
        int lo = 0, hi = BS - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= it) lo = mid;
          else hi = mid - 1;
        }
        uint32_t mx, mxy;
        leaf_masks(g, J, J.cpi_ent[(uint64_t)s_beg[lo] + (it - s_pre[lo])], mx, mxy);
        for (uint32_t B = 1; B < nsub; B++) {
          if ((mx & B) == B) atomicAdd(&s_cx[B][lo], 1u);
          if ((mxy & B) == B) atomicAdd(&s_cxy[B][lo], 1u);
        }
      }
      __syncthreads();
    }
    if (act) {
      uint32_t* out = J.cnt + c * LEAF_WORDS;
#pragma unroll
      for (uint32_t B = 0; B < LEAF_SUBSETS; B++) {
        const bool used = B > 0 && B < nsub;
        out[B] = B ? len : 0u;
        out[LEAF_SUBSETS + B] = used ? (leaf_lits ? s_cx[B][threadIdx.x] : len) : 0u;
        out[2 * LEAF_SUBSETS + B] = used ? (leaf_lits ? s_cxy[B][threadIdx.x] : len) : 0u;
      }
    }
    if (leaf_lits) __syncthreads();  // the next chunk rewrites the shared arrays
  }
}

// A leaf count as a counter increment; out of range sets `ovf`.
__device__ __forceinline__ unsigned long long leaf_add(__int128 x, bool& ovf) {
  if (x < 0 || x > (__int128)LEAF_COUNT_MAX) {
    ovf = true;
    return 0ull;
  }
  return (unsigned long long)x;
}

// flush_acc for counts that may be large: an add whose result would pass
// 2^63 (judged from the value before it) sets the job's overflow flag.
__device__ __forceinline__ void flush_acc_checked(unsigned long long* counters, FinalAcc acc,
                                                  uint32_t* flags, bool ovf) {
  __shared__ unsigned long long s_acc2[2][BS / WAVE];
  __shared__ uint32_t s_ovf;
  acc.match = wave_sum(acc.match);
  acc.viol = wave_sum(acc.viol);
  const uint32_t wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x == 0) s_ovf = 0;
  __syncthreads();
  if (ovf) s_ovf = 1;
  if (lane() == 0) {
    s_acc2[0][wv] = acc.match;
    s_acc2[1][wv] = acc.viol;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long s = 0;
    for (int w = 0; w < BS / WAVE; w++) s += s_acc2[threadIdx.x][w];
    bool bad = s_ovf != 0;
    if (s) {
      const unsigned long long old = atomicAdd(&counters[threadIdx.x], s);
      bad |= old + s < old || ((old + s) >> 63) != 0;
    }
    if (bad) atomicOr(flags, FLAG_COUNTER_OVERFLOW);
  }
}

__device__ __forceinline__ uint64_t leaf_sources(const LeafJob& J) {
  return !J.active ? 0ull : (*J.d_nsrc < J.src_cap ? *J.d_nsrc : J.src_cap);
}

// Split leaves, one chunk of partial matches [s0, s1) of job J (the whole
// block, uniformly).  A partial match h with parent images vb (last leaf)
// and va (the leaf before it) completes to the pairs (a, b) of list members,
// both off h and distinct, so per literal family f the count is
// |A_f| |B_f| less the vertices in both lists that meet both leaves'
// family-f literals.  The shorter list of each match is walked by the whole
// block: its entries across all the round's matches form one index space
// (a block scan of the lengths), so a long list does not hold up the others.
__device__ void leaf_split_chunk(const DevGraph& g, const LeafJob& J, uint64_t s0, uint64_t s1,
                                 FinalAcc& acc, bool& ovf, unsigned long long& by) {
  __shared__ uint64_t s_pre[BS], s_beg[BS];
  __shared__ int32_t s_h[MAXK][BS];
  __shared__ int32_t s_vo[BS];      // the other list's parent image
  __shared__ uint32_t s_walk_a[BS];  // 1: A's list is walked, B's tested
  __shared__ uint32_t s_both[LEAF_FAMILIES][BS];
  for (uint64_t base = s0; base < s1; base += BS) {
    const uint64_t s = base + threadIdx.x;
    const bool act = s < s1;
    int32_t h[MAXK];
#pragma unroll
    for (int j = 0; j < MAXK; j++)
      h[j] = act && j < J.i ? J.src_cols[(uint64_t)j * J.src_stride + s] : -1;
    int64_t ca[LEAF_FAMILIES] = {}, cb[LEAF_FAMILIES] = {};
    bool X = true, Y = !J.y_false, walk_a = false;
    uint64_t len = 0, beg = 0;
    int32_t vo = -1;
    if (act) {
      const int32_t vb = pick(h, J.par_pos), va = pick(h, J.par2_pos);
      const uint32_t rowb = (uint32_t)J.par_posmap[pos_index(g, J.par_by_bucket, vb)];
      const uint32_t rowa = (uint32_t)J.par2_posmap[pos_index(g, J.par2_by_bucket, va)];
      const uint32_t* tb = J.cnt + (uint64_t)rowb * LEAF_WORDS;
      const uint32_t* ta = J.cnt2 + (uint64_t)rowa * LEAF_WORDS;
      // the partial match, both parents' positions and table rows
      by += 4ull * (uint64_t)J.i + 8 + 8ull * LEAF_WORDS;
#pragma unroll
      for (int f = 0; f < LEAF_FAMILIES; f++) {
        ca[f] = ta[f * LEAF_SUBSETS + 1];
        cb[f] = tb[f * LEAF_SUBSETS + 1];
      }
      // matched inner vertices in either list are not available
      for (int j = 0; j < J.i; j++) {
        const int32_t x = pick(h, j);
        uint32_t mx, mxy;
        if (in_leaf_list(g, J.u, J.dir, J.prim, J.other, x, vb, by)) {
          leaf_masks_of(g, J, J.lit_leaf, 1, x, mx, mxy);
          cb[0] -= 1;
          cb[1] -= mx & 1u;
          cb[2] -= mxy & 1u;
        }
        if (in_leaf_list(g, J.u2, J.dir2, J.prim2, J.other2, x, va, by)) {
          leaf_masks_of(g, J, J.lit_leaf2, 1, x, mx, mxy);
          ca[0] -= 1;
          ca[1] -= mx & 1u;
          ca[2] -= mxy & 1u;
        }
      }
      for (int t = 0; t < J.nx + J.ny; t++) {
        if (J.lit_leaf[t] >= 0 || J.lit_leaf2[t] >= 0) continue;
        const bool v = literal_holds(g, J.lit[t], [&](int p) { return pick(h, p); });
        by += J.lit[t].kind == 0 ? 4 : 8;
        if (t < J.nx) X = X && v;
        else Y = Y && v;
      }
      if (J.split_overlap) {  // else no vertex is in both lists
        const uint32_t la = J.cpi2_len[rowa], lb = J.cpi_len[rowb];
        by += 16;  // both lists' bounds
        walk_a = la <= lb;
        beg = walk_a ? J.cpi2_beg[rowa] : J.cpi_beg[rowb];
        len = walk_a ? la : lb;
        vo = walk_a ? vb : va;
      }
    }
    uint64_t total;
    const uint64_t pre = block_excl_scan64(len, total);
    s_pre[threadIdx.x] = pre;
    s_beg[threadIdx.x] = beg;
#pragma unroll
    for (int j = 0; j < MAXK; j++) s_h[j][threadIdx.x] = h[j];
    s_vo[threadIdx.x] = vo;
    s_walk_a[threadIdx.x] = walk_a ? 1u : 0u;
#pragma unroll
    for (int f = 0; f < LEAF_FAMILIES; f++) s_both[f][threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t it = threadIdx.x; it < total; it += BS) {
      // the match whose entries hold `it`: the last t with s_pre[t] <= it
      // (a match with an empty list shares its prefix with the next one)
      int lo = 0, hi = BS - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= it) lo = mid;
        else hi = mid - 1;
      }
      const int t = lo;
      const int32_t x = J.cpi_ent[s_beg[t] + (it - s_pre[t])];
      by += 4;
      bool inner = false;
#pragma unroll
      for (int j = 0; j < MAXK; j++) inner |= j < J.i && s_h[j][t] == x;
      if (inner) continue;
      const bool wa = s_walk_a[t] != 0;
      const bool in_other = wa ? in_leaf_list(g, J.u, J.dir, J.prim, J.other, x, s_vo[t], by)
                               : in_leaf_list(g, J.u2, J.dir2, J.prim2, J.other2, x, s_vo[t], by);
      if (!in_other) continue;
      uint32_t ma, mya, mb, myb;
      leaf_masks_of(g, J, J.lit_leaf2, 1, x, ma, mya);
      leaf_masks_of(g, J, J.lit_leaf, 1, x, mb, myb);
      atomicAdd(&s_both[0][t], 1u);
      if (ma & mb & 1u) atomicAdd(&s_both[1][t], 1u);
      if (mya & myb & 1u) atomicAdd(&s_both[2][t], 1u);
    }
    __syncthreads();
    if (act) {
      __int128 inj[LEAF_FAMILIES];
#pragma unroll
      for (int f = 0; f < LEAF_FAMILIES; f++)
        inj[f] = (__int128)ca[f] * cb[f] - (__int128)s_both[f][threadIdx.x];
      acc.match += leaf_add(inj[0], ovf);
      if (X) acc.viol += leaf_add(Y ? inj[1] - inj[2] : inj[1], ovf);
    }
    __syncthreads();  // the next round rewrites the shared arrays
  }
}

// The partial matches of every job share one chunk space (LBS_CHUNK sources a
// chunk), so a job with most of the work gets most of the chip.
// SPLIT selects the jobs of one form (split leaves or not): the two forms are
// separate kernels so the common one keeps its register budget.
template <bool SPLIT>
__global__ __launch_bounds__(BS) void k_leaf_count(DevGraph g, const LeafJob* __restrict__ jobs,
                                                   int njobs, unsigned long long* bytes) {
  __shared__ ChunkMap cm;
  chunk_map_build(cm, njobs, [&](int j) -> uint64_t {
    return (jobs[j].split != 0) == SPLIT ? chunks_of(leaf_sources(jobs[j])) : 0ull;
  });
  unsigned long long by = 0;
  for (uint64_t ch = blockIdx.x; ch < cm.cs[njobs]; ch += gridDim.x) {
  const int jb = chunk_job(cm, njobs, ch);
  const LeafJob& J = jobs[jb];
  const uint64_t N = leaf_sources(J);
  const uint64_t s0 = (ch - cm.cs[jb]) * LBS_CHUNK;
  const uint64_t s1 = s0 + LBS_CHUNK < N ? s0 + LBS_CHUNK : N;
  const uint32_t nsub = 1u << J.r;
  FinalAcc acc{0, 0, 0, 0};
  bool ovf = false;
  if (SPLIT) leaf_split_chunk(g, J, s0, s1, acc, ovf, by);
  // window pass: the decided high bits of the variable-0 vertex
  const int whs = J.wshift + J.wbits;
  const uint32_t wpre = J.whist && whs < 32 ? *J.wprefix >> whs : 0u;
  for (uint64_t s = s0 + threadIdx.x; s < s1 && !SPLIT; s += BS) {
    if (J.whist && whs < 32 &&
        ((uint32_t)J.src_cols[(uint64_t)J.wkey_pos * J.src_stride + s] >> whs) != wpre)
      continue;  // outside the decided prefix
    // the partial match, its parent's row in the count table and the words read
    by += 4ull * (uint64_t)J.i + 4 + 4ull * LEAF_WORDS;
    int32_t h[MAXK];
#pragma unroll
    for (int j = 0; j < MAXK; j++) h[j] = j < J.i ? J.src_cols[(uint64_t)j * J.src_stride + s] : 0;
    const int32_t vp = pick(h, J.par_pos);
    const uint32_t rowp = (uint32_t)J.par_posmap[pos_index(g, J.par_by_bucket, vp)];
    const uint32_t* cc = J.cnt + (uint64_t)rowp * LEAF_WORDS;
    int64_t c[LEAF_FAMILIES][LEAF_SUBSETS];
#pragma unroll
    for (int f = 0; f < LEAF_FAMILIES; f++)
#pragma unroll
      for (int B = 0; B < LEAF_SUBSETS; B++) c[f][B] = cc[f * LEAF_SUBSETS + B];
    // matched inner vertices that sit in vp's leaf list are not available
    for (int j = 0; j < J.i; j++) {
      const int32_t x = h[j];
      if (!in_leaf_list(g, J.u, J.dir, J.prim, J.other, x, vp, by)) continue;
      uint32_t mx, mxy;
      leaf_masks(g, J, x, mx, mxy);
#pragma unroll
      for (uint32_t B = 1; B < LEAF_SUBSETS; B++) {
        if (B >= nsub) continue;
        c[0][B] -= 1;
        if ((mx & B) == B) c[1][B] -= 1;
        if ((mxy & B) == B) c[2][B] -= 1;
      }
    }
    bool X = true, Y = !J.y_false;
    for (int t = 0; t < J.nx + J.ny; t++) {
      if (J.lit_leaf[t] >= 0) continue;
      const bool v = literal_holds(g, J.lit[t], [&](int p) { return pick(h, p); });
      by += J.lit[t].kind == 0 ? 4 : 8;  // the attribute values read
      if (t < J.nx) X = X && v;
      else Y = Y && v;
    }
    if (J.whist) {  // window pass: this match's violating completions, by digit
      if (X) {
        const __int128 ix = leaf_injective(J.r, c[1]);
        const __int128 v = Y ? ix - leaf_injective(J.r, c[2]) : ix;
        const uint32_t key = (uint32_t)pick(h, J.wkey_pos);
        if (v > 0 && v <= (__int128)LEAF_COUNT_MAX)
          atomicAdd(&J.whist[(key >> J.wshift) & ((1u << J.wbits) - 1u)], (unsigned long long)v);
      }
      continue;
    }
    acc.match += leaf_add(leaf_injective(J.r, c[0]), ovf);
    if (X) {
      const __int128 ix = leaf_injective(J.r, c[1]);
      acc.viol += leaf_add(Y ? ix - leaf_injective(J.r, c[2]) : ix, ovf);
    }
  }
  // counts only: the fingerprint sums stay zero
  flush_acc_checked(J.counters, acc, J.flags, ovf);
  }
  if (bytes) block_add(bytes, by);
}

void leaf_prep(hipStream_t st, const DevGraph& g, const LeafJob* jobs, int njobs, int grid) {
  hipLaunchKernelGGL(k_leaf_prep, dim3(grid), dim3(BS), 0, st, g, jobs, njobs);
}
// Window select (one block per job).  win_begin clears the histogram and
// starts the rank at K.  A digit step finds the bin holding the remaining
// rank (a block scan of the weighted histogram), records its digit in the
// prefix and clears the bins; a prefix whose group holds fewer violations
// than the rank (only when the job has fewer than K) leaves the window
// unbounded: rank 0 and a prefix of all ones.  The last step writes the
// threshold (d, then all ones, in variable order) and restarts the staging.
__global__ __launch_bounds__(BS) void k_win_begin(const WinJob* __restrict__ jobs) {
  const WinJob& J = jobs[blockIdx.x];
  if (!J.active) return;
  for (int b = threadIdx.x; b < RADIX_BINS; b += BS) J.hist[b] = 0ull;
  if (threadIdx.x == 0) {
    *J.prefix = 0u;
    *J.rank = J.K;
  }
}

__global__ __launch_bounds__(BS) void k_win_digit(const WinJob* __restrict__ jobs, int shift,
                                                  int bits, int last) {
  constexpr int PER = RADIX_BINS / BS;
  const WinJob& J = jobs[blockIdx.x];
  if (!J.active) return;
  const unsigned long long r = *J.rank;  // read before the barriers, written after
  const uint32_t nb = 1u << bits;
  unsigned long long h[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t bin = threadIdx.x * PER + j;
    h[j] = bin < nb ? J.hist[bin] : 0ull;
    sum += h[j];
  }
  uint64_t total;
  const uint64_t pre = block_excl_scan64(sum, total);
  __syncthreads();
  if (r != 0) {
    if (total < r) {
      if (threadIdx.x == 0) {
        *J.prefix = 0xFFFFFFFFu;
        *J.rank = 0ull;
      }
    } else if (pre < r && r <= pre + sum) {  // exactly one thread
      unsigned long long cum = pre;
      uint32_t d = threadIdx.x * PER;
      for (int j = 0; j < PER; j++) {
        if (cum + h[j] >= r) {
          d = threadIdx.x * PER + j;
          break;
        }
        cum += h[j];
      }
      *J.prefix |= d << shift;
      *J.rank = r - cum;
    }
  }
#pragma unroll
  for (int j = 0; j < PER; j++) J.hist[threadIdx.x * PER + j] = 0ull;
  __syncthreads();  // the prefix is final
  if (last && threadIdx.x < (uint32_t)J.k) J.thr[threadIdx.x] = threadIdx.x == 0 ? (int32_t)*J.prefix : -1;
  if (last && threadIdx.x == 0) {
    *J.d_thr_valid = 1u;
    *J.d_vcount = 0ull;
  }
}

void win_begin(hipStream_t st, const WinJob* jobs, int njobs) {
  hipLaunchKernelGGL(k_win_begin, dim3(njobs), dim3(BS), 0, st, jobs);
}
void win_digit(hipStream_t st, const WinJob* jobs, int njobs, int shift, int bits, bool last) {
  hipLaunchKernelGGL(k_win_digit, dim3(njobs), dim3(BS), 0, st, jobs, shift, bits, last ? 1 : 0);
}

void leaf_count(hipStream_t st, const DevGraph& g, const LeafJob* jobs, int njobs, int grid,
                bool split, unsigned long long* bytes) {
  if (split) hipLaunchKernelGGL(k_leaf_count<true>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
  else hipLaunchKernelGGL(k_leaf_count<false>, dim3(grid), dim3(BS), 0, st, g, jobs, njobs, bytes);
}

// ---------------------------------------------------------------------------
// lexicographic first-K of the staged violations
// ---------------------------------------------------------------------------

constexpr int SORT_THREADS = 1024;

// Tuples being sorted in one workgroup sit in LDS as k columns: word w of
// tuple j at s[w * SORT_MAX + j], so the threads of a compare-exchange step,
// which take consecutive j, hit consecutive banks.
__device__ __forceinline__ int cmp_lds(const uint32_t* s, uint32_t x, uint32_t y, int k) {
  for (int w = 0; w < k; w++) {
    const uint32_t a = s[w * SORT_MAX + x], b = s[w * SORT_MAX + y];
    if (a != b) return a < b ? -1 : 1;
  }
  return 0;
}

// Loads n tuples (k words each, row-major) into the columns, padding up to p2
// with all-ones tuples, which order last.
__device__ __forceinline__ void sort_load(uint32_t* s, const int32_t* src, uint32_t n, uint32_t p2,
                                          int k) {
  for (uint32_t q = threadIdx.x; q < p2 * (uint32_t)k; q += blockDim.x) {
    const uint32_t j = q / (uint32_t)k, w = q - j * (uint32_t)k;
    s[w * SORT_MAX + j] = j < n ? (uint32_t)src[q] : 0xFFFFFFFFu;
  }
}

// Writes the first n tuples back row-major.
__device__ __forceinline__ void sort_store(const uint32_t* s, int32_t* dst, uint32_t n, int k) {
  for (uint32_t q = threadIdx.x; q < n * (uint32_t)k; q += blockDim.x) {
    const uint32_t j = q / (uint32_t)k, w = q - j * (uint32_t)k;
    dst[q] = (int32_t)s[w * SORT_MAX + j];
  }
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
        if (c != 0 && (c > 0) == asc) {
          for (int w = 0; w < k; w++) {
            const uint32_t tmp = s[w * SORT_MAX + lo];
            s[w * SORT_MAX + lo] = s[w * SORT_MAX + hi];
            s[w * SORT_MAX + hi] = tmp;
          }
        }
      }
    }
  }
  __syncthreads();
}

// One workgroup per job: sort the staged tuples when there are at most
// SORT_MAX of them and keep the first min(K, count); otherwise flag the job
// for the radix select.
// Algorithmic bytes: the staged tuples read and the first K written.
__global__ __launch_bounds__(SORT_THREADS) void k_topk_small(const TopkJob* __restrict__ jobs,
                                                             unsigned long long* bytes) {
  __shared__ uint32_t s[SORT_MAX * MAXK];
  const TopkJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  const uint64_t cnt = *J.d_vcount < J.vcap ? *J.d_vcount : J.vcap;
  if (cnt > (uint64_t)SORT_MAX) {
    if (threadIdx.x == 0) *J.d_need_select = 1;
    return;
  }
  if (threadIdx.x == 0) *J.d_need_select = 0;
  uint32_t p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  sort_load(s, J.vbuf, (uint32_t)cnt, p2, J.k);
  bitonic_lds(s, p2, J.k);
  const uint64_t out = cnt < (uint64_t)J.K ? cnt : (uint64_t)J.K;
  sort_store(s, J.res, (uint32_t)out, J.k);
  if (bytes && threadIdx.x == 0 && cnt) atomicAdd(bytes, 4ull * (uint64_t)J.k * (cnt + out));
}

void topk_small(hipStream_t st, const TopkJob* jobs, int njobs, unsigned long long* bytes) {
  hipLaunchKernelGGL(k_topk_small, dim3(1, njobs), dim3(SORT_THREADS), 0, st, jobs, bytes);
}

// Radix select, batched over jobs (grid row y = job).  State words of a job:
// [0..MAXK) the tuple being decided, [MAXK] the remaining rank (1-based) among
// staged tuples that agree with it so far, [MAXK + 1] blocks done in the
// current pass, [MAXK + 2] set once a single staged tuple agrees with the
// decided prefix, [MAXK + 3] set once that tuple has been copied whole into
// [0..MAXK): the passes left then have nothing to decide and return at once.
__global__ void k_sel_begin(const SelJob* __restrict__ jobs) {
  const SelJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  if (threadIdx.x < MAXK) J.state[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    J.state[MAXK] = (uint32_t)J.K;
    J.state[MAXK + 1] = 0;
    J.state[MAXK + 2] = 0;
    J.state[MAXK + 3] = 0;
    if (J.d_outcount) *J.d_outcount = 0;
  }
}

__device__ __forceinline__ uint64_t sel_count(const SelJob& J) {
  return *J.d_vcount < J.vcap ? *J.d_vcount : J.vcap;
}

// One digit of the radix select.  Tuples that agree with the decided prefix
// (words < word, and the decided high bits of `word`) vote for the next digit
// of `word`; the last block of a job to add its votes (per-job counter
// state[MAXK + 1]) finds the bin holding the remaining rank with a block-wide
// scan of the histogram, records the digit and clears the histogram and the
// counter for the next pass.  Ordering without a cache-flushing fence: the
// histogram adds are agent-scope atomics whose returned values feed the LDS
// before the barrier, so they have been performed before the block's counter
// add is issued; the last block reads the bins with agent-scope atomic loads
// issued after it has seen the final count.
// Algorithmic bytes (COUNT): the tuple words each pass reads.
template <bool COUNT>
__global__ __launch_bounds__(BS) void k_sel_pass(const SelJob* __restrict__ jobs, int word,
                                                 int shift, int bits, unsigned long long* bytes) {
  constexpr int PER = RADIX_BINS / BS;
  __shared__ uint32_t sh[RADIX_BINS];
  __shared__ uint32_t s_last, s_seen;
  const SelJob& J = jobs[blockIdx.y];
  if (!J.active || word >= J.k || J.state[MAXK + 3]) return;
  // one staged tuple agrees with the prefix: it is the one sought, and the
  // thread that meets it copies it whole instead of voting
  const bool single = J.state[MAXK + 2] != 0;
  for (int b = threadIdx.x; b < RADIX_BINS; b += BS) sh[b] = 0;
  if (threadIdx.x == 0) s_seen = 0;
  uint32_t st[MAXK];
#pragma unroll
  for (int w = 0; w < MAXK; w++) st[w] = J.state[w];
  const uint32_t r = J.state[MAXK];  // read before any block can be the last
  __syncthreads();
  const int k = J.k;
  const uint64_t cnt = sel_count(J);
  const uint32_t hi_mask = (shift + bits >= 32) ? 0u : (0xFFFFFFFFu << (shift + bits));
  const uint32_t want_hi = pick(st, word) & hi_mask;
  unsigned long long by = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * BS) {
    const uint32_t* t = (const uint32_t*)J.vbuf + i * (uint64_t)k;
    bool match = true;
    int w = 0;
    for (; w < word && match; w++) match = t[w] == pick(st, w);
    if (COUNT) by += 4ull * (uint64_t)(w + (match ? 1 : 0));
    if (!match) continue;
    const uint32_t x = t[word];
    if ((x & hi_mask) != want_hi) continue;
    if (single) {
      for (int w = word; w < k; w++) J.state[w] = t[w];
      J.state[MAXK + 3] = 1;
      continue;
    }
    atomicAdd(&sh[(x >> shift) & ((1u << bits) - 1)], 1u);
  }
  if (COUNT) block_add(bytes, by);
  __syncthreads();
  uint32_t seen = 0;
  for (int b = threadIdx.x; b < RADIX_BINS; b += BS)
    if (sh[b])
      seen |= __hip_atomic_fetch_add(&J.hist[b], sh[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicOr(&s_seen, seen);  // waits for the adds' return values
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(&J.state[MAXK + 1], 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  const uint32_t nb = 1u << bits;
  uint32_t h[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t bin = threadIdx.x * PER + j;
    h[j] = bin < nb ? __hip_atomic_load(&J.hist[bin], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : 0u;
    sum += h[j];
  }
  uint32_t total;
  const uint32_t pre = block_excl_scan(sum, total);
  if (pre < r && r <= pre + sum) {  // exactly one thread
    uint32_t cum = pre, d = threadIdx.x * PER, in_bin = 0;
    for (int j = 0; j < PER; j++) {
      if (cum + h[j] >= r) {
        d = threadIdx.x * PER + j;
        in_bin = h[j];
        break;
      }
      cum += h[j];
    }
    J.state[MAXK] = r - cum;
    J.state[word] |= d << shift;
    if (in_bin == 1u) J.state[MAXK + 2] = 1;
  }
#pragma unroll
  for (int j = 0; j < PER; j++) J.hist[threadIdx.x * PER + j] = 0;
  if (threadIdx.x == 0) J.state[MAXK + 1] = 0;
}

// Staged tuples <= the selected one (exactly K of them, tuples being
// distinct) into out.
// (Algorithmic bytes, COUNT: the words compared and the tuples written.)
template <bool COUNT>
__global__ __launch_bounds__(BS) void k_sel_compact(const SelJob* __restrict__ jobs,
                                                    unsigned long long* bytes) {
  const SelJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  const int k = J.k;
  uint32_t st[MAXK];
#pragma unroll
  for (int w = 0; w < MAXK; w++) st[w] = J.state[w];
  const uint64_t cnt = sel_count(J);
  unsigned long long by = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * BS) {
    const uint32_t* t = (const uint32_t*)J.vbuf + i * (uint64_t)k;
    int c = 0, w = 0;
    for (; w < k && c == 0; w++) {
      const uint32_t y = pick(st, w);
      c = t[w] < y ? -1 : (t[w] > y ? 1 : 0);
    }
    if (COUNT) by += 4ull * (uint64_t)w;
    if (c <= 0) {
      const unsigned long long slot = atomicAdd(J.d_outcount, 1ull);
      if (slot < (unsigned long long)J.K) {
        for (int q = 0; q < k; q++) J.out[slot * k + q] = (int32_t)t[q];
        if (COUNT) by += 4ull * (uint64_t)(2 * k - w);  // the rest read, all of it written
      }
    }
  }
  if (COUNT) block_add(bytes, by);
}

// Sorts the K selected tuples of every job in place.
__global__ __launch_bounds__(SORT_THREADS) void k_sel_sort(const SelJob* __restrict__ jobs,
                                                           unsigned long long* bytes) {
  __shared__ uint32_t s[SORT_MAX * MAXK];
  const SelJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  const uint64_t n = *J.d_outcount < (uint64_t)J.K ? *J.d_outcount : (uint64_t)J.K;
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  sort_load(s, J.out, (uint32_t)n, p2, J.k);
  bitonic_lds(s, p2, J.k);  // every tuple is in LDS before any is written back
  sort_store(s, J.out, (uint32_t)n, J.k);
  if (bytes && threadIdx.x == 0 && n) atomicAdd(bytes, 8ull * (uint64_t)J.k * n);  // read, written
}

// The selected tuple becomes the job's staging threshold; staging restarts.
__global__ void k_sel_thr(const SelJob* __restrict__ jobs) {
  const SelJob& J = jobs[blockIdx.y];
  if (!J.active) return;
  if (threadIdx.x < (uint32_t)J.k) J.thr[threadIdx.x] = (int32_t)J.state[threadIdx.x];
  if (threadIdx.x == 0) {
    *J.d_thr_valid = 1;
    *J.d_vcount = 0;
  }
}

void sel_begin(hipStream_t st, const SelJob* jobs, int njobs) {
  hipLaunchKernelGGL(k_sel_begin, dim3(1, njobs), dim3(64), 0, st, jobs);
}
void sel_pass(hipStream_t st, const SelJob* jobs, int njobs, int word, int shift, int bits,
              int gx, unsigned long long* bytes) {
  if (bytes)
    hipLaunchKernelGGL(k_sel_pass<true>, dim3(gx, njobs), dim3(BS), 0, st, jobs, word, shift, bits, bytes);
  else
    hipLaunchKernelGGL(k_sel_pass<false>, dim3(gx, njobs), dim3(BS), 0, st, jobs, word, shift, bits, bytes);
}
void sel_first_k(hipStream_t st, const SelJob* jobs, int njobs, int gx, unsigned long long* bytes) {
  if (bytes) hipLaunchKernelGGL(k_sel_compact<true>, dim3(gx, njobs), dim3(BS), 0, st, jobs, bytes);
  else hipLaunchKernelGGL(k_sel_compact<false>, dim3(gx, njobs), dim3(BS), 0, st, jobs, bytes);
  hipLaunchKernelGGL(k_sel_sort, dim3(1, njobs), dim3(SORT_THREADS), 0, st, jobs, bytes);
}
void sel_threshold(hipStream_t st, const SelJob* jobs, int njobs) {
  hipLaunchKernelGGL(k_sel_thr, dim3(1, njobs), dim3(64), 0, st, jobs);
}

}  // namespace gfd
