// Internal declarations shared by the host driver (gfd_api.hip) and the
// kernels (gfd_kernels.hip).  Not part of the public ABI.
//
// Every kernel works on a batch of independent jobs (one per GFD): the grid is
// (x tiles, jobs); block row y reads its job's parameters from a device array.
// Within a job, work is spread evenly over the x blocks by a prefix over the
// job's items and a load-balanced search, so power-law hubs do not serialise.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfd {

constexpr int MAXK = 8;
constexpr int MAXLIT = 8;
constexpr int MAXCONS = 2 * (MAXK - 1);  // pull constraints on one pattern vertex
constexpr int32_t ABSENT = -1;
constexpr int32_t ANY = -1;
constexpr int32_t NOEDGE = -2;

// Constraint on one direction of one vertex pair, checked by a probe:
//   >= 0       a data edge with exactly this label must exist
//   ANY        a data edge with any label must exist
//   PC_ABSENT  no data edge may exist (induced reading, no pattern edge)
//   PC_FREE    no constraint (non-induced reading, no pattern edge)
constexpr int32_t PC_ABSENT = -2;
constexpr int32_t PC_FREE = -3;

constexpr int BS = 256;        // threads per block everywhere
constexpr int WAVE = 64;       // CDNA wavefront
constexpr int SCAN_IPT = 8;    // items per thread in the scan
constexpr int SCAN_TILE = BS * SCAN_IPT;
constexpr int MAX_JOBS = 256;  // jobs per launch (one batch); at most BS
constexpr int LBS_ROUNDS = 8;  // flat work: rounds of BS positions per located chunk
constexpr uint64_t LBS_CHUNK = (uint64_t)BS * LBS_ROUNDS;
constexpr size_t LABEL_TRIPLES_MAX = size_t(1) << 24;  // keys of the label-triple blocks
constexpr int NXCD = 8;        // accelerator dies (XCDs), each with its own L2
constexpr int SORT_MAX = 2048; // violation tuples sorted in one workgroup
constexpr int RADIX_BITS = 11;
constexpr int RADIX_BINS = 1 << RADIX_BITS;

// Device-resident graph (Section II: G = (V, E, L, F_A)).
struct DevGraph {
  int32_t n;
  uint32_t m;
  int32_t num_attrs;
  const uint32_t* out_off;  // [n+1]
  const int32_t* out_nbr;   // [m], each row ascending
  const int32_t* out_lab;   // [m]
  const uint32_t* in_off;   // [n+1]
  const int32_t* in_nbr;    // [m], each row ascending (sources)
  const int32_t* in_lab;    // [m]
  const int32_t* vlab;      // [n]
  const int32_t* attr;      // [num_attrs * n]
  const uint32_t* lab_off;  // [num_vlabels+1]
  const int32_t* lab_vtx;   // [n], vertices grouped by label, ascending ids
  const uint32_t* lab_pos;  // [n], v's position within its label bucket
  // label-ordered view: row p is the row of lab_vtx[p], so one label bucket's
  // rows are one contiguous slice of these arrays
  const uint32_t* lv_out_off;  // [n+1]
  const int32_t* lv_out_nbr;   // [m]
  const int32_t* lv_out_lab;   // [m]
  const uint32_t* lv_in_off;   // [n+1]
  const int32_t* lv_in_nbr;    // [m]
  const int32_t* lv_in_lab;    // [m]
  // edge-label blocks of the label-ordered view, per direction d: block
  // (vertex label L, edge label e) lists the rows of bucket L that have
  // e-labelled edges (row position within the bucket, ascending) and those
  // edges' far ends.  Rows [rb, re) of a block own entries
  // [elb_start[d][rb], elb_start[d][re]) of elb_nbr[d].
  const uint32_t* elb_row[2];    // [rows_d] bucket position of the row
  const uint32_t* elb_start[2];  // [rows_d + 1]
  const int32_t* elb_nbr[2];     // [m]
  // the same keyed by (vertex label, edge label, far end's label), when built
  const uint32_t* elt_row[2];
  const uint32_t* elt_start[2];
  const int32_t* elt_nbr[2];
  // combined rows: row v is the ascending union of v's out- and in-neighbours
  // w, with sym_lab = (label of v -> w, label of w -> v), NOEDGE where absent
  const uint64_t* sym_off;  // [n+1]
  const int32_t* sym_nbr;   // [sym_off[n]]
  const int2* sym_lab;      // [sym_off[n]]
  // neighbour sets of rows with at least HUB_MIN combined entries: an
  // open-addressing table of one-byte fingerprints hub_fp(w) of the row's
  // neighbours w, [hub_off[v], hub_off[v+1]) (empty when the row is
  // shorter), a power of two at least twice the row's length, 0 in free
  // slots, linear probing from hub_slot(w, size).  A free slot reached before
  // w's fingerprint proves w absent; a matching fingerprint is confirmed in
  // the row.  One byte a slot keeps the tables of the 4M/20M graph at 87 MB,
  // a quarter of what the neighbour ids would take.
  const uint64_t* hub_off;  // [n+1]
  const uint8_t* hub_tab;   // [hub_off[n]]
};

constexpr uint64_t HUB_MIN = 8;
__host__ __device__ __forceinline__ uint64_t hub_slot(int32_t w, uint64_t size) {
  // multiplicative hash, scaled to [0, size) by its high bits
  return ((uint64_t)((uint32_t)w * 0x9E3779B1u) * size) >> 32;
}
// fingerprint in 1..255, from a second multiplicative hash (its top bits are
// independent of the slot's)
__host__ __device__ __forceinline__ uint8_t hub_fp(int32_t w) {
  return (uint8_t)(1u + (((uint32_t)w * 0x85EBCA77u) >> 24) % 255u);
}

// A candidate set C(u): its members (list, *cnt), their positions in the list
// (meaningful for members only) and an n-bit membership bitmap, small enough
// to stay in L2 (512 KB for 4M vertices).  The positions of a labelled u are
// indexed by the member's position in u's label bucket (lab_pos), so they take
// the bucket's size rather than n; a wildcard u's are indexed by vertex id.
struct CandSet {
  const int32_t* list;
  const uint64_t* cnt;
  const int32_t* pos;    // [bucket size] (by_bucket) or [n]
  const uint32_t* bits;  // [ceil(n/32)]
  int32_t by_bucket;
};

// Index of member x's entry in a position map.
__device__ __forceinline__ uint32_t pos_index(const DevGraph& g, int32_t by_bucket, int32_t x) {
  return by_bucket ? g.lab_pos[x] : (uint32_t)x;
}

// Prefix over one job's items, computed by a single-pass scan with a
// decoupled look-back (per-job tile states and ticket).
struct JobScan {
  uint64_t* P;         // exclusive prefix [items+1]
  uint64_t* d_total;
  uint64_t* tstate;    // [tiles]
  uint32_t* ticket;    // zero at rest
  uint32_t* err;
  uint32_t epoch;
};

// Pull constraint: v passes when some x adjacent to v (out-row if dir == 0,
// in-row if dir == 1) through an edge of label elab (ANY = any) is in C(w).
struct PullC {
  int32_t dir, elab;
  CandSet w;
  // a labelled vertex and edge: the edge-label block's rows [rb, re) (direct
  // jobs stream them; listed items find their own row among them); blk 1 the
  // (vertex label, edge label) blocks, 2 those keyed by the far end's label
  // too, 0 none
  uint32_t rb, re;
  int32_t blk;
  int32_t nlab;  // label of the constraining pattern vertex (ANY: wildcard)
};

// Candidate filter of one pattern vertex u (Section IV-B: label candidates,
// degree filter, and the BFS candidate-subgraph / dead-end conditions).
struct FilterJob {
  int32_t active;
  int32_t ncons;
  int32_t min_out, min_in;
  const int32_t* list;   // items: nullptr = identity 0..n_host-1
  const uint64_t* d_n;   // device item count (nullptr: n_host)
  uint64_t n_host, cap;  // cap bounds the item count
  // direct: the items are the consecutive rows base .. base+n_host-1 of the
  // label-ordered view (list = lab_vtx + base), or of the plain CSR when list
  // is nullptr; their adjacency is then one contiguous slice and needs no scan
  int32_t direct;
  uint32_t base;
  const uint32_t* keep;  // if set, only members of this bitmap may be kept
  PullC cons[MAXCONS];
  // constraint hits, zero at rest (the compaction clears every non-zero word
  // it reads).  hitmode 1: one bitmap per constraint over the item indices,
  // bit i of hits[c * hit_words + i / 32] set when item i meets constraint c
  // (compact, set by atomics: for sparse hits); hitmode 0: one byte per
  // constraint and item, byte c * 32 * hit_words + i of hits set to 1 by a
  // plain store (no atomics, no line fetch: for dense hits).
  uint32_t* hits;
  uint64_t hit_words;
  int32_t hitmode;
  JobScan sc;            // over (constraint, item) pairs
  int32_t* out;          // the new C(u): list, count (atomic cursor), positions, bits
  uint64_t out_cap;      // the list's capacity (a bound on |C(u)|; passing it is an error)
  uint64_t* d_out_n;
  int32_t* pos;
  int32_t pos_by_bucket; // positions indexed by bucket position (CandSet::by_bucket)
  uint32_t* bits;        // cleared by filter_clear before the compaction
  uint64_t nwords;
};

// CPI adjacency for spanning-tree edge (p, u): for each v_p in C(p) the
// neighbours v (row direction dir) in C(u) through an edge of label prim whose
// reverse direction satisfies `other`.  The list of the i-th member of C(p) is
// arena[beg[i] .. beg[i] + len[i]).
struct CpiJob {
  int32_t active;
  int32_t dir, prim, other;
  CandSet p, u;
  uint64_t cap_p;
  uint32_t* beg;
  uint32_t* len;
  uint32_t* cur;         // two-pass fill: entries written per member
  int32_t* arena;
  unsigned long long* arena_cursor;
  uint64_t arena_cap;
  uint32_t* flags;       // bit 2: arena overflow
  uint64_t* d_base;      // one pass: the job's region of the arena (~0: out of arena)
  uint64_t* d_asked;     // one pass: the job's entries asked, summed over its tree edges
  JobScan sc;            // over rows of C(p)
  // labelled p and prim: the edge-label block (p's bucket, prim) of direction
  // dir is rows [rb, re); bucket base position `base`
  int32_t blk;
  uint32_t rb, re, base;
};

struct DevLit {
  int32_t kind;  // 0 const, 1 var
  int32_t pos, attr, pos2, attr2, value;  // pos/pos2: matching-order positions
};

// One enumeration level of one job: extend partial matches of i vertices by
// the vertex at matching-order position i (Section IV-B, matching over the
// CPI); the last level evaluates X -> Y on every match (Section II).
struct ExtJob {
  int32_t active, i, last, k;
  const int32_t* src_cols;  // column j (j < i) at src_cols + j * src_stride
  uint64_t src_stride;
  const uint64_t* d_nsrc;
  uint64_t src_cap;
  int32_t par_pos;          // position of the spanning-tree parent
  const int32_t* par_posmap;  // C(parent) positions
  int32_t par_by_bucket;      // ... indexed by bucket position
  const uint32_t* cpi_beg;
  const uint32_t* cpi_len;
  const int32_t* cpi_ent;
  // the vertex of this level roots a further component of the pattern: every
  // source's list is all of its candidate set (cpi_ent = that list, of
  // min(*cross_n, cross_cap) members) instead of a CPI list
  int32_t cross;
  const uint64_t* cross_n;
  uint64_t cross_cap;
  uint32_t* begs;           // [src_cap] list start per source
  JobScan sc;               // over sources
  // inner levels of the fast path: the next frontier is reserved from the
  // batch's frontier pool once this level's attempts are counted (at most
  // front_limit slots when nonzero), and dst_* / the next level's src_*,
  // begs and scan arrays are pointed at it on the device
  uint64_t a_begin, a_end;  // attempt window
  int32_t nchk;
  int32_t chk_pos[MAXK];
  int32_t chk_fwd[MAXK];    // constraint on data edge h(x_pos) -> v
  int32_t chk_bwd[MAXK];    // constraint on data edge v -> h(x_pos)
  uint64_t front_limit;
  uint64_t* home_P;         // the job's own prefix array: a level whose frontier
                            // could not be reserved scans no sources into it
  int32_t* dst_cols;
  uint64_t dst_cap;
  uint64_t* d_ndst;
  uint32_t* flags;          // bit0: frontier overflow (a staging overflow shows as
                            // *d_vcount > vcap)
  int32_t var_pos[MAXK];
  int32_t nx, ny, y_false, collect_only;
  int32_t thr_incl;         // stage t <= thr instead of t < thr
  int32_t prune;            // scan: sources whose bound variables already order
                            // them past thr get no attempts (collect-only passes)
  DevLit lit[2 * MAXLIT];
  unsigned long long* counters;  // [4] match, violation, match_fp, violation_fp
  int32_t* vbuf;
  uint64_t* d_vcount;
  uint64_t vcap;
  const int32_t* thr;
  const uint32_t* d_thr_valid;
  // the last level of a count-only job whose last leaf is counted: its
  // record is laid out (the frontier reservation points it at its sources)
  // but the main pass skips it; it runs later only over the window of
  // sources that can hold the first K violations
  int32_t deferred;
};

// Leaf postponement (count-only calls): the last r (<= MAX_LEAVES) vertices
// of the matching order are structurally identical leaves under one parent p,
// each carrying only literals on itself.  Their injective completions of a
// partial match are counted, not enumerated, from per-list counts of the
// members meeting each subset of leaf predicates.
constexpr int MAX_LEAVES = 3;
constexpr int LEAF_SUBSETS = 1 << MAX_LEAVES;  // masks 1 .. 2^r - 1 are used
constexpr int LEAF_FAMILIES = 3;               // no literal, X, X and Y
constexpr int LEAF_WORDS = LEAF_FAMILIES * LEAF_SUBSETS;
// Injective assignments of r leaves to sets A_0 .. A_{r-1}, from c[B] =
// |intersection of A_j, j in B| (bit j of B: leaf j): the sum over set
// partitions of the leaves of the product over blocks of
// (-1)^(|B|-1) (|B|-1)! c[B] (Moebius inversion on the partition lattice).
// Exact in 128 bits for counts below 2^32.
__host__ __device__ inline __int128 leaf_injective(int r, const int64_t (&c)[LEAF_SUBSETS]) {
  const __int128 c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5], c6 = c[6], c7 = c[7];
  if (r == 1) return c1;
  if (r == 2) return c1 * c2 - c3;
  return c1 * c2 * c4 - c3 * c4 - c5 * c2 - c6 * c1 + 2 * c7;
}
// Largest per-partial-match leaf count added to a 64-bit counter: a thread
// adds at most LBS_ROUNDS of them per chunk and a block 256 threads' sums, so
// the block's partial stays below 2^62; a larger count (or a negative one,
// which exact inputs never give) marks the job's counters as overflowed.
constexpr int64_t LEAF_COUNT_MAX = int64_t(1) << 50;
constexpr uint32_t FLAG_COUNTER_OVERFLOW = 8u;  // job flags bit: a counter would pass 2^63

struct LeafJob {
  int32_t active, i, r;       // i: matched vertices in a source; r: leaves
  const int32_t* src_cols;    // column j (j < i) at src_cols + j * src_stride
  uint64_t src_stride;
  const uint64_t* d_nsrc;
  uint64_t src_cap;
  int32_t par_pos;            // the parent's position in a source
  const int32_t* par_posmap;  // C(p) positions
  int32_t par_by_bucket;      // ... indexed by bucket position
  const uint64_t* d_np;       // |C(p)|
  uint64_t cap_p;
  const uint32_t* cpi_beg;    // the leaves' CPI lists (one set: the leaves are identical)
  const uint32_t* cpi_len;
  const int32_t* cpi_ent;
  CandSet u;                  // the leaves' candidate set
  int32_t dir, prim, other;   // the tree edge p - leaf, as in CpiJob
  uint32_t* cnt;              // [cap_p * LEAF_WORDS]
  int32_t nx, ny, y_false;
  DevLit lit[2 * MAXLIT];
  int32_t lit_leaf[2 * MAXLIT];  // leaf slot of a literal, or -1 (inner vertices)
  unsigned long long* counters;  // match, violation
  uint32_t* flags;               // FLAG_COUNTER_OVERFLOW
  // split leaves: this record counts the last leaf (slot 0 of lit_leaf, r = 1);
  // the other leaf, under another parent, has the fields below (its literals
  // in slot 0 of lit_leaf2, its counts in cnt2, filled by a record of its own)
  int32_t split;
  int32_t split_overlap;  // 0: the two leaves' labels differ, their lists share nothing
  int32_t par2_pos;
  const int32_t* par2_posmap;
  int32_t par2_by_bucket;
  const uint32_t* cpi2_beg;
  const uint32_t* cpi2_len;
  CandSet u2;
  int32_t dir2, prim2, other2;
  const uint32_t* cnt2;
  int32_t lit_leaf2[2 * MAXLIT];
  // window pass (whist != nullptr): nothing is counted; each partial match
  // whose variable-0 vertex (at position wkey_pos) agrees with the decided
  // high bits *wprefix above bit wshift + wbits adds its violating
  // completions to whist[bits wshift .. wshift + wbits of that vertex]
  unsigned long long* whist;
  const uint32_t* wprefix;
  int32_t wkey_pos, wshift, wbits;
};

// The first-K window of a job whose last leaf was counted: a radix select over
// the variable-0 vertices of the partial matches, weighted by their violating
// completions, finds the variable-0 vertex d of the K-th violation.  Its
// threshold (d, then all ones) then bounds a collect-only run of the last
// level: sources past it get no attempts.
struct WinJob {
  int32_t active, k;
  uint64_t K;
  unsigned long long* hist;  // [RADIX_BINS], zero at rest
  uint32_t* prefix;          // decided bits of d
  unsigned long long* rank;  // remaining rank within the decided prefix
  int32_t* thr;              // [k]
  uint32_t* d_thr_valid;
  uint64_t* d_vcount;
};

struct TopkJob {
  int32_t active, k, K;
  const int32_t* vbuf;
  const uint64_t* d_vcount;
  uint64_t vcap;
  int32_t* res;
  uint32_t* d_need_select;
};

// Radix select of the K-th smallest staged tuple of one job (lexicographic on
// unsigned ids), then either the first K sorted into `out`, or the K-th tuple
// written to `thr` as the job's staging threshold (staging then restarts).
struct SelJob {
  int32_t active, k, K;
  uint64_t* d_vcount;
  const int32_t* vbuf;
  uint64_t vcap;
  uint32_t* state;                 // [MAXK + 2]: tuple, rank, blocks done
  uint32_t* hist;                  // [RADIX_BINS], zero at rest
  int32_t* out;                    // [K * k]
  unsigned long long* d_outcount;
  int32_t* thr;                    // [k]
  uint32_t* d_thr_valid;
};

// Unit counts of the enumeration, kept by a counting build (compiled with
// -DGFD_COUNT_UNITS) beside the algorithmic bytes: what the last level does
// -- attempts, sources, attempts past injectivity, checks by kind and how
// they were settled, search steps, the sum of ceil(log2 d) over the searched
// rows, matches, literal values read, violations -- and the inner levels'
// attempts.  A normal build keeps none (units_counted() is false).
enum {
  U_ATTEMPTS, U_SOURCES, U_INJECTIVE, U_CHK_BOTH, U_TABLE_FREE, U_TABLE_HIT, U_SHORT_ROW,
  U_BOTH_STEPS, U_BOTH_LOG2D, U_CHK_ONE, U_ONE_STEPS, U_ONE_LOG2D, U_MATCHES, U_LIT_READS,
  U_VIOLATIONS, U_INNER_ATTEMPTS, UNIT_KINDS
};
struct Units {
  unsigned long long c[UNIT_KINDS];
};
bool units_counted();
void units_clear(hipStream_t st);
void units_read(hipStream_t st, uint64_t* host);  // [UNIT_KINDS], synchronous

// Launch wrappers (gfd_kernels.hip).  All asynchronous on `st`; `jobs` points
// to `njobs` (<= MAX_JOBS) device-resident job records.  Per-job kernels run
// on a (gx, njobs) grid; the flat (load-balanced) ones and the scans on a 1-D
// grid of `grid` blocks shared by all jobs (the scans share it by their
// tiles).  `bytes`, when not null, accumulates the algorithmic bytes the
// kernel touched.
void filter_scan(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                 unsigned long long* bytes = nullptr);
// bitmaps: the launch's jobs record hits in bitmaps (hitmode 1) rather than
// bytes; every job of one launch uses the same form
void filter_pull(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                 bool bitmaps, unsigned long long* bytes);
void filter_compact(hipStream_t st, const DevGraph& g, const FilterJob* jobs, int njobs, int grid,
                    bool bitmaps, unsigned long long* bytes);
// zero the output bitmap of every active job
void filter_clear(hipStream_t st, const FilterJob* jobs, int njobs, int gx);
void cpi_scan(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
              unsigned long long* bytes = nullptr);
void cpi_reserve(hipStream_t st, const CpiJob* jobs, int njobs);
// one pass (reserve, then fill) or two (count, alloc, fill) per tree edge
void cpi_count(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
               unsigned long long* bytes);
void cpi_alloc(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int gx);
void cpi_fill(hipStream_t st, const DevGraph& g, const CpiJob* jobs, int njobs, int grid,
              bool onepass, unsigned long long* bytes);
// 1-D grid of `grid` blocks shared among the jobs by their scan tiles
void ext_scan(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int grid,
              unsigned long long* bytes = nullptr);
// After the scan of inner level i (records `cur`): reserves every job's next
// frontier from `pool` (bump cursor *cursor, pool_bytes in all) and points
// cur's dst_*, next's src_* / begs / scan arrays (next may be null) and leaf's
// src_* (for a job whose postponed leaves follow; may be null) at it.  A job
// the pool cannot hold keeps dst_cap = 0 (its first kept match flags a
// frontier overflow).
void front_reserve(hipStream_t st, ExtJob* cur, ExtJob* next, LeafJob* leaf, int njobs,
                   uint8_t* pool, uint64_t pool_bytes, unsigned long long* cursor);
// ahead (last level only): load every round's first probe slot before the
// rounds run -- more loads in flight, fewer waves; for cache-resident graphs
void ext_run(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int grid, bool last,
             bool ahead, bool occ8, unsigned long long* bytes);
// k == 1: every member of the root's candidate set is a match.
void ext_single(hipStream_t st, const DevGraph& g, const ExtJob* jobs, int njobs, int gx,
                unsigned long long* bytes);
void topk_small(hipStream_t st, const TopkJob* jobs, int njobs, unsigned long long* bytes = nullptr);

// n 8-byte words from src (mapped pinned host memory) to dst (device memory)
void copy_words(hipStream_t st, const uint64_t* src, uint64_t* dst, uint64_t n);
// Records of `words` 8-byte words at base + off[r], r < n, back to back into
// dst (which may be mapped host memory): one launch for what would be n
// small device-to-host copies.
struct RecGather {
  uint64_t off[MAX_JOBS];
  int32_t n;
  uint32_t words;
};
void gather_recs(hipStream_t st, const uint8_t* base, const RecGather& g, uint64_t* dst);

// One job's reported tuples: `words` int32 from `src`, packed at word `dst`.
struct PackJob {
  const int32_t* src;
  uint64_t dst;
  uint64_t words;
};
// packs the listed jobs' first-K tuples back to back into `out` (one block per job)
void pack_results(hipStream_t st, const PackJob* jobs, int njobs, int32_t* out);
// per member of C(p): how many of its leaf-list members meet each predicate subset
void leaf_prep(hipStream_t st, const DevGraph& g, const LeafJob* jobs, int njobs, int grid);
// per partial match: its injective leaf completions, counted into the job's
// counters; `split` picks the jobs with split leaves, else the others
void leaf_count(hipStream_t st, const DevGraph& g, const LeafJob* jobs, int njobs, int grid,
                bool split, unsigned long long* bytes);
// window select: before the first digit, prefix = 0 and rank = K; each call
// decides `bits` bits at `shift` from the histogram (and clears it); the
// last writes the threshold and restarts the staging count
void win_begin(hipStream_t st, const WinJob* jobs, int njobs);
void win_digit(hipStream_t st, const WinJob* jobs, int njobs, int shift, int bits, bool last);

// Batched radix select (grid row = job); requires more than K staged tuples
// per active job.  sel_pass decides `bits` bits of tuple word `word` starting
// at bit `shift` (jobs with k <= word are skipped).
void sel_begin(hipStream_t st, const SelJob* jobs, int njobs);
void sel_pass(hipStream_t st, const SelJob* jobs, int njobs, int word, int shift, int bits, int gx,
              unsigned long long* bytes = nullptr);
void sel_first_k(hipStream_t st, const SelJob* jobs, int njobs, int gx, unsigned long long* bytes = nullptr);
void sel_threshold(hipStream_t st, const SelJob* jobs, int njobs);

void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, uint64_t n);
void fill_u64(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n);
void fill_u32(hipStream_t st, uint32_t* p, uint32_t v, uint64_t n);

}  // namespace gfd
