// Internal declarations shared by the host driver (gfd_api.hip) and the
// kernels (gfd_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfd {

constexpr int MAXK = 8;
constexpr int MAXLIT = 8;
constexpr int32_t ABSENT = -1;
constexpr int32_t ANY = -1;
constexpr int32_t NOEDGE = -2;

// Constraint on one direction of one vertex pair, checked by a probe:
//   >= 0     a data edge with exactly this label must exist
//   ANY      a data edge with any label must exist
//   PC_ABSENT  no data edge may exist (induced reading, no pattern edge)
//   PC_FREE    no constraint (non-induced reading, no pattern edge)
constexpr int32_t PC_ABSENT = -2;
constexpr int32_t PC_FREE = -3;

constexpr int BS = 256;        // threads per block everywhere
constexpr int WAVE = 64;       // CDNA wavefront
constexpr int SCAN_IPT = 8;    // items per thread in the scan
constexpr int SCAN_TILE = BS * SCAN_IPT;
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
};

struct DevLit {
  int32_t kind;  // 0 const, 1 var
  int32_t pos, attr, pos2, attr2, value;  // pos/pos2: matching-order positions
};

// Arguments of the enumeration kernels: extend level i (i bound vertices) by
// the vertex at matching-order position i.
struct ExtArgs {
  DevGraph g;
  // source frontier: column j (j < i) at src_cols + j * src_stride
  const int32_t* src_cols;
  uint64_t src_stride;
  const uint64_t* d_nsrc;  // sources (device count), clamped to src_cap
  uint64_t src_cap;
  const uint64_t* P;       // exclusive prefix of candidate-list lengths [nsrc+1]
  const uint32_t* beg;     // CPI list start per source
  const int32_t* cpi_ent;  // CPI entries (vertex ids)
  uint64_t a_begin, a_end; // attempt window (a_end clamped to P[nsrc])
  int32_t i;               // position being bound
  int32_t nchk;
  int32_t chk_pos[MAXK];
  int32_t chk_fwd[MAXK];   // constraint on data edge h(x_pos) -> v
  int32_t chk_bwd[MAXK];   // constraint on data edge v -> h(x_pos)
  // inner levels
  int32_t* dst_cols;
  uint64_t dst_cap;
  uint64_t* d_ndst;
  uint32_t* d_flags;       // bit0: frontier overflow; bit1: violation buffer overflow
  // last level
  int32_t k;
  int32_t var_pos[MAXK];   // matching-order position of variable x_v
  int32_t nx, ny, y_false;
  DevLit lit[2 * MAXLIT];  // X literals then Y literals
  unsigned long long* counters;  // [4] match, violation, match_fp, violation_fp
  int32_t* vbuf;           // violation staging [vcap * k], tuples in variable order
  uint64_t* d_vcount;
  uint64_t vcap;
  const int32_t* thr;      // threshold tuple (variable order)
  const uint32_t* d_thr_valid;
  int32_t collect_only;    // 1: only stage tuples, do not touch counters
};

// Launch wrappers (gfd_kernels.hip).  All are asynchronous on `st`.
struct ScanWs {
  uint64_t* tile_state;  // [max tiles]
  uint32_t* ticket;      // zero at rest
  uint32_t* err;
  uint32_t epoch;        // host side, bumped per launch
  uint64_t max_tiles;
};

// Scan sources: for each of n (device count, clamped to cap) list vertices,
// length of its row in `off`; exclusive prefix -> P[0..n], total -> *d_total.
void scan_row_lengths(hipStream_t st, ScanWs& ws, const int32_t* list, const uint64_t* d_n,
                      uint64_t cap, const uint32_t* off, uint64_t* P, uint64_t* d_total);
// Scan word popcounts (flags compaction): words = ceil(n/64).
void scan_popcounts(hipStream_t st, ScanWs& ws, const uint64_t* masks, const uint64_t* d_n,
                    uint64_t cap, uint64_t* pre, uint64_t* d_total);
// Scan enumeration sources: list length of each partial's parent CPI list.
void scan_sources(hipStream_t st, ScanWs& ws, const int32_t* par_col, const uint64_t* d_n,
                  uint64_t cap, const int32_t* pos_map, const uint32_t* cpi_off,
                  uint32_t* beg, uint64_t* P, uint64_t* d_total);

// Candidate filter (label bucket / list -> flags)
struct FilterArgs {
  DevGraph g;
  const int32_t* list;   // nullptr: identity 0..n-1
  const uint64_t* d_n;   // device count (nullptr: n_host)
  uint64_t n_host, cap;
  int32_t min_out, min_in;
  int32_t nmarks;
  const uint8_t* marks[MAXK];
  uint8_t mark_ep[MAXK];
  uint64_t* masks;       // [ceil(cap/64)]
};
void filter_flags(hipStream_t st, const FilterArgs& a, int grid);
void filter_emit(hipStream_t st, const FilterArgs& a, const uint64_t* pre, int32_t* out,
                 uint8_t* mem, uint8_t mem_ep, int grid);

// CPI marking: for rows (dir) of list C (device count), neighbours reached by
// an edge of label elab (ANY = any) whose vertex label is vlab (ANY = any)
// get mark[v] = ep.
void mark_rows(hipStream_t st, const DevGraph& g, int dir, const int32_t* list,
               const uint64_t* d_n, uint64_t cap, const uint64_t* P, const uint64_t* d_total,
               uint64_t total_cap, int32_t elab, int32_t vlab, uint8_t* mark, uint8_t ep,
               int grid);

// CPI adjacency: rows (dir) of C(p); keep entries v with mem[v] == ep, edge
// label `prim` and the other direction satisfying `other` (probe in the
// opposite row of the parent vertex).
struct AdjArgs {
  DevGraph g;
  int dir;               // 0: out rows of C(p), 1: in rows
  const int32_t* list;
  const uint64_t* d_n;
  uint64_t cap;
  const uint64_t* P;     // row-length prefix over list
  const uint64_t* d_total;
  uint64_t total_cap;
  int32_t prim;          // label constraint on the scanned edge (>= 0 or ANY)
  int32_t other;         // constraint on the reverse direction (PC_* codes)
  const uint8_t* mem;
  uint8_t ep;
  uint64_t* masks;       // [ceil(total_cap/64)]
};
void adj_flags(hipStream_t st, const AdjArgs& a, int grid);
void adj_emit(hipStream_t st, const AdjArgs& a, const uint64_t* pre, int32_t* ent, int grid);
void adj_offsets(hipStream_t st, const AdjArgs& a, const uint64_t* pre, uint32_t* cpi_off,
                 int grid);
void pos_map(hipStream_t st, const int32_t* list, const uint64_t* d_n, uint64_t cap,
             int32_t* pos, int grid);

// Enumeration
void extend(hipStream_t st, const ExtArgs& a, bool last, int grid);
void single_vertex(hipStream_t st, const ExtArgs& a, const int32_t* list, const uint64_t* d_n,
                   uint64_t cap, int grid);

// Top-K
// Sort the staged tuples when count <= SORT_MAX, writing the first min(K,count)
// to `res`; otherwise sets *d_need_select = 1.
void topk_small(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap,
                int k, int K, int32_t* res, uint32_t* d_need_select);
// Radix select: find the K-th smallest tuple of vbuf[0..count) (count > K).
// state: [k + 2] words (prefix tuple, remaining rank, pass); hist: [RADIX_BINS].
void select_begin(hipStream_t st, uint32_t* state, int K);
void select_pass(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount, uint64_t vcap,
                 int k, int word, int shift, int bits, uint32_t* state, uint32_t* hist,
                 int grid);
// Keep tuples <= threshold (state prefix) in vbuf order into out; exactly K.
void select_compact(hipStream_t st, const int32_t* vbuf, const uint64_t* d_vcount,
                    uint64_t vcap, int k, const uint32_t* state, int32_t* out,
                    uint64_t* d_outcount, int grid);
// Sort exactly n_host (<= SORT_MAX) tuples in place.
void sort_tuples(hipStream_t st, int32_t* buf, const uint64_t* d_n, int k);

void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, uint64_t n);
void fill_u64(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n);
void fill_u32(hipStream_t st, uint32_t* p, uint32_t v, uint64_t n);

}  // namespace gfd
