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
  unsigned long long* bytes;  // optional algorithmic-byte counter
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

// Scan enumeration sources: list length of each partial's parent CPI list.
void scan_sources(hipStream_t st, ScanWs& ws, const int32_t* par_col, const uint64_t* d_n,
                  uint64_t cap, const int32_t* pos_map, const uint32_t* cpi_beg,
                  const uint32_t* cpi_len, uint32_t* beg, uint64_t* P, uint64_t* d_total);

// Decoupled look-back state of one scan launch.
struct TileScan {
  uint64_t* state;
  uint32_t* ticket;
  uint32_t* err;
  uint32_t epoch;
};

// A vertex v passes a pull constraint when some x adjacent to v (out-row if
// dir == 0, in-row if dir == 1) through an edge of label elab (ANY = any) is a
// member of another pattern vertex's candidate set (mem[x] == ep).
struct PullCons {
  int32_t dir;
  int32_t elab;
  const uint8_t* mem;
  uint32_t ep;
};

// Candidate filter (Section IV-B: label candidates, degree filter, and the
// BFS candidate-subgraph / dead-end conditions), compacted in one pass into a
// set in no fixed order (*d_out_n must be zero at launch).
struct CandArgs {
  DevGraph g;
  const int32_t* list;   // nullptr: identity 0..n_host-1
  const uint64_t* d_n;   // device count (nullptr: n_host)
  uint64_t n_host, cap;
  int32_t min_out, min_in;
  int32_t ncons;
  PullCons cons[2 * MAXK];
  int32_t* out;
  uint64_t* d_out_n;     // atomic output counter
  uint8_t* mem;          // mem[v] = mem_ep for kept v
  uint32_t mem_ep;
  int32_t* posmap;       // optional: posmap[v] = index of v in out
  unsigned long long* bytes;  // optional algorithmic-byte counter
};
void cand_filter(hipStream_t st, const CandArgs& a, int grid);

// CPI adjacency N_u^p(v_p) for spanning-tree edge (p, u): for each v_p in C(p)
// the neighbours v (row direction dir) with mem[v] == ep, edge label prim and
// the reverse direction satisfying `other`.  List of the i-th candidate of p:
// cpi_ent[cpi_beg[i] .. cpi_beg[i] + cpi_len[i]) (*d_entries zero at launch).
struct CpiArgs {
  DevGraph g;
  int32_t dir;
  const int32_t* list;
  const uint64_t* d_n;
  uint64_t cap;
  int32_t prim, other;
  const uint8_t* mem;
  uint32_t ep;
  uint32_t* cpi_beg;     // [|C(p)|]
  uint32_t* cpi_len;     // [|C(p)|]
  int32_t* cpi_ent;
  uint64_t* d_entries;   // atomic entry counter
  unsigned long long* bytes;
};
void cpi_adjacency(hipStream_t st, const CpiArgs& a, int grid);

// Enumeration: one attempt window over a scanned frontier (P, beg), every
// attempt of the window mapped to its source by load-balanced search.
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
