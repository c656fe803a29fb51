/*
 * gfd.h -- C ABI of the MI355X (gfx950) GFD-validation library.
 *
 * A graph functional dependency (GFD) phi = (Q[x], X -> Y) or (Q[x], X -> false)
 * pairs a graph pattern Q with attribute literals (FastGFDs paper, Section II).
 * Validation of a set of GFDs over a graph G finds the violations: matches h of
 * Q in G with h |= X and h |/= Y (Section II, "the validation problem").  This
 * library computes, per GFD, the exact match and violation counts, the
 * satisfied flag, the lexicographically first K violating matches and two
 * order-independent fingerprints, on one GPU.  The matching follows the
 * Compact Path Index and Core-First decomposition the paper adopts in
 * Section IV-B; those only prune and order the search, so results are those
 * of the plain definition.
 *
 * Conventions
 *   - Every call returns an int32_t status (GFD_OK or a negative GFD_E* code);
 *     gfd_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses this boundary.
 *   - Vertex ids are 0..n-1 (n < 2^31); edge count m < 2^32.
 *   - Labels are int32 >= 0; GFD_WILDCARD (-1) in a pattern matches any label
 *     (vertex labels: Section II's wildcard; edge labels: any label).
 *   - Attributes are dictionary-encoded int32 columns; GFD_ABSENT (-1) means the
 *     vertex has no such attribute.  A literal that touches a missing attribute
 *     is false (Section II: such constraints hold trivially in X, and a
 *     literal in Y demands that the attribute exist).
 *   - Matching semantics: GFD_SEM_INDUCED (default) reads Section II's match
 *     definition literally -- an ordered pair of matched vertices is a data
 *     edge iff it is a pattern edge, with equal labels.  GFD_SEM_MONO drops
 *     the "only if" (extra data edges between matched vertices allowed).
 */
#ifndef GFD_H
#define GFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define GFD_OK 0
#define GFD_EINVAL (-1)       /* malformed graph, spec or option */
#define GFD_ENOMEM (-2)       /* device or host allocation failed, or budget too small */
#define GFD_EDEVICE (-3)      /* HIP runtime error */
#define GFD_EUNSUPPORTED (-4) /* valid input outside this build's limits */
#define GFD_EOVERFLOW (-5)    /* a 64-bit counter would pass 2^63 */
#define GFD_EAGAIN (-6)       /* a server request did not finish within the wait's timeout */

#define GFD_WILDCARD (-1)
#define GFD_ABSENT (-1)
#define GFD_MAX_K 8          /* pattern vertices per GFD */
#define GFD_MAX_LITERALS 8   /* literals in X, and separately in Y */
#define GFD_MAX_PATTERN_EDGES (GFD_MAX_K * (GFD_MAX_K - 1))

#define GFD_LIT_CONST 0 /* x_var.attr = constant            (Section II, constant literal) */
#define GFD_LIT_VAR 1   /* x_var.attr = x_var2.attr2         (Section II, variable literal) */

#define GFD_SEM_INDUCED 0
#define GFD_SEM_MONO 1

typedef struct gfd_graph gfd_graph; /* opaque; device-resident graph */

typedef struct {
  int32_t kind;     /* GFD_LIT_CONST or GFD_LIT_VAR */
  int32_t var;      /* pattern variable index, 0..num_vertices-1 */
  int32_t attr;     /* attribute column, 0..num_attrs-1 */
  int32_t var2;     /* GFD_LIT_VAR only */
  int32_t attr2;    /* GFD_LIT_VAR only */
  int32_t constant; /* GFD_LIT_CONST only; must be >= 0 */
} gfd_literal;

typedef struct {
  int32_t src, dst; /* pattern variables; src != dst */
  int32_t label;    /* edge label, or GFD_WILDCARD */
} gfd_edge;

/* One GFD.  Variable order x = (x_0 .. x_{k-1}) is the index order below; it is
 * the order of every reported tuple.  At most one edge per ordered pair.  The
 * pattern may have several connected components (Section IV-A); a further
 * component is joined to the first by a cross product of candidates. */
typedef struct {
  int32_t num_vertices;                 /* k, 1..GFD_MAX_K */
  int32_t vertex_labels[GFD_MAX_K];     /* label or GFD_WILDCARD */
  int32_t num_edges;
  gfd_edge edges[GFD_MAX_PATTERN_EDGES];
  int32_t num_x;
  gfd_literal x[GFD_MAX_LITERALS];
  int32_t num_y;
  gfd_literal y[GFD_MAX_LITERALS];
  int32_t y_is_false;                   /* nonzero: X -> false (Y ignored) */
} gfd_spec;

/* Per-GFD result.  violations is caller-owned with room for
 * k_max * num_vertices int32 (row-major tuples in variable order); it may be
 * NULL when k_max == 0. */
typedef struct {
  int32_t satisfied;        /* 1 iff violation_count == 0 */
  int32_t num_reported;     /* min(k_max, violation_count) */
  uint64_t match_count;     /* number of matches (embeddings, tuples in x order) */
  uint64_t violation_count; /* matches with X true and Y false */
  uint64_t match_fp;        /* sum over matches of H(t) mod 2^64 */
  uint64_t violation_fp;    /* sum over violations of H(t) mod 2^64 */
  int32_t* violations;      /* [k_max * num_vertices], ascending lexicographic */
} gfd_result;
/* H(t): splitmix64 finaliser mix (Steele, Lea & Flood 2014) chained over the
 * tuple: h = 0x9E3779B97F4A7C15 * k; for each t_i: h = mix(h ^ (uint32)t_i). */

/* Device memory callbacks.  alloc returns `bytes` of device memory, aligned to
 * at least 256 bytes, that work on `hip_stream` may use (NULL on failure: the
 * call then fails with GFD_ENOMEM); free returns a block alloc gave, with its
 * size.  ctx is passed back unchanged.  alloc == NULL means the library's own
 * hipMalloc / hipFree.  Callbacks may be called from any thread that calls
 * into the library (and from server worker threads).  Memory given to a graph
 * is returned by gfd_free_graph; workspace memory a graph keeps between
 * validate calls is returned by gfd_trim or gfd_free_graph, so the callbacks
 * must stay valid until then. */
typedef struct {
  void* (*alloc)(void* ctx, int64_t bytes, void* hip_stream);
  void (*free)(void* ctx, void* ptr, int64_t bytes);
  void* ctx;
} gfd_allocator;

#define GFD_MEM_HOST 0   /* input arrays are host memory */
#define GFD_MEM_DEVICE 1 /* input arrays are device memory of the current device */

typedef struct {
  void* hip_stream;        /* hipStream_t for the upload; NULL = the null stream */
  int32_t mem_kind;        /* GFD_MEM_HOST or GFD_MEM_DEVICE: where row_ptr, col, vlabel,
                              elabel and the attribute columns live (the array of
                              column pointers itself is always host memory) */
  gfd_allocator allocator; /* device memory of the graph; alloc == NULL: hipMalloc */
} gfd_load_opts;

/* Launch shapes of a call (an autotuner's choices; 0 keeps the library's
 * default).  They change only how work is spread over the GPU, never a
 * result.  Out-of-range values are GFD_EINVAL. */
typedef struct {
  int32_t flat_grid;     /* blocks of the enumeration launches (64..16384; 0: 2048) */
  int32_t scan_grid;     /* blocks of the enumeration level scans (64..16384; 0: 2048) */
  int32_t probe_ahead;   /* last level: 1 loads every round's first probe slot before
                            any round runs, 2 does not, 0 picks by graph size */
  int32_t staging_log2;  /* violation staging per GFD in a batch, 2^n tuples (10..24;
                            0: from the budget, at most 2^18) */
  int32_t ext_occupancy; /* enumeration levels: 1 runs the kernels with the registers
                            the compiler allocates (5 waves per SIMD at the last
                            level), 2 with at most 64 per lane so that 8 waves share
                            a SIMD (the rest spilled to scratch), which hides more
                            HBM latency when the graph does not fit in cache; 0
                            picks by graph size */
} gfd_tuning;

typedef struct {
  int32_t k_max;            /* K: violations to report per GFD, >= 0 */
  int32_t semantics;        /* GFD_SEM_INDUCED or GFD_SEM_MONO */
  int64_t mem_budget_bytes; /* device bytes for frontiers and buffers; 0 = default */
  void* hip_stream;         /* hipStream_t to run on; NULL = the null stream */
  int32_t batched;          /* 0: one GFD after another; 1: GFDs run together in
                               batches, one launch per kernel per phase of a batch */
  int32_t flags;            /* GFD_FLAG_* bits */
  int64_t frontier_cap;     /* testing: max partial matches per level (0 = from budget) */
  int64_t violation_cap;    /* testing: violation staging capacity in tuples (0 = default) */
  gfd_allocator allocator;  /* device memory of the call's workspace; alloc == NULL:
                               hipMalloc.  The graph keeps a workspace per allocator
                               between calls (see gfd_trim) */
  gfd_tuning tuning;        /* launch shapes; all zero = the defaults */
} gfd_validate_opts;

#define GFD_FLAG_FORCE_CHUNKED 1 /* skip the single-pass fast path */
#define GFD_FLAG_TIMING 2        /* record HIP event timings for every kernel class */
/* Counts only: match and violation counts, satisfied flags and (k_max > 0)
 * the first k_max violations; both fingerprints are reported as 0.  Under
 * GFD_SEM_MONO, a pattern whose matching order ends in up to 3 leaves with
 * one parent, equal labels and edges, and literals on themselves alone has
 * those leaves counted per partial match (inclusion-exclusion over their
 * candidate lists) instead of enumerated: the leaf postponement of CFL-Match
 * that Section IV-B adopts.  Two last leaves under different parents are
 * counted together too: the product of their lists' sizes less the vertices
 * both lists hold.  With k_max > 0 only the last leaf is counted, and only
 * when it is not variable 0; its level then runs again over the first-K
 * window alone: the partial matches whose variable-0 vertex is at most that
 * of the k_max-th violation (found from the per-match counts). */
#define GFD_FLAG_COUNT_ONLY 4
/* Run every launch eagerly.  By default a batch's main pass (its clears, the
 * candidate filter, CPI construction, enumeration with the literal check and
 * the first K, and the read-back of its counters) is captured as a HIP graph
 * the first time a batch of that shape runs on a workspace and replayed as
 * one graph launch afterwards; results are the same either way.  Calls with
 * timing flags run eagerly. */
#define GFD_FLAG_NO_GRAPH 8
/* record HIP event timings for kernel class c (0..7, see gfd_stats) only */
#define GFD_FLAG_TIMING_CLASS(c) (1 << (8 + (c)))

/* Per-call work and timing statistics (filled when requested). */
typedef struct {
  double wall_ms;             /* host wall time of the call */
  int32_t launches;           /* kernels launched */
  int32_t chunked_gfds;       /* GFDs that needed the chunked (budgeted) path: a
                                 frontier or the CPI entry arena overflowed */
  uint64_t attempts;          /* extension attempts over all enumeration levels */
  uint64_t partials;          /* partial matches written over all levels */
  uint64_t cpi_candidates;    /* sum of final candidate-set sizes */
  uint64_t cpi_entries;       /* CPI arena entries reserved: the rows of every tree
                                 parent's candidates, which bound their lists */
  /* per kernel class: [0] candidate compaction, [1] candidate pull constraints,
   * [2] CPI adjacency, [3] enumeration (inner levels), [4] enumeration + literal
   * check (last level), [5] scans, [6] top-K selection, [7] other */
  int32_t class_launches[8];
  double class_ms[8];         /* summed HIP event time (GFD_FLAG_TIMING) */
  uint64_t class_bytes[8];    /* algorithmic bytes of that class (bytes each item
                                must touch, counted on the device) */
  int32_t threshold_gfds;     /* GFDs whose violation staging overflowed: their last
                                 enumeration level ran again, collecting only the
                                 violations up to a bound on the K-th smallest */
  int32_t threshold_passes;   /* such re-runs (one launch each for all those GFDs) */
  int32_t leaf_gfds;          /* GFDs whose last leaves were counted (GFD_FLAG_COUNT_ONLY) */
  int32_t regrown_gfds;       /* GFDs run again in the fast path: after the frontier pool or
                                 the CPI entry arena grew to what their batch asked for,
                                 or, when a shared pool or arena was at its cap, in a
                                 smaller batch packed by what they asked for, then alone */
  int64_t front_pool_bytes;   /* frontier pool and CPI entry arena sizes after the call */
  int64_t cpi_arena_bytes;
  int32_t graph_captures;     /* batches whose main pass was captured as a graph */
  int32_t graph_replays;      /* batches whose main pass replayed a captured graph */
  int32_t units_counted;      /* 1 in a counting build of the library (units filled) */
  /* enumeration units of a counting build: [0] last-level attempts, [1] their
   * sources, [2] attempts past injectivity, [3] checks of both directions,
   * [4] of them settled by a free table slot, [5] by a fingerprint match and
   * a row search, [6] by a search of a short row, [7] combined-row search
   * steps, [8] sum of ceil(log2 d) over the anchors' combined rows, [9]
   * one-direction probes, [10] their search steps, [11] sum of ceil(log2 d)
   * over their rows, [12] matches, [13] attribute values read by literals,
   * [14] violations, [15] inner-level attempts */
  uint64_t units[16];
  int32_t leaf_split_gfds;    /* of leaf_gfds, those whose last two leaves hang from different
                                 parents (counted as list products less shared vertices) */
  int32_t batches;            /* batches whose main pass ran: the planned ones and those of
                                 GFDs run again (regrown_gfds) */
} gfd_stats;

/* Load a graph given as out-CSR, in host memory or (opts->mem_kind ==
 * GFD_MEM_DEVICE) in device memory of the current device.  Inputs are read
 * and copied: the caller may free them on return.  Rows need not be sorted.
 * attr is a host array of num_attrs pointers to columns of n int32 (values
 * >= 0 or GFD_ABSENT).  The graph's device memory comes from opts->allocator
 * (hipMalloc when none is given).  Errors: GFD_EINVAL for row_ptr not
 * starting at 0 / not non-decreasing / not ending at m, col out of range, a
 * self-loop, a duplicate ordered pair, negative labels, attribute values
 * < -1, null pointers, an allocator with alloc but no free, an unknown
 * mem_kind; GFD_EUNSUPPORTED for n >= 2^31, m >= 2^32, a label id above
 * GFD_MAX_LABEL or more than GFD_MAX_LABEL_PAIRS (vertex label, edge label)
 * combinations (max vertex label + 1 times max edge label + 1); GFD_ENOMEM
 * (host or device allocation) / GFD_EDEVICE from the device.
 * (Section II: E is a subset of V x V, one label per vertex and per edge,
 * attributes on vertices only.) */
#define GFD_MAX_LABEL ((1 << 24) - 1)
#define GFD_MAX_LABEL_PAIRS (1 << 24)
int32_t gfd_load_graph(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                       const int32_t* vlabel, const int32_t* elabel, int32_t num_attrs,
                       const int32_t* const* attr, const gfd_load_opts* opts,
                       gfd_graph** out);

/* Release a graph and every device buffer it owns (through the allocators
 * they came from).  NULL is ignored. */
void gfd_free_graph(gfd_graph* g);

/* Return the device workspaces the graph keeps between validate calls (one
 * per allocator used) to their allocators.  The next call allocates again.
 * Must not overlap a validate call or a server on the same graph. */
int32_t gfd_trim(gfd_graph* g);

/* Validate num_specs GFDs over g (Section II's validation problem, per GFD).
 * Synchronous: returns once every result is on the host.  results is
 * caller-allocated [num_specs], each with its violations buffer.  A malformed
 * spec fails the whole call with GFD_EINVAL before any launch.  Concurrent
 * calls on one graph are allowed on distinct streams. */
int32_t gfd_validate(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                     const gfd_validate_opts* opts, gfd_result* results);

/* gfd_validate plus per-call statistics (stats may be NULL). */
int32_t gfd_validate_ex(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                        const gfd_validate_opts* opts, gfd_result* results, gfd_stats* stats);

/* gfd_validate for callers that cannot allocate (code that must not call
 * hipMalloc or an allocator: tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as gfd_validate, but no
 * device or pinned host memory is allocated and no HIP event is created:
 * every device byte comes from a scratch area of GFD_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on, from its first use until
 * the process ends.  Host staging is ordinary memory, so copies to and from
 * the device are synchronous.  opts->allocator must be empty and opts->flags
 * may hold only GFD_FLAG_FORCE_CHUNKED and GFD_FLAG_COUNT_ONLY; the current
 * device must be the graph's.  A call whose working set does not fit the area
 * fails with GFD_ENOMEM (a smaller batch, or one GFD at a time, needs less).
 * Calls on one device share its area, which keeps the last call's contents:
 * the library runs them one at a time (a second call waits for the first),
 * and nothing else may use the area. */
#define GFD_NOALLOC_SCRATCH_BYTES (256u << 20)
int32_t gfd_validate_noalloc(const gfd_graph* g, const gfd_spec* specs, int32_t num_specs,
                             const gfd_validate_opts* opts, gfd_result* results);

/* Graph facts: sizes and the device bytes it holds. */
typedef struct {
  int64_t n, m;
  int32_t num_attrs, num_vertex_labels, num_edge_labels;
  int64_t device_bytes;
} gfd_graph_info;
int32_t gfd_get_graph_info(const gfd_graph* g, gfd_graph_info* info);

/* ---------------------------------------------------------------------------
 * Serving: the graph stays resident and validation requests (each a list of
 * GFDs) arrive over time.  Worker threads, each with its own HIP stream and
 * workspace, take every request waiting in arrival order -- as many as fit the
 * GFD limit and the per-worker memory budget by their estimated device bytes
 * (candidate sets, CPI lists, frontiers, violation staging) -- and validate
 * them as one batch (gfd_validate with batched = 1).  A request that arrives
 * while batches run joins the next batch a worker forms, and batches on
 * different workers overlap on the GPU.  Results are exactly those of
 * gfd_validate on the request alone (Section II's validation problem per
 * GFD; batching changes only the schedule).
 * ------------------------------------------------------------------------- */
typedef struct gfd_server gfd_server; /* opaque */

typedef struct {
  int32_t workers;          /* batches in flight at once (1..8); 0 = 2 */
  int32_t max_batch_gfds;   /* GFDs per batch (1..256); 0 = 256 */
  int64_t mem_budget_bytes; /* device bytes per worker; 0 = default share */
  int32_t k_max;            /* violations reported per GFD (0..2048) */
  int32_t semantics;        /* GFD_SEM_INDUCED or GFD_SEM_MONO */
  gfd_allocator allocator;  /* device memory of the workers' workspaces; alloc == NULL:
                               hipMalloc.  Must stay valid until gfd_trim or
                               gfd_free_graph on the graph */
} gfd_server_opts;

typedef struct {
  int64_t submit_ns, start_ns, done_ns; /* steady clock: queued, batch start, batch end */
  uint64_t batch_id;                    /* the batch that served the request */
  int32_t batch_gfds, batch_requests;   /* that batch's size */
  int32_t worker;
} gfd_request_info;

/* Start a server on a loaded graph (which must outlive it).  Errors: GFD_EINVAL
 * for options out of range, GFD_EDEVICE / GFD_ENOMEM from the device. */
int32_t gfd_server_create(const gfd_graph* g, const gfd_server_opts* opts, gfd_server** out);

/* Queue one request of num_specs (1..max_batch_gfds) GFDs; specs are copied.
 * A malformed spec fails the submit with GFD_EINVAL (nothing is queued).
 * Thread-safe. */
int32_t gfd_server_submit(gfd_server* s, const gfd_spec* specs, int32_t num_specs,
                          uint64_t* request_id);

/* Wait for a request: timeout_ms < 0 waits without limit; GFD_EAGAIN if it has
 * not finished in time (wait again later).  On completion fills results
 * [num_specs] (each violations buffer caller-owned, room for k_max tuples of
 * that GFD) and info (may be NULL), forgets the request and returns its
 * status: a batch that fails is validated again request by request, so a
 * failing request does not fail the others.  Each request is waited for
 * successfully once; while one thread waits for a request, another wait for
 * the same request fails with GFD_EINVAL. */
int32_t gfd_server_wait(gfd_server* s, uint64_t request_id, int32_t timeout_ms,
                        gfd_result* results, gfd_request_info* info);

/* Finish every queued request, stop the workers and free the server (results
 * never waited for are dropped).  NULL is ignored. */
void gfd_server_destroy(gfd_server* s);

/* Message for the last failing call on this thread ("" if none). */
const char* gfd_last_error(void);

/* Library version, as major*10000 + minor*100 + patch. */
int32_t gfd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GFD_H */
