/*
 * CPU oracle for GFD validation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The product path never calls it and shares no code
 * with it.
 *
 * What it computes is the plain definition of Section II of the FastGFDs paper
 * (graph, pattern, match, GFD, satisfaction, violation), by naive backtracking
 * over the pattern variables in their declared order x0, x1, ...  There is no
 * index, no ordering heuristic and no pruning beyond the definition itself.
 *
 *   Match (Section II, definition of a match of Q[x] in G): an assignment
 *   t = (t_0..t_{k-1}) of pairwise distinct data vertices such that
 *     - every pattern vertex label equals the data vertex label, unless the
 *       pattern label is the wildcard (-1);
 *     - for every pattern edge (x_i, x_j, l): (t_i, t_j) is a data edge, and its
 *       label equals l unless l is the wildcard;
 *     - induced semantics (the paper's "if and only if" on edges, and the
 *       remark that a match may not contain additional edges): for every
 *       ordered pair i != j that is NOT a pattern edge, (t_i, t_j) is not a data
 *       edge.  The non-induced ("mono") reading drops this third condition.
 *   Literals (Section II, GFD definition and the remark on missing attributes):
 *     constant x_i.A = c holds iff t_i has attribute A (value != -1) and it
 *     equals c; variable x_i.A = x_j.B holds iff both attributes exist and are
 *     equal.  An empty X or Y holds.  Y = false never holds.
 *   Violation (Section II, validation problem): a match with X true and Y false.
 *
 * Outputs per GFD: match count, violation count, the violations' lexicographic
 * first K tuples (in variable order, compared as unsigned 32-bit ids), and two
 * order-independent fingerprints: the sums mod 2^64 of H(t) over all matches
 * and over all violations, H being the splitmix64 finaliser (Steele, Lea and
 * Flood 2014) chained over the tuple: h0 = 0x9E3779B97F4A7C15 * k,
 * h_{i+1} = mix(h_i XOR t_i), H = h_k.
 *
 * Root range: only assignments with t_0 in [root_lo, root_hi) are explored, so a
 * bounded sample (or a partition across threads) of the full job can be run.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONE (-2) /* "no edge" marker in the edge lookup and pattern matrix */
#define ORC_ANY (-1)  /* wildcard label */
#define ORC_ABSENT (-1)
#define ORC_MAXK 16

typedef struct {
  int32_t kind; /* 0 = constant literal, 1 = variable literal */
  int32_t var, attr, var2, attr2, value;
} orc_lit;

typedef struct {
  int64_t n, m;
  int64_t *out_ptr, *in_ptr;
  int32_t *out_dst, *out_lab, *in_src, *in_lab;
  int32_t *vlabel;
  int32_t num_attrs;
  int32_t *attrs; /* [num_attrs * n] */
} orc_graph;

/* ------------------------------------------------------------------------ */
/* graph: private copy with every row sorted by neighbour id                */
/* ------------------------------------------------------------------------ */

static int cmp_pair(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  return (x[0] > y[0]) - (x[0] < y[0]);
}

static void sort_rows(int64_t n, const int64_t *ptr, int32_t *nbr, int32_t *lab) {
  int64_t maxd = 0;
  for (int64_t v = 0; v < n; v++)
    if (ptr[v + 1] - ptr[v] > maxd) maxd = ptr[v + 1] - ptr[v];
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(maxd + 1));
  for (int64_t v = 0; v < n; v++) {
    int64_t a = ptr[v], d = ptr[v + 1] - a;
    for (int64_t i = 0; i < d; i++) { tmp[2 * i] = nbr[a + i]; tmp[2 * i + 1] = lab[a + i]; }
    qsort(tmp, (size_t)d, 2 * sizeof(int32_t), cmp_pair);
    for (int64_t i = 0; i < d; i++) { nbr[a + i] = tmp[2 * i]; lab[a + i] = tmp[2 * i + 1]; }
  }
  free(tmp);
}

void orc_graph_free(void *h) {
  orc_graph *g = (orc_graph *)h;
  if (!g) return;
  free(g->out_ptr); free(g->in_ptr); free(g->out_dst); free(g->out_lab);
  free(g->in_src); free(g->in_lab); free(g->vlabel); free(g->attrs);
  free(g);
}

/* Returns NULL on malformed input (range errors, self-loops, duplicate pairs). */
void *orc_graph_new(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                    const int32_t *vlabel, const int32_t *elabel, int32_t num_attrs,
                    const int32_t *attrs) {
  orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
  g->n = n; g->m = m; g->num_attrs = num_attrs;
  g->out_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  g->in_ptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  g->out_dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->out_lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->in_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->in_lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->vlabel = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  g->attrs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(num_attrs * n + 1));
  memcpy(g->out_ptr, row_ptr, sizeof(int64_t) * (size_t)(n + 1));
  memcpy(g->out_dst, col, sizeof(int32_t) * (size_t)m);
  memcpy(g->out_lab, elabel, sizeof(int32_t) * (size_t)m);
  memcpy(g->vlabel, vlabel, sizeof(int32_t) * (size_t)n);
  if (num_attrs) memcpy(g->attrs, attrs, sizeof(int32_t) * (size_t)(num_attrs * n));
  if (row_ptr[0] != 0 || row_ptr[n] != m) { orc_graph_free(g); return NULL; }
  for (int64_t v = 0; v < n; v++)
    if (row_ptr[v + 1] < row_ptr[v]) { orc_graph_free(g); return NULL; }
  for (int64_t e = 0; e < m; e++)
    if (col[e] < 0 || col[e] >= n) { orc_graph_free(g); return NULL; }
  sort_rows(n, g->out_ptr, g->out_dst, g->out_lab);
  for (int64_t v = 0; v < n; v++)
    for (int64_t e = g->out_ptr[v]; e < g->out_ptr[v + 1]; e++) {
      if (g->out_dst[e] == v) { orc_graph_free(g); return NULL; }
      if (e > g->out_ptr[v] && g->out_dst[e] == g->out_dst[e - 1]) { orc_graph_free(g); return NULL; }
    }
  /* in-rows: counting sort by target; sources visited in increasing order */
  for (int64_t e = 0; e < m; e++) g->in_ptr[g->out_dst[e] + 1]++;
  for (int64_t v = 0; v < n; v++) g->in_ptr[v + 1] += g->in_ptr[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  memcpy(fill, g->in_ptr, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t v = 0; v < n; v++)
    for (int64_t e = g->out_ptr[v]; e < g->out_ptr[v + 1]; e++) {
      int64_t s = fill[g->out_dst[e]]++;
      g->in_src[s] = (int32_t)v;
      g->in_lab[s] = g->out_lab[e];
    }
  free(fill);
  return g;
}

/* Label of data edge a->b, or ORC_NONE when (a, b) is not in E. */
static int32_t edge_label(const orc_graph *g, int32_t a, int32_t b) {
  int64_t lo = g->out_ptr[a], hi = g->out_ptr[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->out_dst[mid] < b) lo = mid + 1; else hi = mid;
  }
  if (lo < g->out_ptr[a + 1] && g->out_dst[lo] == b) return g->out_lab[lo];
  return ORC_NONE;
}

/* ------------------------------------------------------------------------ */
/* fingerprint                                                              */
/* ------------------------------------------------------------------------ */

static uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27; z *= 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return z;
}

static uint64_t tuple_hash(const int32_t *t, int k) {
  uint64_t h = 0x9E3779B97F4A7C15ULL * (uint64_t)k;
  for (int i = 0; i < k; i++) h = mix64(h ^ (uint64_t)(uint32_t)t[i]);
  return h;
}

/* ------------------------------------------------------------------------ */
/* one search                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_graph *g;
  int k;
  int32_t qlab[ORC_MAXK];
  int32_t qe[ORC_MAXK][ORC_MAXK]; /* label of pattern edge i->j, ORC_ANY, or ORC_NONE */
  int nx, ny, y_false, induced;
  const orc_lit *x, *y;
  int K;
  /* results */
  uint64_t matches, violations, match_fp, viol_fp;
  int32_t *heap; /* K tuples, max-heap in lexicographic order */
  int heap_n;
  int32_t t[ORC_MAXK];
} orc_search;

/* lexicographic comparison of tuples as unsigned 32-bit ids */
static int lex_cmp(const int32_t *a, const int32_t *b, int k) {
  for (int i = 0; i < k; i++) {
    uint32_t x = (uint32_t)a[i], y = (uint32_t)b[i];
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

static void heap_offer(orc_search *s, const int32_t *t) {
  int k = s->k;
  if (s->K <= 0) return;
  if (s->heap_n < s->K) {
    int i = s->heap_n++;
    memcpy(s->heap + (size_t)i * k, t, sizeof(int32_t) * k);
    while (i > 0) {
      int p = (i - 1) / 2;
      if (lex_cmp(s->heap + (size_t)p * k, s->heap + (size_t)i * k, k) >= 0) break;
      int32_t tmp[ORC_MAXK];
      memcpy(tmp, s->heap + (size_t)p * k, sizeof(int32_t) * k);
      memcpy(s->heap + (size_t)p * k, s->heap + (size_t)i * k, sizeof(int32_t) * k);
      memcpy(s->heap + (size_t)i * k, tmp, sizeof(int32_t) * k);
      i = p;
    }
    return;
  }
  if (lex_cmp(t, s->heap, k) >= 0) return; /* not below the current K-th */
  memcpy(s->heap, t, sizeof(int32_t) * k);
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, big = i;
    if (l < s->heap_n && lex_cmp(s->heap + (size_t)l * k, s->heap + (size_t)big * k, k) > 0) big = l;
    if (r < s->heap_n && lex_cmp(s->heap + (size_t)r * k, s->heap + (size_t)big * k, k) > 0) big = r;
    if (big == i) break;
    int32_t tmp[ORC_MAXK];
    memcpy(tmp, s->heap + (size_t)big * k, sizeof(int32_t) * k);
    memcpy(s->heap + (size_t)big * k, s->heap + (size_t)i * k, sizeof(int32_t) * k);
    memcpy(s->heap + (size_t)i * k, tmp, sizeof(int32_t) * k);
    i = big;
  }
}

static int32_t attr_of(const orc_graph *g, int32_t a, int32_t v) {
  return g->attrs[(int64_t)a * g->n + v];
}

static int literal_holds(const orc_search *s, const orc_lit *l) {
  const orc_graph *g = s->g;
  int32_t a = attr_of(g, l->attr, s->t[l->var]);
  if (l->kind == 0) return a != ORC_ABSENT && a == l->value;
  int32_t b = attr_of(g, l->attr2, s->t[l->var2]);
  return a != ORC_ABSENT && b != ORC_ABSENT && a == b;
}

static void record_match(orc_search *s) {
  uint64_t h = tuple_hash(s->t, s->k);
  s->matches++;
  s->match_fp += h;
  int X = 1, Y = 1;
  for (int i = 0; i < s->nx; i++) X = X && literal_holds(s, &s->x[i]);
  if (s->y_false) Y = 0;
  else for (int i = 0; i < s->ny; i++) Y = Y && literal_holds(s, &s->y[i]);
  if (X && !Y) {
    s->violations++;
    s->viol_fp += h;
    heap_offer(s, s->t);
  }
}

/* Does data vertex v fit variable i given t_0..t_{i-1}?  The definition. */
static int fits(const orc_search *s, int i, int32_t v) {
  const orc_graph *g = s->g;
  if (s->qlab[i] != ORC_ANY && g->vlabel[v] != s->qlab[i]) return 0;
  for (int j = 0; j < i; j++)
    if (s->t[j] == v) return 0;
  for (int j = 0; j < i; j++) {
    int32_t fwd = edge_label(g, s->t[j], v); /* data edge t_j -> v */
    int32_t bwd = edge_label(g, v, s->t[j]); /* data edge v -> t_j */
    if (s->qe[j][i] != ORC_NONE) {
      if (fwd == ORC_NONE) return 0;
      if (s->qe[j][i] != ORC_ANY && fwd != s->qe[j][i]) return 0;
    } else if (s->induced && fwd != ORC_NONE) {
      return 0;
    }
    if (s->qe[i][j] != ORC_NONE) {
      if (bwd == ORC_NONE) return 0;
      if (s->qe[i][j] != ORC_ANY && bwd != s->qe[i][j]) return 0;
    } else if (s->induced && bwd != ORC_NONE) {
      return 0;
    }
  }
  return 1;
}

static void extend(orc_search *s, int i, int64_t lo0, int64_t hi0) {
  const orc_graph *g = s->g;
  if (i == s->k) { record_match(s); return; }
  /* candidates: neighbours of the first earlier variable adjacent to x_i,
     else every vertex (the root range at depth 0) */
  for (int j = 0; j < i; j++) {
    if (s->qe[j][i] != ORC_NONE) {
      int32_t u = s->t[j];
      for (int64_t e = g->out_ptr[u]; e < g->out_ptr[u + 1]; e++) {
        int32_t v = g->out_dst[e];
        if (fits(s, i, v)) { s->t[i] = v; extend(s, i + 1, 0, 0); }
      }
      return;
    }
    if (s->qe[i][j] != ORC_NONE) {
      int32_t u = s->t[j];
      for (int64_t e = g->in_ptr[u]; e < g->in_ptr[u + 1]; e++) {
        int32_t v = g->in_src[e];
        if (fits(s, i, v)) { s->t[i] = v; extend(s, i + 1, 0, 0); }
      }
      return;
    }
  }
  int64_t lo = i == 0 ? lo0 : 0, hi = i == 0 ? hi0 : g->n;
  for (int64_t v = lo; v < hi; v++)
    if (fits(s, i, (int32_t)v)) { s->t[i] = (int32_t)v; extend(s, i + 1, 0, 0); }
}

/* ------------------------------------------------------------------------ */
/* threads: root ids in chunks handed out by an atomic counter              */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_search s;
  int64_t lo, hi, chunk;
  int64_t *next;
} orc_worker;

static void *worker_main(void *arg) {
  orc_worker *w = (orc_worker *)arg;
  for (;;) {
    int64_t c = __atomic_fetch_add(w->next, 1, __ATOMIC_RELAXED);
    int64_t a = w->lo + c * w->chunk;
    if (a >= w->hi) break;
    int64_t b = a + w->chunk < w->hi ? a + w->chunk : w->hi;
    extend(&w->s, 0, a, b);
  }
  return NULL;
}

static int qsort_lex(const void *a, const void *b, void *kp) {
  return lex_cmp((const int32_t *)a, (const int32_t *)b, *(const int *)kp);
}

/*
 * Validate one GFD.  Returns 0, or -1 on malformed pattern/literals.
 *   qedges: ne triples (src, dst, label); label -1 = any label
 *   out[4] = {match_count, violation_count, match_fp, violation_fp}
 *   viol: capacity K*k, filled with the first min(K, violations) violations,
 *         ascending; *nrep receives that number.
 */
int orc_validate(void *gh, int32_t k, const int32_t *qlab, int32_t ne, const int32_t *qedges,
                 int32_t nx, const orc_lit *x, int32_t ny, const orc_lit *y, int32_t y_false,
                 int32_t induced, int32_t K, int64_t root_lo, int64_t root_hi, int32_t nthreads,
                 uint64_t *out, int32_t *viol, int32_t *nrep) {
  const orc_graph *g = (const orc_graph *)gh;
  if (k < 1 || k > ORC_MAXK || K < 0) return -1;
  orc_search base;
  memset(&base, 0, sizeof(base));
  base.g = g; base.k = k; base.nx = nx; base.ny = ny; base.x = x; base.y = y;
  base.y_false = y_false; base.induced = induced; base.K = K;
  for (int i = 0; i < k; i++) base.qlab[i] = qlab[i];
  for (int i = 0; i < ORC_MAXK; i++)
    for (int j = 0; j < ORC_MAXK; j++) base.qe[i][j] = ORC_NONE;
  for (int e = 0; e < ne; e++) {
    int32_t a = qedges[3 * e], b = qedges[3 * e + 1];
    if (a < 0 || a >= k || b < 0 || b >= k || a == b) return -1;
    if (base.qe[a][b] != ORC_NONE) return -1;
    base.qe[a][b] = qedges[3 * e + 2] < 0 ? ORC_ANY : qedges[3 * e + 2];
  }
  for (int i = 0; i < nx + ny; i++) {
    const orc_lit *l = i < nx ? &x[i] : &y[i - nx];
    if (l->var < 0 || l->var >= k || l->attr < 0 || l->attr >= g->num_attrs) return -1;
    if (l->kind == 1 && (l->var2 < 0 || l->var2 >= k || l->attr2 < 0 || l->attr2 >= g->num_attrs)) return -1;
  }
  if (root_lo < 0) root_lo = 0;
  if (root_hi > g->n || root_hi < 0) root_hi = g->n;
  if (nthreads < 1) nthreads = 1;

  orc_worker *ws = (orc_worker *)calloc((size_t)nthreads, sizeof(orc_worker));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  int64_t next = 0;
  for (int i = 0; i < nthreads; i++) {
    ws[i].s = base;
    ws[i].s.heap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1) * k);
    ws[i].lo = root_lo; ws[i].hi = root_hi; ws[i].chunk = 256; ws[i].next = &next;
  }
  if (nthreads == 1) worker_main(&ws[0]);
  else {
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, worker_main, &ws[i]);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
  }
  /* merge: sums, and the union of the per-thread first-K sets cut to K */
  uint64_t mc = 0, vc = 0, mf = 0, vf = 0;
  int64_t total = 0;
  for (int i = 0; i < nthreads; i++) {
    mc += ws[i].s.matches; vc += ws[i].s.violations;
    mf += ws[i].s.match_fp; vf += ws[i].s.viol_fp;
    total += ws[i].s.heap_n;
  }
  int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1) * k);
  int64_t pos = 0;
  for (int i = 0; i < nthreads; i++) {
    memcpy(all + pos * k, ws[i].s.heap, sizeof(int32_t) * (size_t)ws[i].s.heap_n * k);
    pos += ws[i].s.heap_n;
    free(ws[i].s.heap);
  }
  int kk = k;
  qsort_r(all, (size_t)total, sizeof(int32_t) * k, qsort_lex, &kk);
  int64_t rep = total < K ? total : K;
  memcpy(viol, all, sizeof(int32_t) * (size_t)rep * k);
  *nrep = (int32_t)rep;
  out[0] = mc; out[1] = vc; out[2] = mf; out[3] = vf;
  free(all); free(ws); free(th);
  return 0;
}
