/*
 * Streaming CPU oracle ("tier B") for batches of group-by aggregates over the
 * natural join of the relations of a join tree.
 *
 * TEST INFRASTRUCTURE ONLY: called from oracle/tierb.py by the tests, the
 * scripts under tests/golden/ and the cpu_baseline leg of bench.py.  It shares
 * no code with the GPU library.
 *
 * What it computes is the plain definition (paper, section 2 "LMFAO by
 * Example": D is the natural join of all relations, bag semantics; a query
 * SELECT G, SUM(f_1..f_m) FROM D WHERE P GROUP BY G maps each group carried
 * by at least one qualifying tuple of D to the sums of the aggregate terms
 * over those tuples).  Unlike the tier-A oracle it never materialises D: it
 * enumerates the tuples of D one at a time, by nested loops along the join
 * tree -- for every row of the first relation, every row of each next
 * relation (breadth-first order) whose values agree with the rows already
 * chosen on every attribute the two hold, found through an index on the
 * attributes the relation shares with its tree parent -- and adds every
 * query's term into its accumulators.  There is no factorisation: the work is
 * O(|D| * aggregates).
 *
 * Accumulators: int64 counts; per aggregate an FP64 sum with Neumaier
 * compensation plus the sum of |term|.  Queries with few groups are
 * accumulated per thread over row ranges of the first relation and merged in
 * thread order; queries with many groups are owned by one thread each, which
 * enumerates all of D for them (dense arrays, or an open-addressing map when
 * the key space is large).
 *
 * A condition compares the attribute in its column's type: an FP32 column
 * against the constant rounded to FP32, integer and FP64 columns in FP64.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { TB_I32 = 0, TB_F32 = 1, TB_F64 = 2 };
enum { TB_LE = 0, TB_LT = 1, TB_GT = 2, TB_GE = 3, TB_EQ = 4, TB_NE = 5 };

typedef struct {
  /* relations, listed in breadth-first order of the join tree from rel 0 */
  int32_t n_rels;
  const int64_t* n_rows;        /* [n_rels] */
  const int32_t* parent;        /* [n_rels] index of the tree parent, -1 for rel 0 */
  const int32_t* col_off;       /* [n_rels + 1] columns of rel r: col_off[r] .. col_off[r+1] */
  const int32_t* col_attr;      /* [cols] global attribute id */
  const int32_t* col_dtype;     /* [cols] TB_I32 / TB_F32 / TB_F64 */
  const void* const* col_ptr;   /* [cols] column data */
  int32_t n_attrs;
  const int64_t* attr_dom;      /* [n_attrs] integer domain [0, dom), 0 = none */
  /* queries */
  int32_t n_queries;
  const int32_t* gb_off;        /* [n_queries + 1] into gb_attr */
  const int32_t* gb_attr;
  const int32_t* cond_off;      /* [n_queries + 1] into cond_* */
  const int32_t* cond_attr;
  const int32_t* cond_op;
  const double* cond_c;
  const int32_t* agg_off;       /* [n_queries + 1] into agg_f_off (one entry per aggregate) */
  const int32_t* agg_f_off;     /* [aggs + 1] into f_attr / f_pow */
  const int32_t* f_attr;
  const int32_t* f_pow;
} tb_problem;

/* ------------------------------------------------------------------------ */
/* attribute access                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int rel;
  const void* ptr;
  int dtype;
} src_t;

static double get_f(const src_t* s, int64_t row) {
  switch (s->dtype) {
    case TB_I32: return (double)((const int32_t*)s->ptr)[row];
    case TB_F32: return (double)((const float*)s->ptr)[row];
    default: return ((const double*)s->ptr)[row];
  }
}

static int64_t get_i(const src_t* s, int64_t row) {
  switch (s->dtype) {
    case TB_I32: return (int64_t)((const int32_t*)s->ptr)[row];
    case TB_F32: return (int64_t)((const float*)s->ptr)[row];
    default: return (int64_t)((const double*)s->ptr)[row];
  }
}

/* ------------------------------------------------------------------------ */
/* per-edge index: rows of relation r grouped by the attributes it shares    */
/* with its parent (mixed-radix key over their domains)                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n_key;
  int key_attr[8];
  src_t key_src_self[8];        /* the key columns in this relation */
  int64_t key_dom[8];
  int dense;                    /* offsets over the whole key space */
  int64_t space;
  int64_t* off;                 /* dense: [space + 1] */
  int64_t* keys;                /* sparse: sorted distinct keys */
  int64_t* koff;                /* sparse: [n_keys + 1] */
  int64_t n_keys;
  int64_t* rows;                /* row ids ordered by key */
  /* attributes of this relation already bound by earlier relations, other
   * than the key: checked per candidate row */
  int n_extra;
  src_t extra_self[16];
  int extra_attr[16];
} index_t;

typedef struct {
  int64_t k;
  int64_t r;
} kr_t;

static int cmp_kr(const void* a, const void* b) {
  const kr_t* x = (const kr_t*)a;
  const kr_t* y = (const kr_t*)b;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  return x->r < y->r ? -1 : (x->r > y->r);
}

static int64_t row_key(const index_t* ix, const src_t* srcs, int64_t row) {
  int64_t k = 0;
  for (int i = 0; i < ix->n_key; ++i) k = k * ix->key_dom[i] + get_i(&srcs[i], row);
  return k;
}

/* ------------------------------------------------------------------------ */
/* accumulators                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s, c, a;   /* Neumaier sum, compensation, sum of |term| */
} acc_t;

static inline void acc_add(acc_t* x, double t) {
  const double y = x->s + t;
  if (fabs(x->s) >= fabs(t)) x->c += (x->s - y) + t;
  else x->c += (t - y) + x->s;
  x->s = y;
  x->a += fabs(t);
}

static inline void acc_merge(acc_t* x, const acc_t* o) {
  acc_add(x, o->s);
  x->a -= fabs(o->s);
  acc_add(x, o->c);
  x->a -= fabs(o->c);
  x->a += o->a;
}

/* open-addressing map: cell -> slot in parallel arrays */
typedef struct {
  int64_t cap, n;
  int64_t* key;     /* -1 empty */
  int64_t* cnt;
  acc_t* acc;       /* [cap x n_aggs] */
  int n_aggs;
} map_t;

static void map_init(map_t* m, int n_aggs, int64_t cap) {
  m->cap = cap;
  m->n = 0;
  m->n_aggs = n_aggs;
  m->key = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
  m->cnt = (int64_t*)calloc((size_t)cap, sizeof(int64_t));
  m->acc = (acc_t*)calloc((size_t)cap * (n_aggs ? n_aggs : 1), sizeof(acc_t));
  for (int64_t i = 0; i < cap; ++i) m->key[i] = -1;
}

static inline uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static int64_t map_slot(map_t* m, int64_t k);

static void map_grow(map_t* m) {
  map_t n;
  map_init(&n, m->n_aggs, m->cap * 2);
  for (int64_t i = 0; i < m->cap; ++i) {
    if (m->key[i] < 0) continue;
    int64_t j = map_slot(&n, m->key[i]);
    n.cnt[j] = m->cnt[i];
    memcpy(&n.acc[j * (n.n_aggs ? n.n_aggs : 1)], &m->acc[i * (m->n_aggs ? m->n_aggs : 1)],
           sizeof(acc_t) * (m->n_aggs ? m->n_aggs : 1));
  }
  free(m->key);
  free(m->cnt);
  free(m->acc);
  *m = n;
}

static int64_t map_slot(map_t* m, int64_t k) {
  if (2 * (m->n + 1) > m->cap) map_grow(m);
  int64_t i = (int64_t)(mix64((uint64_t)k) & (uint64_t)(m->cap - 1));
  while (m->key[i] >= 0 && m->key[i] != k) i = (i + 1) & (m->cap - 1);
  if (m->key[i] < 0) {
    m->key[i] = k;
    m->n++;
  }
  return i;
}

/* ------------------------------------------------------------------------ */
/* query evaluation state                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n_gb;
  int gb[8];
  int64_t gb_dom[8];
  int64_t cells;          /* product of group-by domains (1 without group-by) */
  int n_cond;
  int cond[64];           /* indices into the distinct condition list */
  int n_aggs;
  int agg_nf[512];
  int agg_fa[512][4];     /* factor attributes, a power-2 factor repeated */
  int big;                /* owned by one thread (many groups) */
  int use_map;
} query_t;

typedef struct {
  int attr, op;
  double c;       /* in the column's comparison type */
} cond_t;

typedef struct {
  const tb_problem* P;
  int n_rels;
  src_t* attr_src;        /* [n_attrs] first relation (BFS order) holding it */
  index_t* ix;            /* [n_rels] (ix[0] unused) */
  int* used_attrs;
  int n_used;
  cond_t* conds;
  int n_conds;
  query_t* q;
  int nq;
} ctx_t;

/* per-thread enumeration scratch */
typedef struct {
  int64_t rows[64];
  double* val;            /* [n_attrs] */
  int64_t* ival;          /* [n_attrs] */
  uint8_t* cond_ok;       /* [n_conds] */
  const int* bind;        /* attributes the sink reads */
  int n_bind;
  const int* bind_cond;   /* conditions the sink reads */
  int n_bind_cond;
} tup_t;

typedef void (*sink_fn)(const ctx_t* C, tup_t* T, void* arg);

static void bind_values(const ctx_t* C, tup_t* T) {
  for (int u = 0; u < T->n_bind; ++u) {
    const int a = T->bind[u];
    const src_t* s = &C->attr_src[a];
    const int64_t row = T->rows[s->rel];
    T->val[a] = get_f(s, row);
    T->ival[a] = get_i(s, row);
  }
  for (int kk = 0; kk < T->n_bind_cond; ++kk) {
    const int k = T->bind_cond[kk];
    const cond_t* c = &C->conds[k];
    const src_t* s = &C->attr_src[c->attr];
    const int64_t row = T->rows[s->rel];
    int ok;
    if (s->dtype == TB_F32) {
      const float x = ((const float*)s->ptr)[row];
      const float y = (float)c->c;
      switch (c->op) {
        case TB_LE: ok = x <= y; break;
        case TB_LT: ok = x < y; break;
        case TB_GT: ok = x > y; break;
        case TB_GE: ok = x >= y; break;
        case TB_EQ: ok = x == y; break;
        default: ok = x != y; break;
      }
    } else {
      const double x = get_f(s, row);
      const double y = c->c;
      switch (c->op) {
        case TB_LE: ok = x <= y; break;
        case TB_LT: ok = x < y; break;
        case TB_GT: ok = x > y; break;
        case TB_GE: ok = x >= y; break;
        case TB_EQ: ok = x == y; break;
        default: ok = x != y; break;
      }
    }
    T->cond_ok[k] = (uint8_t)ok;
  }
}

/* depth-first enumeration of the tuples of D that extend rows[0..level) */
static void enumerate(const ctx_t* C, tup_t* T, int level, sink_fn sink, void* arg) {
  if (level == C->n_rels) {
    bind_values(C, T);
    sink(C, T, arg);
    return;
  }
  const index_t* ix = &C->ix[level];
  const int p = C->P->parent[level];
  /* key from the parent's row */
  int64_t k = 0;
  for (int i = 0; i < ix->n_key; ++i) {
    const src_t* ps = &C->attr_src[ix->key_attr[i]];
    /* the key attribute is bound by the parent or an earlier relation */
    const int64_t v = get_i(ps, T->rows[ps->rel]);
    if (v < 0 || v >= ix->key_dom[i]) return;
    k = k * ix->key_dom[i] + v;
  }
  (void)p;
  int64_t b, e;
  if (ix->dense) {
    b = ix->off[k];
    e = ix->off[k + 1];
  } else {
    int64_t lo = 0, hi = ix->n_keys;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (ix->keys[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    if (lo == ix->n_keys || ix->keys[lo] != k) return;
    b = ix->koff[lo];
    e = ix->koff[lo + 1];
  }
  for (int64_t j = b; j < e; ++j) {
    const int64_t r = ix->rows[j];
    int ok = 1;
    for (int x = 0; x < ix->n_extra && ok; ++x) {
      const src_t* es = &C->attr_src[ix->extra_attr[x]];
      ok = get_f(&ix->extra_self[x], r) == get_f(es, T->rows[es->rel]);
    }
    if (!ok) continue;
    T->rows[level] = r;
    enumerate(C, T, level + 1, sink, arg);
  }
}

static inline int query_pass(const query_t* q, const tup_t* T) {
  for (int k = 0; k < q->n_cond; ++k)
    if (!T->cond_ok[q->cond[k]]) return 0;
  return 1;
}

static inline int64_t query_cell(const query_t* q, const tup_t* T) {
  int64_t cell = 0;
  for (int i = 0; i < q->n_gb; ++i) cell = cell * q->gb_dom[i] + T->ival[q->gb[i]];
  return cell;
}

static inline double agg_term(const query_t* q, int k, const tup_t* T) {
  double t = 1.0;
  for (int f = 0; f < q->agg_nf[k]; ++f) t *= T->val[q->agg_fa[k][f]];
  return t;
}

/* small queries: every thread keeps dense accumulators for all of them */
typedef struct {
  int64_t** cnt;    /* [nq] -> [cells] (NULL for big queries) */
  acc_t** acc;      /* [nq] -> [cells x n_aggs] */
} dense_set_t;

static void sink_small(const ctx_t* C, tup_t* T, void* arg) {
  dense_set_t* D = (dense_set_t*)arg;
  for (int qi = 0; qi < C->nq; ++qi) {
    const query_t* q = &C->q[qi];
    if (q->big || !query_pass(q, T)) continue;
    const int64_t cell = query_cell(q, T);
    if (cell < 0 || cell >= q->cells) continue;
    D->cnt[qi][cell]++;
    acc_t* a = &D->acc[qi][cell * q->n_aggs];
    for (int k = 0; k < q->n_aggs; ++k) acc_add(&a[k], agg_term(q, k, T));
  }
}

typedef struct {
  int qi;
  int64_t* cnt;
  acc_t* acc;
  map_t map;
} big_t;

static void sink_big(const ctx_t* C, tup_t* T, void* arg) {
  big_t* B = (big_t*)arg;
  const query_t* q = &C->q[B->qi];
  if (!query_pass(q, T)) return;
  const int64_t cell = query_cell(q, T);
  if (cell < 0 || cell >= q->cells) return;
  acc_t* a;
  if (q->use_map) {
    const int64_t s = map_slot(&B->map, cell);
    B->map.cnt[s]++;
    a = &B->map.acc[s * (q->n_aggs ? q->n_aggs : 1)];
  } else {
    B->cnt[cell]++;
    a = &B->acc[cell * q->n_aggs];
  }
  for (int k = 0; k < q->n_aggs; ++k) acc_add(&a[k], agg_term(q, k, T));
}

/* ------------------------------------------------------------------------ */
/* results                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int64_t* cell;
  int64_t* cnt;
  double* sum;
  double* abs;
} res_t;

typedef struct {
  int nq;
  int n_aggs_max;
  res_t* r;
  int* n_aggs;
  double seconds, index_seconds;
  int threads;
} tb_result;

static void res_from_dense(res_t* R, const int64_t* cnt, const acc_t* acc, int64_t cells, int n_aggs) {
  int64_t n = 0;
  for (int64_t i = 0; i < cells; ++i) n += cnt[i] > 0;
  R->n = n;
  R->cell = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  R->cnt = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  R->sum = (double*)malloc(sizeof(double) * ((n * n_aggs) > 0 ? n * n_aggs : 1));
  R->abs = (double*)malloc(sizeof(double) * ((n * n_aggs) > 0 ? n * n_aggs : 1));
  int64_t g = 0;
  for (int64_t i = 0; i < cells; ++i) {
    if (cnt[i] <= 0) continue;
    R->cell[g] = i;
    R->cnt[g] = cnt[i];
    for (int k = 0; k < n_aggs; ++k) {
      R->sum[g * n_aggs + k] = acc[i * n_aggs + k].s + acc[i * n_aggs + k].c;
      R->abs[g * n_aggs + k] = acc[i * n_aggs + k].a;
    }
    ++g;
  }
}


static void res_from_map(res_t* R, const map_t* m, int n_aggs) {
  int64_t n = 0;
  kr_t* order = (kr_t*)malloc(sizeof(kr_t) * (m->n ? m->n : 1));
  for (int64_t i = 0; i < m->cap; ++i)
    if (m->key[i] >= 0 && m->cnt[i] > 0) {
      order[n].k = m->key[i];
      order[n].r = i;
      ++n;
    }
  qsort(order, (size_t)n, sizeof(kr_t), cmp_kr);
  R->n = n;
  R->cell = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  R->cnt = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  R->sum = (double*)malloc(sizeof(double) * ((n * n_aggs) > 0 ? n * n_aggs : 1));
  R->abs = (double*)malloc(sizeof(double) * ((n * n_aggs) > 0 ? n * n_aggs : 1));
  const int stride = n_aggs ? n_aggs : 1;
  for (int64_t g = 0; g < n; ++g) {
    const int64_t i = order[g].r;
    R->cell[g] = order[g].k;
    R->cnt[g] = m->cnt[i];
    for (int k = 0; k < n_aggs; ++k) {
      R->sum[g * n_aggs + k] = m->acc[i * stride + k].s + m->acc[i * stride + k].c;
      R->abs[g * n_aggs + k] = m->acc[i * stride + k].a;
    }
  }
  free(order);
}

/* ------------------------------------------------------------------------ */
/* entry points                                                              */
/* ------------------------------------------------------------------------ */
static double now_s(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* Queries whose key space has at most this many cells are accumulated per
 * thread (dense) and merged; larger ones are owned by one thread. */
#define TB_SMALL_CELLS 16384
/* A thread-owned query keeps a dense array up to this many cells. */
#define TB_DENSE_CELLS (1LL << 24)

void* tb_run(const tb_problem* P, int n_threads, int64_t root_rows) {
  const double t0 = now_s();
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  ctx_t C;
  memset(&C, 0, sizeof C);
  C.P = P;
  C.n_rels = P->n_rels;
  if (C.n_rels > 64) return NULL;
  C.attr_src = (src_t*)calloc((size_t)P->n_attrs, sizeof(src_t));
  int* bound_by = (int*)malloc(sizeof(int) * P->n_attrs);
  for (int a = 0; a < P->n_attrs; ++a) bound_by[a] = -1;
  C.ix = (index_t*)calloc((size_t)C.n_rels, sizeof(index_t));
  const int64_t n_root = (root_rows >= 0 && root_rows < P->n_rows[0]) ? root_rows : P->n_rows[0];
  for (int r = 0; r < C.n_rels; ++r) {
    index_t* ix = &C.ix[r];
    for (int c = P->col_off[r]; c < P->col_off[r + 1]; ++c) {
      const int a = P->col_attr[c];
      src_t self = {r, P->col_ptr[c], P->col_dtype[c]};
      if (bound_by[a] < 0) {
        bound_by[a] = r;
        C.attr_src[a] = self;
        continue;
      }
      if (r == 0) continue;
      /* shared with an earlier relation: part of the key if the parent holds
       * it, else a value checked per candidate row */
      int in_parent = 0;
      const int p = P->parent[r];
      for (int pc = P->col_off[p]; pc < P->col_off[p + 1]; ++pc) in_parent |= P->col_attr[pc] == a;
      if (in_parent && ix->n_key < 8) {
        ix->key_attr[ix->n_key] = a;
        ix->key_src_self[ix->n_key] = self;
        ix->key_dom[ix->n_key] = P->attr_dom[a] > 0 ? P->attr_dom[a] : 1;
        ix->n_key++;
      } else if (ix->n_extra < 16) {
        ix->extra_attr[ix->n_extra] = a;
        ix->extra_self[ix->n_extra] = self;
        ix->n_extra++;
      }
    }
  }
  /* indexes */
  for (int r = 1; r < C.n_rels; ++r) {
    index_t* ix = &C.ix[r];
    const int64_t n = P->n_rows[r];
    ix->space = 1;
    for (int i = 0; i < ix->n_key; ++i) ix->space *= ix->key_dom[i];
    kr_t* kr = (kr_t*)malloc(sizeof(kr_t) * (n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
      kr[i].k = row_key(ix, ix->key_src_self, i);
      kr[i].r = i;
    }
    qsort(kr, (size_t)n, sizeof(kr_t), cmp_kr);
    ix->rows = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
    for (int64_t i = 0; i < n; ++i) ix->rows[i] = kr[i].r;
    ix->dense = ix->space <= ((int64_t)1 << 28);
    if (ix->dense) {
      ix->off = (int64_t*)calloc((size_t)ix->space + 1, sizeof(int64_t));
      for (int64_t i = 0; i < n; ++i) ix->off[kr[i].k + 1]++;
      for (int64_t k = 0; k < ix->space; ++k) ix->off[k + 1] += ix->off[k];
    } else {
      int64_t nk = 0;
      for (int64_t i = 0; i < n; ++i) nk += (i == 0 || kr[i].k != kr[i - 1].k);
      ix->n_keys = nk;
      ix->keys = (int64_t*)malloc(sizeof(int64_t) * (nk ? nk : 1));
      ix->koff = (int64_t*)malloc(sizeof(int64_t) * (nk + 1));
      int64_t g = -1;
      for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || kr[i].k != kr[i - 1].k) {
          ++g;
          ix->keys[g] = kr[i].k;
          ix->koff[g] = i;
        }
      }
      ix->koff[nk] = n;
    }
    free(kr);
  }
  const double t_index = now_s() - t0;
  /* distinct conditions and queries */
  int total_conds = P->cond_off[P->n_queries];
  C.conds = (cond_t*)malloc(sizeof(cond_t) * (total_conds ? total_conds : 1));
  C.q = (query_t*)calloc((size_t)P->n_queries, sizeof(query_t));
  C.nq = P->n_queries;
  char* used = (char*)calloc((size_t)P->n_attrs, 1);
  for (int qi = 0; qi < P->n_queries; ++qi) {
    query_t* q = &C.q[qi];
    q->n_gb = P->gb_off[qi + 1] - P->gb_off[qi];
    if (q->n_gb > 8 || P->cond_off[qi + 1] - P->cond_off[qi] > 64 || P->agg_off[qi + 1] - P->agg_off[qi] > 512)
      return NULL;
    q->cells = 1;
    for (int i = 0; i < q->n_gb; ++i) {
      q->gb[i] = P->gb_attr[P->gb_off[qi] + i];
      q->gb_dom[i] = P->attr_dom[q->gb[i]] > 0 ? P->attr_dom[q->gb[i]] : 1;
      q->cells *= q->gb_dom[i];
      used[q->gb[i]] = 1;
    }
    q->n_cond = 0;
    for (int k = P->cond_off[qi]; k < P->cond_off[qi + 1]; ++k) {
      cond_t c = {P->cond_attr[k], P->cond_op[k], P->cond_c[k]};
      int j = 0;
      for (; j < C.n_conds; ++j)
        if (C.conds[j].attr == c.attr && C.conds[j].op == c.op && C.conds[j].c == c.c) break;
      if (j == C.n_conds) C.conds[C.n_conds++] = c;
      q->cond[q->n_cond++] = j;
    }
    q->n_aggs = P->agg_off[qi + 1] - P->agg_off[qi];
    for (int k = 0; k < q->n_aggs; ++k) {
      const int ag = P->agg_off[qi] + k;
      int nf = 0;
      for (int f = P->agg_f_off[ag]; f < P->agg_f_off[ag + 1]; ++f)
        for (int pw = 0; pw < P->f_pow[f] && nf < 4; ++pw) {
          q->agg_fa[k][nf++] = P->f_attr[f];
          used[P->f_attr[f]] = 1;
        }
      q->agg_nf[k] = nf;
    }
    q->big = q->cells > TB_SMALL_CELLS;
    q->use_map = q->cells > TB_DENSE_CELLS;
  }
  C.used_attrs = (int*)malloc(sizeof(int) * P->n_attrs);
  for (int a = 0; a < P->n_attrs; ++a)
    if (used[a] && bound_by[a] >= 0) C.used_attrs[C.n_used++] = a;
  free(used);

  tb_result* out = (tb_result*)calloc(1, sizeof(tb_result));
  out->nq = C.nq;
  out->r = (res_t*)calloc((size_t)C.nq, sizeof(res_t));
  out->n_aggs = (int*)malloc(sizeof(int) * (C.nq ? C.nq : 1));
  for (int qi = 0; qi < C.nq; ++qi) out->n_aggs[qi] = C.q[qi].n_aggs;

  int* all_conds = (int*)malloc(sizeof(int) * (C.n_conds ? C.n_conds : 1));
  for (int k = 0; k < C.n_conds; ++k) all_conds[k] = k;
  /* phase 1: small queries, row ranges of relation 0 per thread */
  int any_small = 0;
  for (int qi = 0; qi < C.nq; ++qi) any_small |= !C.q[qi].big;
  dense_set_t* parts = (dense_set_t*)calloc((size_t)n_threads, sizeof(dense_set_t));
  if (any_small) {
#pragma omp parallel num_threads(n_threads)
    {
      const int t = omp_get_thread_num();
      dense_set_t* D = &parts[t];
      D->cnt = (int64_t**)calloc((size_t)C.nq, sizeof(int64_t*));
      D->acc = (acc_t**)calloc((size_t)C.nq, sizeof(acc_t*));
      for (int qi = 0; qi < C.nq; ++qi) {
        if (C.q[qi].big) continue;
        D->cnt[qi] = (int64_t*)calloc((size_t)C.q[qi].cells, sizeof(int64_t));
        D->acc[qi] = (acc_t*)calloc((size_t)(C.q[qi].cells * (C.q[qi].n_aggs ? C.q[qi].n_aggs : 1)), sizeof(acc_t));
      }
      tup_t T;
      T.val = (double*)calloc((size_t)P->n_attrs, sizeof(double));
      T.ival = (int64_t*)calloc((size_t)P->n_attrs, sizeof(int64_t));
      T.cond_ok = (uint8_t*)calloc((size_t)(C.n_conds ? C.n_conds : 1), 1);
      T.bind = C.used_attrs;
      T.n_bind = C.n_used;
      T.bind_cond = all_conds;
      T.n_bind_cond = C.n_conds;
#pragma omp for schedule(dynamic, 4096)
      for (int64_t row = 0; row < n_root; ++row) {
        T.rows[0] = row;
        enumerate(&C, &T, 1, sink_small, D);
      }
      free(T.val);
      free(T.ival);
      free(T.cond_ok);
    }
    /* merge in thread order */
    for (int qi = 0; qi < C.nq; ++qi) {
      const query_t* q = &C.q[qi];
      if (q->big) continue;
      const int na = q->n_aggs ? q->n_aggs : 1;
      for (int t = 1; t < n_threads; ++t) {
        for (int64_t i = 0; i < q->cells; ++i) parts[0].cnt[qi][i] += parts[t].cnt[qi][i];
        for (int64_t i = 0; i < q->cells * q->n_aggs; ++i) acc_merge(&parts[0].acc[qi][i], &parts[t].acc[qi][i]);
      }
      (void)na;
      res_from_dense(&out->r[qi], parts[0].cnt[qi], parts[0].acc[qi], q->cells, q->n_aggs);
    }
    for (int t = 0; t < n_threads; ++t) {
      for (int qi = 0; qi < C.nq; ++qi) {
        free(parts[t].cnt[qi]);
        free(parts[t].acc[qi]);
      }
      free(parts[t].cnt);
      free(parts[t].acc);
    }
  }
  free(parts);

  /* phase 2: big queries, one thread each over all of D */
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
  for (int qi = 0; qi < C.nq; ++qi) {
    const query_t* q = &C.q[qi];
    if (!q->big) continue;
    big_t B;
    memset(&B, 0, sizeof B);
    B.qi = qi;
    if (q->use_map) {
      map_init(&B.map, q->n_aggs, 1 << 16);
    } else {
      B.cnt = (int64_t*)calloc((size_t)q->cells, sizeof(int64_t));
      B.acc = (acc_t*)calloc((size_t)(q->cells * (q->n_aggs ? q->n_aggs : 1)), sizeof(acc_t));
    }
    tup_t T;
    T.val = (double*)calloc((size_t)P->n_attrs, sizeof(double));
    T.ival = (int64_t*)calloc((size_t)P->n_attrs, sizeof(int64_t));
    T.cond_ok = (uint8_t*)calloc((size_t)(C.n_conds ? C.n_conds : 1), 1);
    int qattr[8 + 512 * 4], nqa = 0;
    for (int i = 0; i < q->n_gb; ++i) qattr[nqa++] = q->gb[i];
    for (int k = 0; k < q->n_aggs; ++k)
      for (int f = 0; f < q->agg_nf[k]; ++f) qattr[nqa++] = q->agg_fa[k][f];
    T.bind = qattr;
    T.n_bind = nqa;
    T.bind_cond = q->cond;
    T.n_bind_cond = q->n_cond;
    for (int64_t row = 0; row < n_root; ++row) {
      T.rows[0] = row;
      enumerate(&C, &T, 1, sink_big, &B);
    }
    if (q->use_map) {
      res_from_map(&out->r[qi], &B.map, q->n_aggs);
      free(B.map.key);
      free(B.map.cnt);
      free(B.map.acc);
    } else {
      res_from_dense(&out->r[qi], B.cnt, B.acc, q->cells, q->n_aggs);
      free(B.cnt);
      free(B.acc);
    }
    free(T.val);
    free(T.ival);
    free(T.cond_ok);
  }

  for (int r = 0; r < C.n_rels; ++r) {
    free(C.ix[r].off);
    free(C.ix[r].keys);
    free(C.ix[r].koff);
    free(C.ix[r].rows);
  }
  free(C.ix);
  free(C.attr_src);
  free(C.conds);
  free(C.q);
  free(C.used_attrs);
  free(all_conds);
  free(bound_by);
  out->seconds = now_s() - t0;
  out->index_seconds = t_index;
  out->threads = n_threads;
  return out;
}

int64_t tb_groups(const void* h, int q) { return ((const tb_result*)h)->r[q].n; }
double tb_seconds(const void* h) { return ((const tb_result*)h)->seconds; }
double tb_index_seconds(const void* h) { return ((const tb_result*)h)->index_seconds; }
int tb_threads(const void* h) { return ((const tb_result*)h)->threads; }

/* copies query q's result: cells (mixed-radix group key, last attribute
 * fastest, ascending = lexicographic), counts, sums and sums of |term| */
void tb_copy(const void* h, int q, int64_t* cell, int64_t* cnt, double* sum, double* abs_) {
  const tb_result* R = (const tb_result*)h;
  const res_t* r = &R->r[q];
  const int na = R->n_aggs[q];
  memcpy(cell, r->cell, sizeof(int64_t) * r->n);
  memcpy(cnt, r->cnt, sizeof(int64_t) * r->n);
  memcpy(sum, r->sum, sizeof(double) * r->n * na);
  memcpy(abs_, r->abs, sizeof(double) * r->n * na);
}

void tb_free(void* h) {
  tb_result* R = (tb_result*)h;
  if (!R) return;
  for (int q = 0; q < R->nq; ++q) {
    free(R->r[q].cell);
    free(R->r[q].cnt);
    free(R->r[q].sum);
    free(R->r[q].abs);
  }
  free(R->r);
  free(R->n_aggs);
  free(R);
}
