// Host planner: the view generation and multi-output optimization layers of
// the paper (section 2, Figure 1), followed by this engine's physical
// planning of each group into a factorized scan + contraction program.
//
//  1. validate schema / join tree / batch;
//  2. assign a root to every query (section 2: one root per query, chosen by a
//     heuristic; two heuristics here, see lmfao.h);
//  3. decompose every query top-down from its root into one view per edge
//     (section 2: the view on an edge leaving node n is the query restricted
//     to the attributes of the subtree rooted at n, over the join of n's
//     relation and its incoming views; group-by attributes of the subtree are
//     carried along);
//  4. merge views with the same direction, group-by attributes and condition;
//  5. group the views and queries leaving the same node by dependency level
//     (this reproduces the seven groups and the dependency graph of Figure 2);
//  6. pick a total attribute order per node and compile each group into the
//     program the GPU runs: per-tuple inner factors and codes, per-piece
//     partial sums (the running sums of Figure 3), per-piece outer features
//     and the contraction that multiplies them (the partial aggregates of
//     Figure 3 pushed past the inner loops).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <iterator>
#include <tuple>
#include <cstring>
#include <functional>
#include <iomanip>
#include <numeric>
#include <queue>
#include <sstream>

#include "engine.hpp"

namespace lmfao {

static void fail(int st, const std::string& m) { throw PlanError{st, m}; }

std::vector<int> join_attrs(const Plan& P, int a, int b) {
  std::vector<int> out;
  for (int x : P.rels[a].attrs)
    if (P.rels[b].has(x)) out.push_back(x);
  std::sort(out.begin(), out.end());
  return out;
}

static std::string mono_str(const Plan& P, const Mono& m) {
  if (m.empty()) return "1";
  std::string s;
  for (size_t i = 0; i < m.size(); ++i) {
    if (i) s += "*";
    s += P.attrs[m[i]].name;
  }
  return s;
}

static std::string json_escape(const std::string& s) {
  std::string o;
  for (char c : s) {
    if (c == '"' || c == '\\') o += '\\';
    o += c;
  }
  return o;
}

// ---------------------------------------------------------------------------
// 1. validation and intake
// ---------------------------------------------------------------------------
static void rewrite_conditions(Plan& P);

static void intake(Plan& P, const lmfao_schema* schema, const lmfao_join_tree* tree,
                   const lmfao_batch* batch) {
  if (!schema || schema->n_relations <= 0 || !schema->relations) fail(LMFAO_EINVAL, "empty schema");
  int n = schema->n_relations;
  if (n > 31) fail(LMFAO_EUNSUPPORTED, "more than 31 relations");
  P.rels.resize(n);
  for (int r = 0; r < n; ++r) {
    const lmfao_relation& R = schema->relations[r];
    RelDef& D = P.rels[r];
    D.name = R.name ? R.name : ("R" + std::to_string(r));
    if (R.n_rows < 0) fail(LMFAO_EINVAL, "negative row count for " + D.name);
    D.n_rows = R.n_rows;
    if (R.n_attrs <= 0 || !R.attrs) fail(LMFAO_EINVAL, "relation " + D.name + " has no attributes");
    for (int a = 0; a < R.n_attrs; ++a) {
      const lmfao_attr& A = R.attrs[a];
      if (!A.name || !*A.name) fail(LMFAO_EINVAL, "unnamed attribute in " + D.name);
      if (A.dtype < LMFAO_I32 || A.dtype > LMFAO_F64) fail(LMFAO_EINVAL, std::string("bad dtype for ") + A.name);
      int id;
      auto it = P.attr_id.find(A.name);
      if (it == P.attr_id.end()) {
        id = (int)P.attrs.size();
        P.attr_id[A.name] = id;
        P.attrs.push_back(AttrDef{A.name, A.dtype, A.domain});
      } else {
        id = it->second;
        AttrDef& G = P.attrs[id];
        if (G.dtype != A.dtype)
          fail(LMFAO_EINVAL, std::string("attribute ") + A.name + " has different dtypes across relations");
        G.domain = std::max(G.domain, A.domain);
      }
      if (D.has(id)) fail(LMFAO_EINVAL, std::string("duplicate attribute ") + A.name + " in " + D.name);
      D.col[id] = (int)D.attrs.size();
      D.attrs.push_back(id);
      D.dtypes.push_back(A.dtype);
      D.is_key.push_back(A.is_key ? 1 : 0);
    }
    D.n_input_attrs = (int)D.attrs.size();
  }
  // join tree
  P.adj.assign(n, {});
  int ne = tree ? tree->n_edges : 0;
  if (ne != n - 1) fail(LMFAO_EINVAL, "join tree must have n_relations-1 edges");
  for (int e = 0; e < ne; ++e) {
    int a = tree->edges[e].a, b = tree->edges[e].b;
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) fail(LMFAO_EINVAL, "bad join tree edge");
    P.edges.push_back({a, b});
    P.adj[a].push_back(b);
    P.adj[b].push_back(a);
  }
  for (auto& v : P.adj) std::sort(v.begin(), v.end());
  {  // connected (n-1 edges + connected => tree)
    std::vector<char> seen(n, 0);
    std::vector<int> st{0};
    seen[0] = 1;
    while (!st.empty()) {
      int u = st.back();
      st.pop_back();
      for (int v : P.adj[u])
        if (!seen[v]) { seen[v] = 1; st.push_back(v); }
    }
    for (int r = 0; r < n; ++r)
      if (!seen[r]) fail(LMFAO_EINVAL, "join tree does not connect relation " + P.rels[r].name);
  }
  for (auto& e : P.edges)
    if (join_attrs(P, e.first, e.second).empty())
      fail(LMFAO_EINVAL, "join tree edge " + P.rels[e.first].name + "-" + P.rels[e.second].name +
                             " shares no attribute");
  // running intersection: relations holding an attribute are connected
  for (int a = 0; a < (int)P.attrs.size(); ++a) {
    std::vector<int> holders;
    for (int r = 0; r < n; ++r)
      if (P.rels[r].has(a)) holders.push_back(r);
    if (holders.size() < 2) continue;
    std::vector<char> seen(n, 0);
    std::vector<int> st{holders[0]};
    seen[holders[0]] = 1;
    while (!st.empty()) {
      int u = st.back();
      st.pop_back();
      for (int v : P.adj[u])
        if (!seen[v] && P.rels[v].has(a)) { seen[v] = 1; st.push_back(v); }
    }
    for (int h : holders)
      if (!seen[h])
        fail(LMFAO_EINVAL, "attribute " + P.attrs[a].name + " violates the running-intersection property");
    if (P.attrs[a].dtype != LMFAO_I32 || P.attrs[a].domain <= 0)
      fail(LMFAO_EUNSUPPORTED, "join attribute " + P.attrs[a].name + " needs an integer domain");
  }
  // user-defined factors: an FP64 column of the smallest relation holding
  // the argument, gathered from the function's table at prepare time
  if (batch && batch->n_functions < 0) fail(LMFAO_EINVAL, "negative function count");
  for (int fi = 0; batch && fi < batch->n_functions; ++fi) {
    const lmfao_function& F = batch->functions[fi];
    if (!F.name || !*F.name || !F.attr) fail(LMFAO_EINVAL, "unnamed function or argument");
    if (P.attr_id.count(F.name)) fail(LMFAO_EINVAL, std::string("function name ") + F.name + " is taken");
    auto it = P.attr_id.find(F.attr);
    if (it == P.attr_id.end()) fail(LMFAO_EINVAL, std::string("unknown function argument ") + F.attr);
    const AttrDef& A = P.attrs[it->second];
    if (A.dtype != LMFAO_I32 || A.domain <= 0 || F.n_values != A.domain || !F.values)
      fail(LMFAO_EINVAL, std::string("function ") + F.name + ": needs one value per value of an integer attribute");
    DerivedAttr D;
    D.src = it->second;
    D.kind = 2;
    D.thr.assign(F.values, F.values + F.n_values);
    for (size_t r = 0; r < P.rels.size(); ++r)
      if (P.rels[r].has(D.src) && (D.rel < 0 || P.rels[r].n_rows < P.rels[D.rel].n_rows)) D.rel = (int)r;
    D.attr = (int)P.attrs.size();
    P.attr_id[F.name] = D.attr;
    P.attrs.push_back(AttrDef{F.name, LMFAO_F64, 0});
    RelDef& R = P.rels[D.rel];
    R.col[D.attr] = (int)R.attrs.size();
    R.attrs.push_back(D.attr);
    R.dtypes.push_back(LMFAO_F64);
    R.is_key.push_back(0);
    P.derived.push_back(D);
  }
  // batch
  if (!batch || batch->n_queries <= 0) fail(LMFAO_EINVAL, "empty batch");
  for (int qi = 0; qi < batch->n_queries; ++qi) {
    const lmfao_query& Q = batch->queries[qi];
    QueryDef q;
    auto lookup = [&](const char* nm) {
      if (!nm) fail(LMFAO_EINVAL, "null attribute name in query " + std::to_string(qi));
      auto it = P.attr_id.find(nm);
      if (it == P.attr_id.end()) fail(LMFAO_EINVAL, std::string("unknown attribute ") + nm);
      return it->second;
    };
    if (Q.n_groupby < 0 || Q.n_groupby > 2)
      fail(LMFAO_EUNSUPPORTED, "query " + std::to_string(qi) + ": at most 2 group-by attributes");
    for (int g = 0; g < Q.n_groupby; ++g) {
      int a = lookup(Q.groupby[g]);
      if (P.attrs[a].dtype != LMFAO_I32 || P.attrs[a].domain <= 0)
        fail(LMFAO_EUNSUPPORTED, "group-by attribute " + P.attrs[a].name + " needs an integer domain");
      if (std::find(q.groupby.begin(), q.groupby.end(), a) != q.groupby.end())
        fail(LMFAO_EINVAL, "repeated group-by attribute");
      q.groupby.push_back(a);
    }
    for (int c = 0; c < Q.n_conditions; ++c) {
      const lmfao_condition& C = Q.conditions[c];
      if (C.op < LMFAO_LE || C.op > LMFAO_NE) fail(LMFAO_EINVAL, "bad condition operator");
      q.conds.push_back(Cond{lookup(C.attr), C.op, C.constant});
    }
    std::sort(q.conds.begin(), q.conds.end());
    q.conds.erase(std::unique(q.conds.begin(), q.conds.end()), q.conds.end());
    if (Q.n_aggregates <= 0) fail(LMFAO_EINVAL, "query without aggregates");
    for (int k = 0; k < Q.n_aggregates; ++k) {
      const lmfao_aggregate& A = Q.aggregates[k];
      Mono m;
      for (int f = 0; f < A.n_factors; ++f) {
        int a = lookup(A.factors[f].attr);
        int p = A.factors[f].power;
        if (p < 1 || p > 2) fail(LMFAO_EUNSUPPORTED, "factor power must be 1 or 2");
        for (int i = 0; i < p; ++i) m.push_back(a);
      }
      if (m.size() > 2) fail(LMFAO_EUNSUPPORTED, "aggregate of degree > 2");
      std::sort(m.begin(), m.end());
      q.aggs.push_back(m);
    }
    q.root = Q.root;
    if (q.root < -1 || q.root >= n) fail(LMFAO_EINVAL, "bad root override");
    P.queries.push_back(q);
  }
  rewrite_conditions(P);
}

// ---------------------------------------------------------------------------
// conditions.  The conjunction every query of the batch shares becomes one
// filter applied to the relations (a tuple failing it has multiplicity 0).
// A query may carry one more condition on a single attribute -- the split
// candidates of a CART node batch (section 3, decision trees): X op t with a
// threshold, or X = c / X != c on an integer attribute.  Such queries are
// planned as one query grouped by a bucket code of X (or by X itself) whose
// buckets are summed over the range the condition selects, so a batch of many
// thresholds on one attribute is one group-by instead of many filters.
// ---------------------------------------------------------------------------
static double cmp_value(const AttrDef& A, double c) {
  // the comparison happens in the column's type for FP32 columns
  return A.dtype == LMFAO_F32 ? (double)(float)c : c;
}

static void rewrite_conditions(Plan& P) {
  const std::vector<QueryDef> given = P.queries;
  const int nq = (int)given.size();
  std::vector<Cond> common = given[0].conds;
  for (int i = 1; i < nq; ++i) {
    std::vector<Cond> x;
    std::set_intersection(common.begin(), common.end(), given[i].conds.begin(), given[i].conds.end(),
                          std::back_inserter(x));
    common = x;
  }
  for (auto& c : common)
    if (P.attrs[c.attr].dtype == LMFAO_F32) c.c = cmp_value(P.attrs[c.attr], c.c);
  P.filter = common;
  P.queries.clear();
  P.user.assign(nq, UserQuery{});
  // candidate conditions per (attribute, threshold kind)
  struct Cand {
    int q;
    Cond c;
  };
  std::vector<Cand> cands;
  std::map<std::pair<int, int>, std::set<double>> thr;   // (attr, kind) -> thresholds
  for (int i = 0; i < nq; ++i) {
    std::vector<Cond> extra;
    std::set_difference(given[i].conds.begin(), given[i].conds.end(), common.begin(), common.end(),
                        std::back_inserter(extra));
    if (extra.empty()) {
      QueryDef q = given[i];
      q.conds = common;
      P.user[i].internal = (int)P.queries.size();
      P.queries.push_back(q);
      continue;
    }
    if (extra.size() > 1)
      fail(LMFAO_EUNSUPPORTED, "query " + std::to_string(i) +
                                   ": more than one condition beyond those every query of the batch shares");
    const Cond& c = extra[0];
    const AttrDef& A = P.attrs[c.attr];
    if (given[i].groupby.size() > 1)
      fail(LMFAO_EUNSUPPORTED, "query " + std::to_string(i) + ": a condition of its own and 2 group-by attributes");
    if (std::find(given[i].groupby.begin(), given[i].groupby.end(), c.attr) != given[i].groupby.end())
      fail(LMFAO_EUNSUPPORTED, "query " + std::to_string(i) + ": condition on its own group-by attribute");
    if (c.op == LMFAO_EQ || c.op == LMFAO_NE) {
      if (A.dtype != LMFAO_I32 || A.domain <= 0)
        fail(LMFAO_EUNSUPPORTED, "query " + std::to_string(i) + ": = / != needs an integer attribute with a domain");
    } else {
      thr[{c.attr, (c.op == LMFAO_LE || c.op == LMFAO_GT) ? 0 : 1}].insert(cmp_value(A, c.c));
    }
    cands.push_back(Cand{i, c});
  }
  // derived bucket attributes, on the first relation holding the attribute
  std::map<std::pair<int, int>, int> dattr;
  for (auto& kv : thr) {
    DerivedAttr D;
    D.src = kv.first.first;
    D.kind = kv.first.second;
    D.thr.assign(kv.second.begin(), kv.second.end());
    for (size_t r = 0; r < P.rels.size() && D.rel < 0; ++r)
      if (P.rels[r].has(D.src)) D.rel = (int)r;
    std::string name = P.attrs[D.src].name + (D.kind == 0 ? "#le" : "#lt");
    if (P.attr_id.count(name)) fail(LMFAO_EINVAL, "attribute name " + name + " is reserved");
    D.attr = (int)P.attrs.size();
    P.attr_id[name] = D.attr;
    P.attrs.push_back(AttrDef{name, LMFAO_I32, (int64_t)D.thr.size() + 1});
    RelDef& R = P.rels[D.rel];
    R.col[D.attr] = (int)R.attrs.size();
    R.attrs.push_back(D.attr);
    R.dtypes.push_back(LMFAO_I32);
    R.is_key.push_back(0);
    dattr[kv.first] = (int)P.derived.size();
    P.derived.push_back(D);
  }
  // planned queries grouped by the bucket (or code) attribute, shared by
  // every candidate with the same group-by and aggregates
  std::map<std::tuple<std::vector<int>, std::vector<Mono>, int>, int> planned;
  for (auto& cd : cands) {
    const QueryDef& g = given[cd.q];
    const Cond& c = cd.c;
    int key_attr = c.attr;
    int64_t nb = P.attrs[c.attr].domain;
    UserQuery& U = P.user[cd.q];
    U.range = true;
    if (c.op == LMFAO_EQ || c.op == LMFAO_NE) {
      const double v = c.c;
      const bool integral = v == std::floor(v) && v >= 0 && v < (double)nb;
      if (c.op == LMFAO_EQ) {
        U.lo = integral ? (int64_t)v : 0;
        U.hi = integral ? (int64_t)v + 1 : 0;
      } else {
        U.lo = 0;
        U.hi = nb;
        U.ex = integral ? (int64_t)v : -1;
      }
    } else {
      const int kind = (c.op == LMFAO_LE || c.op == LMFAO_GT) ? 0 : 1;
      const DerivedAttr& D = P.derived[dattr.at({c.attr, kind})];
      key_attr = D.attr;
      nb = (int64_t)D.thr.size() + 1;
      const double t = cmp_value(P.attrs[c.attr], c.c);
      const int64_t k = std::lower_bound(D.thr.begin(), D.thr.end(), t) - D.thr.begin();
      // bucket b counts thresholds below (kind 0) or at most (kind 1) the
      // value: x <= t_k (x < t_k) iff b <= k
      const bool below = c.op == LMFAO_LE || c.op == LMFAO_LT;
      U.lo = below ? 0 : k + 1;
      U.hi = below ? k + 1 : nb;
    }
    U.nb = nb;
    std::vector<int> gb = g.groupby;
    gb.push_back(key_attr);
    auto key = std::make_tuple(gb, g.aggs, g.root);
    auto it = planned.find(key);
    if (it == planned.end()) {
      QueryDef q = g;
      q.groupby = gb;
      q.conds = common;
      it = planned.emplace(key, (int)P.queries.size()).first;
      P.queries.push_back(q);
    }
    U.internal = it->second;
  }
}

// ---------------------------------------------------------------------------
// uniqueness of directed edge views: V_{n->p} has at most one subtree join
// tuple per key value iff n's primary key is inside the edge's join
// attributes and every view into n from below is unique as well.
// ---------------------------------------------------------------------------
static void compute_uniqueness(Plan& P) {
  int n = (int)P.rels.size();
  P.uniq.assign(n, std::vector<char>(n, 0));
  std::function<bool(int, int)> uq = [&](int u, int p) -> bool {
    const RelDef& R = P.rels[u];
    bool has_key = false;
    std::vector<int> J = join_attrs(P, u, p);
    for (size_t i = 0; i < R.attrs.size(); ++i) {
      if (!R.is_key[i]) continue;
      has_key = true;
      if (!std::binary_search(J.begin(), J.end(), R.attrs[i])) return false;
    }
    if (!has_key) return false;
    for (int c : P.adj[u])
      if (c != p && !uq(c, u)) return false;
    return true;
  };
  for (auto& e : P.edges) {
    P.uniq[e.first][e.second] = uq(e.first, e.second);
    P.uniq[e.second][e.first] = uq(e.second, e.first);
  }
}

// relations reachable from r in direction away from `par`
static void subtree(const Plan& P, int u, int par, std::vector<int>& out) {
  out.push_back(u);
  for (int v : P.adj[u])
    if (v != par) subtree(P, v, u, out);
}

// owner of an attribute w.r.t. a root: the relation holding it closest to the root
static std::vector<int> owners_from(const Plan& P, int root, std::vector<int>& parent) {
  int n = (int)P.rels.size();
  parent.assign(n, -1);
  std::vector<int> order{root};
  std::vector<char> seen(n, 0);
  seen[root] = 1;
  for (size_t i = 0; i < order.size(); ++i)
    for (int v : P.adj[order[i]])
      if (!seen[v]) { seen[v] = 1; parent[v] = order[i]; order.push_back(v); }
  std::vector<int> owner(P.attrs.size(), -1);
  for (int u : order)
    for (int a : P.rels[u].attrs)
      if (owner[a] < 0) owner[a] = u;
  return owner;
}

// ---------------------------------------------------------------------------
// 2. roots
// ---------------------------------------------------------------------------
static int root_groupby(const Plan& P, const QueryDef& q) {
  int n = (int)P.rels.size();
  int best = -1;
  for (int r = 0; r < n; ++r) {
    bool all = true;
    for (int g : q.groupby) all &= P.rels[r].has(g);
    if (!all) continue;
    if (best < 0 || P.rels[r].n_rows > P.rels[best].n_rows) best = r;
  }
  if (best >= 0) return best;
  // no relation holds all of them: the relation holding the group-by
  // attribute with the largest domain
  int ga = q.groupby[0];
  for (int g : q.groupby)
    if (P.attrs[g].domain > P.attrs[ga].domain) ga = g;
  for (int r = 0; r < n; ++r)
    if (P.rels[r].has(ga) && (best < 0 || P.rels[r].n_rows > P.rels[best].n_rows)) best = r;
  return best;
}

// is attribute a single-valued for every tuple of r (reached through unique views)?
static bool fd_reachable(const Plan& P, int r, int a) {
  if (P.rels[r].has(a)) return true;
  for (int c : P.adj[r]) {
    std::vector<int> sub;
    subtree(P, c, r, sub);
    for (int u : sub)
      if (P.rels[u].has(a)) return P.uniq[c][r] != 0;
  }
  return false;
}

static int root_fact(const Plan& P, const QueryDef& q) {
  int n = (int)P.rels.size();
  std::set<int> attrs(q.groupby.begin(), q.groupby.end());
  for (auto& m : q.aggs) attrs.insert(m.begin(), m.end());
  for (auto& c : q.conds) attrs.insert(c.attr);
  // a query over the attributes of a single relation is rooted there
  if (!attrs.empty()) {
    int best = -1;
    for (int r = 0; r < n; ++r) {
      bool all = true;
      for (int a : attrs) all &= P.rels[r].has(a);
      if (all && (best < 0 || P.rels[r].n_rows < P.rels[best].n_rows)) best = r;
    }
    if (best >= 0) return best;
  }
  int best = -1;
  for (int r = 0; r < n; ++r) {
    bool ok = true;
    for (int g : q.groupby) ok &= fd_reachable(P, r, g);
    if (ok && (best < 0 || P.rels[r].n_rows > P.rels[best].n_rows)) best = r;
  }
  if (best >= 0) return best;
  return root_groupby(P, q);
}

// ---------------------------------------------------------------------------
// 3-5. views, merging, levels, groups
// ---------------------------------------------------------------------------
struct ViewKey {
  int from, to;
  std::vector<int> carried;
  std::vector<Cond> conds;
  bool operator<(const ViewKey& o) const {
    return std::tie(from, to, carried, conds) < std::tie(o.from, o.to, o.carried, o.conds);
  }
};

// The view a query rooted at `root` needs along the edge from node u to its
// parent p (its identity as view generation merges views: direction,
// carried group-by attributes unless the view is single-valued, conditions).
static ViewKey view_key_of(const Plan& P, const QueryDef& q, const std::vector<int>& owner, int u, int p,
                           const std::set<int>& subset, std::vector<int>* carried_out = nullptr) {
  auto owned = [&](int a) { return subset.count(owner[a]) != 0; };
  ViewKey k{u, p, {}, {}};
  std::vector<int> carried;
  for (int g : q.groupby)
    if (owned(g)) carried.push_back(g);
  std::sort(carried.begin(), carried.end());
  if (!P.uniq[u][p]) k.carried = carried;
  for (auto& c : q.conds)
    if (owned(c.attr)) k.conds.push_back(c);
  if (carried_out) *carried_out = carried;
  return k;
}

// Root cost model: the bytes a root assignment makes the fused plan move --
// one pass over every node that computes a view or a query (rows x 16 B) and,
// per distinct view (views are merged across queries as view generation
// merges them), its dense key space written once (cells x 8 B).
static double root_assignment_cost(const Plan& P, const std::vector<int>& roots) {
  const int n = (int)P.rels.size();
  std::set<ViewKey> views;
  std::vector<char> active(n, 0);
  double out = 0;
  for (size_t qi = 0; qi < P.queries.size(); ++qi) {
    const QueryDef& q = P.queries[qi];
    const int root = roots[qi];
    active[root] = 1;
    std::vector<int> parent;
    std::vector<int> owner = owners_from(P, root, parent);
    for (int u = 0; u < n; ++u) {
      if (u == root) continue;
      std::vector<int> sub;
      subtree(P, u, parent[u], sub);
      std::set<int> subset(sub.begin(), sub.end());
      std::vector<int> carried;
      ViewKey k = view_key_of(P, q, owner, u, parent[u], subset, &carried);
      if (!views.insert(k).second) continue;
      active[u] = 1;
      double cells = 1;
      for (int a : join_attrs(P, u, parent[u])) cells *= (double)std::max<int64_t>(P.attrs[a].domain, 1);
      for (int g : carried) cells *= (double)std::max<int64_t>(P.attrs[g].domain, 1);
      out += std::min(cells, 1e15) * 8.0;
    }
  }
  double scans = 0;
  for (int u = 0; u < n; ++u)
    if (active[u]) scans += (double)P.rels[u].n_rows * 16.0;
  return scans + out;
}

// ROOT_COST policy: queries without an override start at the FACT roots;
// queries with the same group-by attributes and conditions (the parts that
// decide their views) move together, class by class (largest first), to the
// root of least plan cost with the others fixed, until a round changes
// nothing (at most 4 rounds).
static void assign_roots_by_cost(Plan& P) {
  const int n = (int)P.rels.size();
  std::vector<int> roots(P.queries.size());
  std::map<std::pair<std::vector<int>, std::vector<Cond>>, std::vector<int>> classes;
  for (size_t qi = 0; qi < P.queries.size(); ++qi) {
    const QueryDef& q = P.queries[qi];
    roots[qi] = q.root >= 0 ? q.root : root_fact(P, q);
    if (roots[qi] < 0) {
      int best = 0;
      for (int r = 1; r < n; ++r)
        if (P.rels[r].n_rows > P.rels[best].n_rows) best = r;
      roots[qi] = best;
    }
    if (q.root >= 0) continue;   // the caller's override stays
    std::vector<int> gb = q.groupby;
    std::sort(gb.begin(), gb.end());
    classes[{gb, q.conds}].push_back((int)qi);
  }
  std::vector<const std::vector<int>*> order;
  for (auto& kv : classes) order.push_back(&kv.second);
  std::stable_sort(order.begin(), order.end(), [](auto* a, auto* b) { return a->size() > b->size(); });
  double cost = root_assignment_cost(P, roots);
  for (int round = 0; round < 4; ++round) {
    bool moved = false;
    for (const std::vector<int>* cls : order) {
      const int cur = roots[(*cls)[0]];
      int best = cur;
      for (int r = 0; r < n; ++r) {
        if (r == cur) continue;
        for (int qi : *cls) roots[qi] = r;
        const double c = root_assignment_cost(P, roots);
        if (c < cost * (1.0 - 1e-12)) {
          cost = c;
          best = r;
        }
      }
      for (int qi : *cls) roots[qi] = best;
      moved |= best != cur;
    }
    if (!moved) break;
  }
  for (size_t qi = 0; qi < P.queries.size(); ++qi) P.queries[qi].root = roots[qi];
}

static void generate_views(Plan& P) {
  int n = (int)P.rels.size();
  std::map<ViewKey, int> index;
  if (P.opts.root_policy == LMFAO_ROOT_COST) assign_roots_by_cost(P);
  for (size_t qi = 0; qi < P.queries.size(); ++qi) {
    QueryDef& q = P.queries[qi];
    if (q.root < 0) {
      if (q.groupby.empty()) {
        // no group-by: the FACT heuristic still roots single-relation queries there
        q.root = (P.opts.root_policy == LMFAO_ROOT_FACT) ? root_fact(P, q) : -1;
        if (q.root < 0) {
          int best = 0;
          for (int r = 1; r < n; ++r)
            if (P.rels[r].n_rows > P.rels[best].n_rows) best = r;
          q.root = best;
        }
      } else {
        q.root = (P.opts.root_policy == LMFAO_ROOT_FACT) ? root_fact(P, q) : root_groupby(P, q);
      }
    }
    std::vector<int> parent;
    std::vector<int> owner = owners_from(P, q.root, parent);
    for (int g : q.groupby)
      if (owner[g] < 0) fail(LMFAO_EINVAL, "group-by attribute not in schema");
    // bottom-up over nodes: children first so dependencies exist
    std::vector<int> bfs{q.root};
    for (size_t i = 0; i < bfs.size(); ++i)
      for (int v : P.adj[bfs[i]])
        if (v != parent[bfs[i]]) bfs.push_back(v);
    std::vector<int> vid(n, -1);
    for (int i = (int)bfs.size() - 1; i >= 1; --i) {
      int u = bfs[i], p = parent[u];
      std::vector<int> sub;
      subtree(P, u, p, sub);
      std::set<int> subset(sub.begin(), sub.end());
      auto owned = [&](int a) { return subset.count(owner[a]) != 0; };
      // a single-valued view determines its carried attributes from its key,
      // so views that differ only in them are one view storing all of them
      std::vector<int> carried;
      ViewKey k = view_key_of(P, q, owner, u, p, subset, &carried);
      int id;
      auto it = index.find(k);
      if (it == index.end()) {
        id = (int)P.views.size();
        ViewDef V;
        V.id = id;
        V.from = u;
        V.to = p;
        V.key = join_attrs(P, u, p);
        V.carried = carried;
        V.conds = k.conds;
        V.unique = P.uniq[u][p] != 0;
        P.views.push_back(V);
        index[k] = id;
      } else {
        id = it->second;
      }
      ViewDef& V = P.views[id];
      for (int g : carried)
        if (std::find(V.carried.begin(), V.carried.end(), g) == V.carried.end()) V.carried.push_back(g);
      std::sort(V.carried.begin(), V.carried.end());
      for (auto& m : q.aggs) {
        Mono r;
        for (int a : m)
          if (owned(a)) r.push_back(a);
        if (!r.empty()) V.comps.insert(r);
      }
      for (int c : P.adj[u])
        if (c != p) V.deps.insert(vid[c]);
      vid[u] = id;
    }
    for (int c : P.adj[q.root]) q.in_view[c] = vid[c];
  }
  {
    std::vector<int> roots;
    for (auto& q : P.queries) roots.push_back(q.root);
    P.root_cost = root_assignment_cost(P, roots);
  }
  // levels (dependencies form a DAG by construction)
  std::function<int(int)> lvl = [&](int v) -> int {
    ViewDef& V = P.views[v];
    if (V.level > 0 || V.deps.empty()) return V.level;
    int m = 0;
    for (int d : V.deps) m = std::max(m, lvl(d) + 1);
    V.level = m;
    return m;
  };
  for (auto& V : P.views) lvl(V.id);
  for (auto& q : P.queries) {
    int m = 0;
    for (auto& kv : q.in_view) m = std::max(m, P.views[kv.second].level + 1);
    q.level = m;
  }
  // groups: outputs leaving the same node at the same dependency level
  std::map<std::pair<int, int>, int> gidx;
  // fused form: the outputs leaving a node at a level share one pass;
  // per-view form: every output is computed by a pass of its own
  const bool per_view = P.opts.form == LMFAO_FORM_PER_VIEW;
  int solo = 0;
  auto group_of = [&](int node, int level) {
    auto k = std::make_pair(level, per_view ? -1 - solo++ * (int)P.rels.size() - node : node);
    auto it = gidx.find(k);
    if (it != gidx.end()) return it->second;
    int id = (int)P.groups.size();
    GroupDef G;
    G.node = node;
    G.level = level;
    P.groups.push_back(G);
    gidx[k] = id;
    return id;
  };
  // deterministic numbering: by level, then node
  std::vector<std::pair<std::pair<int, int>, OutRef>> all;
  for (auto& V : P.views) all.push_back({{V.level, V.from}, OutRef{1, V.id}});
  for (size_t i = 0; i < P.queries.size(); ++i)
    all.push_back({{P.queries[i].level, P.queries[i].root}, OutRef{0, (int)i}});
  std::stable_sort(all.begin(), all.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  for (auto& e : all) {
    int g = group_of(e.first.second, e.first.first);
    P.groups[g].outs.push_back(e.second);
    if (e.second.kind == 1) P.views[e.second.id].group = g;
    else P.queries[e.second.id].group = g;
  }
  auto compute_deps = [&]() {
    for (auto& G : P.groups) {
      G.deps.clear();
      for (auto& o : G.outs) {
        if (o.kind == 1)
          for (int d : P.views[o.id].deps) G.deps.insert(P.views[d].group);
        else
          for (auto& kv : P.queries[o.id].in_view) G.deps.insert(P.views[kv.second].group);
      }
    }
  };
  compute_deps();
  // one scan per relation where possible: two groups of the same node with no
  // dependency path between them become one group (no cycle can arise)
  for (bool merged = !per_view; merged;) {
    merged = false;
    int ng = (int)P.groups.size();
    std::vector<std::vector<char>> reach(ng, std::vector<char>(ng, 0));
    for (int a = 0; a < ng; ++a) {
      std::vector<int> st(P.groups[a].deps.begin(), P.groups[a].deps.end());
      while (!st.empty()) {
        int u = st.back();
        st.pop_back();
        if (reach[a][u]) continue;
        reach[a][u] = 1;   // a depends on u
        for (int d : P.groups[u].deps) st.push_back(d);
      }
    }
    for (int a = 0; a < ng && !merged; ++a)
      for (int b = a + 1; b < ng && !merged; ++b) {
        if (P.groups[a].node != P.groups[b].node || reach[a][b] || reach[b][a]) continue;
        // merge b into a, renumber
        for (auto& o : P.groups[b].outs) P.groups[a].outs.push_back(o);
        P.groups.erase(P.groups.begin() + b);
        for (auto& V : P.views)
          if (V.group == b) V.group = a; else if (V.group > b) V.group--;
        for (auto& q : P.queries)
          if (q.group == b) q.group = a; else if (q.group > b) q.group--;
        compute_deps();
        merged = true;
      }
  }
  // levels: longest dependency path
  std::function<int(int)> glevel = [&](int g) -> int {
    int m = 0;
    for (int d : P.groups[g].deps) m = std::max(m, glevel(d) + 1);
    return m;
  };
  for (size_t g = 0; g < P.groups.size(); ++g) P.groups[g].level = glevel((int)g);
  for (auto& V : P.views) V.level = P.groups[V.group].level;
  for (auto& q : P.queries) q.level = P.groups[q.group].level;
  for (auto& G : P.groups) P.n_levels = std::max(P.n_levels, G.level + 1);
}

// ---------------------------------------------------------------------------
// 6a. view layouts and attribute orders
// ---------------------------------------------------------------------------
static void view_layouts(Plan& P) {
  bool f64 = P.opts.precision == LMFAO_PREC_F64;
  for (auto& V : P.views) {
    V.n_keys = 1;
    for (int a : V.key) V.n_keys *= P.attrs[a].domain;
    if (V.unique) {
      std::set<int> s;
      for (auto& m : V.comps) s.insert(m.begin(), m.end());
      V.val_attrs.assign(s.begin(), s.end());
      V.code_attrs = V.carried;
      V.vals_f64 = f64;
    } else {
      V.val_monos.assign(V.comps.begin(), V.comps.end());
      V.vals_f64 = true;   // produced by a merged contraction (FP64)
      if (!V.carried.empty()) {
        P.supported = false;
        P.unsupported_reason = "a group-by attribute is carried through a view that is not "
                               "single-valued on its join key (multi-valued lookup)";
      }
    }
  }
}

static void attribute_orders(Plan& P) {
  int n = (int)P.rels.size();
  P.order.assign(n, {});
  for (int r = 0; r < n; ++r) {
    if (P.opts.order && P.opts.n_order && P.opts.n_order[r] > 0) {
      for (int i = 0; i < P.opts.n_order[r]; ++i) {
        auto it = P.attr_id.find(P.opts.order[r][i]);
        if (it == P.attr_id.end() || !P.rels[r].has(it->second))
          fail(LMFAO_EINVAL, "attribute order names an attribute not in " + P.rels[r].name);
        P.order[r].push_back(it->second);
      }
      // the order must cover every join attribute of the relation
      for (int c : P.adj[r])
        for (int a : join_attrs(P, r, c))
          if (std::find(P.order[r].begin(), P.order[r].end(), a) == P.order[r].end())
            fail(LMFAO_EINVAL, "attribute order of " + P.rels[r].name + " misses join attribute " +
                                   P.attrs[a].name);
      continue;
    }
    // heuristic: edges with the largest neighbouring subtree first, so the
    // biggest incoming views are looked up once per outer segment and the
    // smallest (cache-resident) ones per tuple; inside an edge, attributes
    // shared with more edges first, then smaller domains first
    std::vector<std::pair<int64_t, int>> edges;
    for (int c : P.adj[r]) {
      std::vector<int> sub;
      subtree(P, c, r, sub);
      int64_t sz = 0;
      for (int u : sub) sz += P.rels[u].n_rows;
      edges.push_back({-sz, c});
    }
    std::sort(edges.begin(), edges.end());
    std::map<int, int> shared;
    for (int c : P.adj[r])
      for (int a : join_attrs(P, r, c)) shared[a]++;
    for (auto& e : edges) {
      std::vector<int> J = join_attrs(P, r, e.second);
      std::sort(J.begin(), J.end(), [&](int x, int y) {
        if (shared[x] != shared[y]) return shared[x] > shared[y];
        if (P.attrs[x].domain != P.attrs[y].domain) return P.attrs[x].domain < P.attrs[y].domain;
        return x < y;
      });
      for (int a : J)
        if (std::find(P.order[r].begin(), P.order[r].end(), a) == P.order[r].end())
          P.order[r].push_back(a);
    }
  }
}

// ---------------------------------------------------------------------------
// 6b. group programs
// ---------------------------------------------------------------------------
struct ProgBuilder {
  Plan& P;
  GroupDef& G;
  GroupProgram& g;
  int node;
  int L;
  std::map<int, int> pos;              // attribute -> order position (1-based)
  std::map<int, int> view_index;       // view id -> program view index
  std::map<AtomRef, int> in_atom_idx, out_atom_idx, in_code_idx, out_code_idx;
  std::map<int, int> scan_col_idx, piece_col_idx;   // relation column / order pos -> position
  std::map<FeatDef, int> feat_idx;
  std::map<ColDef, int> col_idx;
  std::map<std::tuple<int, int, uint32_t>, int> pf_idx;
  std::map<uint32_t, int> pi_idx;
  std::map<std::tuple<int, int, int, int, uint32_t>, int> hist_idx;
  std::vector<std::pair<std::pair<int, int>, CellDst>> cells;

  ProgBuilder(Plan& P_, GroupDef& G_) : P(P_), G(G_), g(G_.prog), node(G_.node) {}

  int view_level(int vid) {
    int lv = 0;
    for (int a : P.views[vid].key) lv = std::max(lv, pos.at(a));
    return lv;
  }
  int add_view(int vid) {
    auto it = view_index.find(vid);
    if (it != view_index.end()) return it->second;
    int k = (int)g.views.size();
    if (k >= kMaxViews) fail(LMFAO_EUNSUPPORTED, "too many incoming views in one group");
    g.views.push_back(vid);
    int lv = view_level(vid);
    g.view_level.push_back(lv);
    g.view_outer.push_back(g.row_pieces || lv <= g.cut ? 1 : 0);
    view_index[vid] = k;
    return k;
  }
  bool attr_outer(int a) {   // local attribute
    if (g.row_pieces) return true;
    auto it = pos.find(a);
    return it != pos.end() && it->second <= g.cut;
  }
  int scan_col(int c) {
    auto it = scan_col_idx.find(c);
    if (it != scan_col_idx.end()) return it->second;
    int k = (int)g.scan_cols.size();
    if (k >= kMaxScanCols) fail(LMFAO_EUNSUPPORTED, "too many scanned columns");
    g.scan_cols.push_back(c);
    scan_col_idx[c] = k;
    return k;
  }
  // piece columns: row pieces -> relation column index; cut pieces -> order position
  int piece_col(int key) {
    auto it = piece_col_idx.find(key);
    if (it != piece_col_idx.end()) return it->second;
    int k = (int)g.piece_cols.size();
    if (k >= kMaxPieceCols) fail(LMFAO_EUNSUPPORTED, "too many piece columns");
    g.piece_cols.push_back(key);
    piece_col_idx[key] = k;
    return k;
  }
  int local_piece_col(int a) {
    if (g.row_pieces) return piece_col(P.rels[node].col.at(a));
    return piece_col(pos.at(a) - 1);
  }
  int atom(bool outer, AtomRef r) {
    auto& idx = outer ? out_atom_idx : in_atom_idx;
    auto& vec = outer ? g.out_atoms : g.in_atoms;
    auto it = idx.find(r);
    if (it != idx.end()) return it->second;
    int k = (int)vec.size();
    vec.push_back(r);
    idx[r] = k;
    return k;
  }
  int code(bool outer, CodeRef r) {
    auto& idx = outer ? out_code_idx : in_code_idx;
    auto& vec = outer ? g.out_codes : g.in_codes;
    auto it = idx.find(r);
    if (it != idx.end()) return it->second;
    int k = (int)vec.size();
    vec.push_back(r);
    idx[r] = k;
    return k;
  }
  int feat(const FeatDef& f) {
    auto it = feat_idx.find(f);
    if (it != feat_idx.end()) return it->second;
    int k = (int)feat_idx.size();
    feat_idx[f] = k;
    return k;
  }
  int col(const ColDef& c) {
    auto it = col_idx.find(c);
    if (it != col_idx.end()) return it->second;
    int k = (int)col_idx.size();
    col_idx[c] = k;
    return k;
  }
  int pi_entry(uint32_t mask) {
    auto it = pi_idx.find(mask);
    if (it != pi_idx.end()) return it->second;
    int k = (int)g.psi_i.size();
    g.psi_i.push_back(mask);
    pi_idx[mask] = k;
    return k;
  }
  int pf_entry(int ai, int aj, uint32_t mask) {
    if (ai > aj) std::swap(ai, aj);
    auto key = std::make_tuple(ai, aj, mask);
    auto it = pf_idx.find(key);
    if (it != pf_idx.end()) return it->second;
    int k = (int)g.psi_f.size();
    g.psi_f.push_back(PsiEntryF{ai, aj, mask});
    pf_idx[key] = k;
    return k;
  }
  int hist(int code, int is_float, int ai, int aj, uint32_t mask) {
    if (ai > aj) std::swap(ai, aj);
    auto key = std::make_tuple(code, is_float, ai, aj, mask);
    auto it = hist_idx.find(key);
    if (it != hist_idx.end()) return it->second;
    int k = (int)g.hists.size();
    HistDef h;
    h.code = code;
    h.dom = (int)P.attrs[attr_of_code(code)].domain;
    h.is_float = is_float;
    h.ai = ai;
    h.aj = aj;
    h.imask = mask;
    g.hists.push_back(h);
    hist_idx[key] = k;
    return k;
  }
  std::vector<int> in_code_attr;   // inner code index -> attribute
  int attr_of_code(int c) { return in_code_attr.at(c); }

  // one factor source of an output: atoms and the view it comes from
  struct Part {
    bool outer;
    int atom;      // atom index (outer or inner list)
    int view;      // program view index or -1 (local)
  };

  void build();
};

void ProgBuilder::build() {
  const RelDef& R = P.rels[node];
  g.node = node;
  g.order = P.order[node];
  L = (int)g.order.size();
  for (int i = 0; i < L; ++i) pos[g.order[i]] = i + 1;
  // cut level: small relations are contracted row by row; large ones are
  // scanned with per-piece partial sums at the deepest level whose average
  // segment is still long
  int64_t min_seg = P.opts.min_segment > 0 ? P.opts.min_segment : 64;
  const int64_t kRowPieceMax = P.opts.row_piece_max == 0 ? (int64_t)1 << 16 : P.opts.row_piece_max;
  // an output whose dense key space is too large is kept in a hash table; its
  // group is evaluated row by row, where every output's cells are scattered
  bool hashed = false;
  for (auto& o : G.outs) {
    const std::vector<int>& gb = o.kind == 0 ? P.queries[o.id].groupby : P.views[o.id].carried;
    double cells = 1;
    for (int a : gb) cells *= (double)P.attrs[a].domain;
    if (o.kind == 1)
      for (int a : P.views[o.id].key) cells *= (double)P.attrs[a].domain;
    hashed |= cells > (double)kDenseRowsMax;
  }
  if (R.n_rows <= kRowPieceMax || hashed || G.force_rows) {
    g.row_pieces = true;
    g.cut = L + 1;
  } else {
    g.row_pieces = false;
    g.cut = 0;
    double prod = 1;
    for (int l = 1; l <= L; ++l) {
      prod *= (double)P.attrs[g.order[l - 1]].domain;
      double seg = (double)R.n_rows / std::min<double>(prod, (double)R.n_rows);
      if (seg >= (double)min_seg) g.cut = l;
      else break;
    }
  }
  // outputs of the program: queries and non-unique views
  std::vector<OutRef> outs;
  for (auto& o : G.outs) {
    if (o.kind == 1 && P.views[o.id].unique) G.unique_views.push_back(o.id);
    else outs.push_back(o);
  }
  if (outs.empty()) return;
  G.has_program = true;
  for (size_t oi = 0; oi < outs.size(); ++oi) {
    OutRef o = outs[oi];
    // incoming views and cells of this output
    std::vector<int> invs;
    std::vector<int> keyattrs;
    std::vector<Mono> monos;
    int excluded = -1;
    if (o.kind == 0) {
      const QueryDef& q = P.queries[o.id];
      for (auto& kv : q.in_view) invs.push_back(kv.second);
      keyattrs = q.groupby;
      monos = q.aggs;
    } else {
      const ViewDef& V = P.views[o.id];
      invs.assign(V.deps.begin(), V.deps.end());
      keyattrs = V.key;
      for (int a : V.carried) keyattrs.push_back(a);
      monos = V.val_monos;
      excluded = V.to;
    }
    (void)excluded;
    uint32_t omask = 0, imask = 0;
    std::map<int, int> side_view;   // neighbour -> program view index
    for (int vid : invs) {
      int k = add_view(vid);
      side_view[P.views[vid].from] = k;
      if (g.view_outer[k]) omask |= 1u << k;
      else imask |= 1u << k;
    }
    // where does an attribute come from at this node?
    auto source_view = [&](int a) -> int {
      for (auto& kv : side_view) {
        std::vector<int> sub;
        subtree(P, kv.first, node, sub);
        for (int u : sub)
          if (P.rels[u].has(a)) return kv.second;
      }
      fail(LMFAO_EINVAL, "attribute " + P.attrs[a].name + " unreachable from " + R.name);
      return -1;
    };
    // codes of the key
    ProgOutput po;
    po.ref = o;
    po.dst_is_view = o.kind == 1;
    std::vector<int> kcode;
    std::vector<char> kouter;
    for (int a : keyattrs) {
      bool outer;
      CodeRef cr;
      if (R.has(a)) {
        outer = attr_outer(a);
        cr = outer ? CodeRef{SRC_COL, local_piece_col(a), 0}
                   : CodeRef{SRC_COL, scan_col(R.col.at(a)), 0};
      } else {
        int vk = source_view(a);
        const ViewDef& V = P.views[g.views[vk]];
        int slot = V.slot_of_code(a);
        if (slot < 0) fail(LMFAO_EUNSUPPORTED, "group-by attribute " + P.attrs[a].name +
                                                   " is not single-valued at " + R.name);
        outer = g.view_outer[vk] != 0;
        cr = CodeRef{SRC_VIEW, vk, slot};
      }
      int ci = code(outer, cr);
      if (!outer) {
        if ((int)in_code_attr.size() <= ci) in_code_attr.resize(ci + 1, -1);
        in_code_attr[ci] = a;
      }
      kcode.push_back(ci);
      kouter.push_back(outer);
      po.key_codes.push_back(ci);
      po.key_codes_outer.push_back(outer);
    }
    po.n_rows = 1;
    std::vector<int64_t> dom;
    for (int a : keyattrs) dom.push_back(P.attrs[a].domain);
    po.key_stride.assign(keyattrs.size(), 1);
    for (int i = (int)keyattrs.size() - 1; i >= 0; --i) {
      po.key_stride[i] = po.n_rows;
      po.n_rows *= dom[i];
    }
    po.hashed = po.n_rows > kDenseRowsMax;
    if (po.hashed && o.kind == 1)
      fail(LMFAO_EUNSUPPORTED, "view " + std::to_string(o.id) + " at " + R.name + ": key space too large for a dense view");
    po.n_comps = (int)monos.size();
    // split every component monomial into atoms (outer / inner)
    struct Split {
      std::vector<Part> parts;
    };
    std::vector<Split> splits;
    for (auto& m : monos) {
      Split s;
      std::map<int, Mono> per_view;   // program view -> restricted monomial
      for (int a : m) {
        if (R.has(a)) {
          bool outer = attr_outer(a);
          AtomRef ar = outer ? AtomRef{SRC_COL, local_piece_col(a), 0}
                             : AtomRef{SRC_COL, scan_col(R.col.at(a)), 0};
          s.parts.push_back(Part{outer, atom(outer, ar), -1});
        } else {
          per_view[source_view(a)].push_back(a);
        }
      }
      for (auto& kv : per_view) {
        int vk = kv.first;
        const ViewDef& V = P.views[g.views[vk]];
        bool outer = g.view_outer[vk] != 0;
        if (V.unique) {
          for (int a : kv.second) {
            int slot = V.slot_of_attr(a);
            if (slot < 0) fail(LMFAO_EINVAL, "internal: view lacks attribute " + P.attrs[a].name);
            s.parts.push_back(Part{outer, atom(outer, AtomRef{SRC_VIEW, vk, slot}), vk});
          }
        } else {
          Mono mm = kv.second;
          std::sort(mm.begin(), mm.end());
          int slot = V.slot_of_mono(mm);
          if (slot < 0) fail(LMFAO_EINVAL, "internal: view lacks component " + mono_str(P, mm));
          s.parts.push_back(Part{outer, atom(outer, AtomRef{SRC_VIEW, vk, slot}), vk});
        }
      }
      splits.push_back(s);
    }
    // multiplicity masks: non-unique views that contribute a value carry
    // their own multiplicity, so they leave the mask of that cell
    auto masks_for = [&](const Split& s, uint32_t& om, uint32_t& im) {
      om = omask;
      im = imask;
      for (auto& p : s.parts)
        if (p.view >= 0 && !P.views[g.views[p.view]].unique) {
          if (p.outer) om &= ~(1u << p.view);
          else im &= ~(1u << p.view);
        }
    };
    // mode
    std::vector<int> inner_codes, outer_codes;
    for (size_t i = 0; i < kcode.size(); ++i) (kouter[i] ? outer_codes : inner_codes).push_back((int)i);
    bool any_outer_atom = false;
    for (auto& s : splits)
      for (auto& p : s.parts) any_outer_atom |= p.outer;
    int64_t outer_prod = 1;
    for (int i : outer_codes) outer_prod *= dom[i];
    bool outer_small = outer_prod <= kOneHotMax;
    // an output keyed only by outer codes can take either form: one-hot
    // features of the matrix product (cheap for small domains) or a scatter
    // of each piece's cells (cheap once the one-hot features outnumber them)
    const int64_t pure_one_hot = P.opts.one_hot_max > 0 ? P.opts.one_hot_max
                                 : G.one_hot_pure > 0  ? G.one_hot_pure
                                                       : kOneHotMax;
    bool counts_only = monos.empty();
    bool pure_inner = outer_codes.empty() && !any_outer_atom;
    if (inner_codes.empty()) {
      po.mode = outer_prod <= pure_one_hot ? 0 : 1;
    } else if (pure_inner && (counts_only || inner_codes.size() > 1 || dom[inner_codes[0]] > kHistMax)) {
      po.mode = 2;   // direct table: no outer factor to multiply later
    } else if (inner_codes.size() == 1 && dom[inner_codes[0]] <= kHistMax && outer_small) {
      po.mode = 0;   // per-piece histogram, contracted with the outer features
    } else {
      fail(LMFAO_EUNSUPPORTED, std::string(o.kind == 0 ? "query " : "view ") + std::to_string(o.id) +
                                   " at " + R.name + " mixes large inner group-by keys with outer factors");
    }
    if (g.row_pieces && po.mode == 2) po.mode = 1;   // row pieces: every code is outer
    po.omask = omask;
    int out_index = (int)g.outs.size();
    // enumerate cells
    int ncomp = (int)monos.size();
    for (int ci = -1; ci < ncomp; ++ci) {
      Split s = ci < 0 ? Split{} : splits[ci];
      uint32_t om, im;
      masks_for(s, om, im);
      std::vector<int> oat, iat;
      for (auto& p : s.parts) (p.outer ? oat : iat).push_back(p.atom);
      if (oat.size() > 2 || iat.size() > 2) fail(LMFAO_EUNSUPPORTED, "component of degree > 2");
      if (po.mode == 1 && o.kind == 0 && ci >= 0 && oat.empty() && iat.empty()) {
        // a SUM(1) component of a query (FP64 results) under the count's
        // masks scatters the same cells as the count: it is copied from the
        // count instead
        uint32_t om0, im0;
        masks_for(Split{}, om0, im0);
        if (om == om0 && im == im0) {
          po.count_copies.push_back(ci);
          continue;
        }
      }
      if (po.mode == 2) {   // table: inner codes only, inner atoms only
        TableComp tc;
        tc.comp = ci;
        tc.ai = iat.size() > 0 ? iat[0] : -1;
        tc.aj = iat.size() > 1 ? iat[1] : -1;
        tc.imask = im;
        po.tcomps.push_back(tc);
        if (om) { g.needs_mu_out_in_scan = true; g.tables_outer_mask |= om; }
        po.omask = om;
        continue;
      }
      // enumerate key values
      int nk = (int)kcode.size();
      std::vector<int> val(nk, 0);
      std::function<void(int)> rec = [&](int d) {
        if (d < nk) {
          bool expand = po.mode == 0;   // scatter: codes give the row, not features
          if (expand) {
            for (int v = 0; v < dom[d]; ++v) { val[d] = v; rec(d + 1); }
          } else {
            val[d] = 0;
            rec(d + 1);
          }
          return;
        }
        // inner part
        int icode = -1, ibin = 0;
        for (int i : inner_codes) { icode = kcode[i]; ibin = val[i]; }
        std::vector<std::pair<int, int>> ocodes;   // (outer code index, value)
        if (po.mode == 0)
          for (int i : outer_codes) ocodes.push_back({kcode[i], val[i]});
        bool inner_trivial = icode < 0 && iat.empty();
        FeatDef f;
        f.mask = om;
        ColDef c;
        if (!inner_trivial) {
          if (g.row_pieces) fail(LMFAO_EINVAL, "internal: inner part with row pieces");
          if (icode >= 0) {
            int h = hist(icode, iat.empty() ? 0 : 1, iat.size() > 0 ? iat[0] : -1,
                         iat.size() > 1 ? iat[1] : -1, im);
            c.kind = iat.empty() ? B_PSI_I : B_PSI_F;
            c.entry = h;   // resolved to a row position later
            c.bin = ibin;
          } else {
            c.kind = B_PSI_F;
            c.entry = pf_entry(iat.size() > 0 ? iat[0] : -1, iat.size() > 1 ? iat[1] : -1, im);
            c.bin = -1;
          }
          if (ocodes.size() > 0) { f.c1 = ocodes[0].first; f.v1 = ocodes[0].second; }
          if (ocodes.size() > 1) { f.c2 = ocodes[1].first; f.v2 = ocodes[1].second; }
          if (oat.size() > 0) f.a1 = oat[0];
          if (oat.size() > 1) f.a2 = oat[1];
        } else {
          c.kind = B_CNTF;
          c.entry = pi_entry(g.row_pieces ? 0u : im);
          c.bin = -1;
          // the feature takes one outer part (a code, else a factor), the
          // column the rest, so features and columns stay single factors
          std::vector<std::pair<int, int>> rc = ocodes;
          std::vector<int> ra = oat;
          if (!rc.empty()) {
            f.c1 = rc[0].first;
            f.v1 = rc[0].second;
            rc.erase(rc.begin());
          } else if (!ra.empty()) {
            f.a1 = ra[0];
            ra.erase(ra.begin());
          }
          if (rc.size() > 0) { c.feat.c1 = rc[0].first; c.feat.v1 = rc[0].second; }
          if (rc.size() > 1) { c.feat.c2 = rc[1].first; c.feat.v2 = rc[1].second; }
          if (ra.size() > 0) c.feat.a1 = ra[0];
          if (ra.size() > 1) c.feat.a2 = ra[1];
          if (c.feat.a1 > c.feat.a2 && c.feat.a2 >= 0) std::swap(c.feat.a1, c.feat.a2);
        }
        if (f.a1 > f.a2 && f.a2 >= 0) std::swap(f.a1, f.a2);
        int fi = feat(f);
        int gi = col(c);
        if (po.mode == 0) {
          int64_t row = 0;
          for (int i = 0; i < nk; ++i) row += val[i] * po.key_stride[i];
          cells.push_back({{fi, gi}, CellDst{out_index, row, ci}});
        } else {
          g.scatter.push_back(ScatterCell{out_index, ci, fi, gi});
        }
      };
      rec(0);
    }
    g.outs.push_back(po);
  }
  // inner masks list
  std::set<uint32_t> ms;
  for (auto m : g.psi_i) ms.insert(m);
  for (auto& e : g.psi_f) ms.insert(e.imask);
  for (auto& h : g.hists) ms.insert(h.imask);
  for (auto& o : g.outs)
    for (auto& t : o.tcomps) ms.insert(t.imask);
  g.in_masks.assign(ms.begin(), ms.end());
  // histogram block offsets
  g.hist_f_bins = g.hist_i_bins = 0;
  for (auto& h : g.hists) {
    if (h.is_float) { h.offset = g.hist_f_bins; g.hist_f_bins += h.dom; }
    else { h.offset = g.hist_i_bins; g.hist_i_bins += h.dom; }
  }
  // order features and columns: integer ones first
  std::vector<FeatDef> fv(feat_idx.size());
  for (auto& kv : feat_idx) fv[kv.second] = kv.first;
  std::vector<ColDef> cv(col_idx.size());
  for (auto& kv : col_idx) cv[kv.second] = kv.first;
  std::vector<int> fperm(fv.size()), cperm(cv.size());
  std::vector<int> fo(fv.size()), co(cv.size());
  std::iota(fo.begin(), fo.end(), 0);
  std::iota(co.begin(), co.end(), 0);
  std::stable_sort(fo.begin(), fo.end(), [&](int a, int b) { return fv[a].is_int() > fv[b].is_int(); });
  std::stable_sort(co.begin(), co.end(), [&](int a, int b) { return cv[a].is_int() > cv[b].is_int(); });
  g.feats.clear();
  g.cols.clear();
  for (size_t i = 0; i < fo.size(); ++i) { fperm[fo[i]] = (int)i; g.feats.push_back(fv[fo[i]]); }
  for (size_t i = 0; i < co.size(); ++i) { cperm[co[i]] = (int)i; g.cols.push_back(cv[co[i]]); }
  g.n_feat_int = 0;
  for (auto& f : g.feats) g.n_feat_int += f.is_int();
  g.n_col_int = 0;
  for (auto& c : g.cols) g.n_col_int += c.is_int();
  // resolve psi row positions of columns
  int pf_n = (int)g.psi_f.size();
  int pi_n = (int)g.psi_i.size();
  for (auto& c : g.cols) {
    if (c.kind == B_PSI_F) {
      if (c.bin < 0) c.entry = c.entry;                       // float entry slot
      else c.entry = pf_n + g.hists[c.entry].offset + c.bin;  // float histogram bin
    } else if (c.kind == B_PSI_I) {
      c.entry = pi_n + g.hists[c.entry].offset + c.bin;       // count histogram bin
    }
    c.bin = 0;
  }
  for (auto& cl : cells) {
    cl.first.first = fperm[cl.first.first];
    cl.first.second = cperm[cl.first.second];
  }
  for (auto& s : g.scatter) {
    s.f = fperm[s.f];
    s.g = cperm[s.g];
  }
  g.gemm_cells = cells;
}

// cells of an output's dense key space
static double out_cells(const Plan& P, const OutRef& o) {
  const std::vector<int>& gb = o.kind == 0 ? P.queries[o.id].groupby : P.views[o.id].carried;
  double cells = 1;
  for (int a : gb) cells *= (double)P.attrs[a].domain;
  if (o.kind == 1)
    for (int a : P.views[o.id].key) cells *= (double)P.attrs[a].domain;
  return cells;
}

// factors a scan holds: the inner atoms, plus one copy of an atom for every
// further mask under which a float entry needs the same triangle slot (the
// runtime builds the scan descriptor the same way)
static int scan_atoms(const GroupProgram& g) {
  int n = (int)g.in_atoms.size();
  std::map<std::pair<int, int>, uint32_t> taken;
  for (const PsiEntryF& e : g.psi_f) {
    int ai = e.ai, aj = e.aj;
    auto it = taken.find({ai, aj});
    if (it != taken.end() && it->second != e.imask) {
      const int dup = n++;
      if (aj >= 0) aj = dup; else ai = dup;
      if (ai > aj) std::swap(ai, aj);
    }
    taken[{ai, aj}] = e.imask;
  }
  return n;
}

// what the kernels of one group can hold
static bool program_fits(const GroupProgram& g) {
  int tables = 0, inner_views = 0;
  bool table_ok = true;
  for (const ProgOutput& po : g.outs) {
    tables += po.mode == 2;
    if (po.mode == 2)
      table_ok = table_ok && po.key_codes.size() <= 3 && po.tcomps.size() <= (size_t)kMaxTableComps;
  }
  for (int o : g.view_outer) inner_views += o == 0;
  if (!g.row_pieces && (scan_atoms(g) > kMaxAtoms || inner_views > kMaxInnerViews || !table_ok)) return false;
  // a scan block holds every histogram once per wavefront (FP64 bins at most),
  // the per-wave factor staging and the LDS-privatized tables
  const int64_t wave = (int64_t)g.hist_i_bins * 4 + (int64_t)g.hist_f_bins * 8 + 16 + (kMaxAtoms + 5) * 64 * 8;
  const bool lds_ok = (int64_t)kScanWaves * wave + kLdsTableMax * 4 <= kLdsBytes;
  return g.in_masks.size() <= (size_t)kMaxMasks && g.psi_i.size() <= (size_t)kMaxMasks &&
         g.in_codes.size() <= (size_t)kMaxCodes && g.hists.size() <= (size_t)kMaxHists &&
         g.views.size() <= (size_t)kMaxViews && (g.row_pieces || (tables <= kMaxTables && lds_ok));
}

// Moves outputs [from, end) of group gi into a new group at the same node and
// level (no dependency between the two) and renumbers the outputs' groups.
static void split_group(Plan& P, int gi, size_t from) {
  GroupDef H;
  H.node = P.groups[gi].node;
  H.level = P.groups[gi].level;
  H.force_rows = P.groups[gi].force_rows;
  H.one_hot_pure = P.groups[gi].one_hot_pure;
  H.outs.assign(P.groups[gi].outs.begin() + from, P.groups[gi].outs.end());
  P.groups[gi].outs.resize(from);
  const int hi = (int)P.groups.size();
  for (auto& o : H.outs) {
    if (o.kind == 1) P.views[o.id].group = hi;
    else P.queries[o.id].group = hi;
  }
  P.groups.push_back(H);
  for (auto& G : P.groups) {
    G.deps.clear();
    for (auto& o : G.outs) {
      if (o.kind == 1)
        for (int d : P.views[o.id].deps) G.deps.insert(P.views[d].group);
      else
        for (auto& kv : P.queries[o.id].in_view) G.deps.insert(P.views[kv.second].group);
    }
  }
}

// A query whose every aggregate is SUM(1), rooted at `node`, grouped by at
// most 3 attributes into a table larger than a scan keeps in LDS (dense, or a
// hash table past 2^24 cells), whose group-by attributes are columns of the
// node or carried by the single-valued views into it: its table is counted by
// radix partition (a slice of the key space, or of a hash of the key, at a
// time, in LDS) instead of by global atomics from a scan or a row pass.
// Views with several subtree tuples per key may join in (carrying no
// group-by attribute): each row then counts with the product of their
// counts.
static double query_cells(const Plan& P, int qid) {
  double cells = 1;
  for (int a : P.queries[qid].groupby) cells *= (double)std::max<int64_t>(P.attrs[a].domain, 0);
  return cells;
}

static bool partition_eligible(const Plan& P, int qid, int node, double min_cells = (double)kLdsTableMax) {
  const QueryDef& Q = P.queries[qid];
  if (Q.root != node || Q.groupby.empty() || Q.groupby.size() > 3) return false;
  for (const Mono& m : Q.aggs)
    if (!m.empty()) return false;
  for (int a : Q.groupby)
    if (P.attrs[a].domain <= 0) return false;
  const double cells = query_cells(P, qid);
  // dense tables past what a scan keeps in LDS, and hash tables (key spaces
  // past 2^24 cells) of cells below 2^62
  if (cells <= min_cells || cells >= 4.6e18) return false;
  if (Q.in_view.size() > 4) return false;
  for (auto& kv : Q.in_view) {
    const ViewDef& V = P.views[kv.second];
    if (V.key.size() > 2) return false;
    // a view of several subtree tuples per key weights the row by its count;
    // it may not carry a group-by attribute (the row would not determine
    // the cell)
    if (!V.unique && !V.carried.empty()) return false;
  }
  for (int a : Q.groupby) {
    if (P.rels[node].has(a)) continue;
    bool carried = false;
    for (auto& kv : Q.in_view)
      for (int c : P.views[kv.second].carried) carried |= c == a;
    if (!carried) return false;
  }
  return true;
}

// A scan keeps its group-by tables in LDS, in output order, while they fit
// in kLdsTableMax cells, and adds to the others with a global atomic per row.
// The partition-eligible ones among those
// that would not fit move to a partitioned group of the same node and level
// (counted in LDS a slice at a time).  Returns whether any moved.
static bool move_lds_overflow(Plan& P, int gi) {
  GroupDef& G = P.groups[gi];
  int64_t used = 0;
  std::vector<OutRef> moved;
  for (const ProgOutput& po : G.prog.outs) {
    if (po.mode != 2) continue;
    if (used + po.n_rows <= kLdsTableMax) {
      used += po.n_rows;
      continue;
    }
    if (po.ref.kind == 0 && partition_eligible(P, po.ref.id, G.node, (double)kPartMinCells)) moved.push_back(po.ref);
  }
  if (moved.empty()) return false;
  int target = -1;
  for (size_t h = 0; h < P.groups.size(); ++h)
    if ((int)h != gi && P.groups[h].partitioned && P.groups[h].node == G.node && P.groups[h].level == G.level)
      target = (int)h;
  std::vector<OutRef> keep;
  for (const OutRef& o : G.outs)
    if (std::find_if(moved.begin(), moved.end(), [&](const OutRef& m) { return m.kind == o.kind && m.id == o.id; }) ==
        moved.end())
      keep.push_back(o);
  if (target < 0) {
    G.outs = keep;
    G.outs.insert(G.outs.end(), moved.begin(), moved.end());
    split_group(P, gi, keep.size());
    P.groups.back().partitioned = true;
    P.groups.back().has_program = false;
  } else {
    P.groups[gi].outs = keep;
    for (const OutRef& m : moved) {
      P.groups[target].outs.push_back(m);
      P.queries[m.id].group = target;
    }
    for (auto& H : P.groups) {
      H.deps.clear();
      for (auto& o : H.outs) {
        if (o.kind == 1)
          for (int d : P.views[o.id].deps) H.deps.insert(P.views[d].group);
        else
          for (auto& kv : P.queries[o.id].in_view) H.deps.insert(P.views[kv.second].group);
      }
    }
  }
  return true;
}

// Moves the partition-eligible queries of every group into a group of their
// own at the same node and level (no program; the runtime counts them).
// Tables past a scan's LDS tables (kLdsTableMax cells) move.  Once a group
// has such a table (so the partition count's row pass is paid anyway), the
// tables keyed by the node's own columns move too once they are past what a
// scan keeps in registers (kPartSmallCells), or, on relations of
// kPartLargeRows rows or more, past kPartScanCells (smaller ones cost less
// in the scan's shared pass).  Tables keyed by a code a view carries stay at
// the LDS threshold: the partition count gathers such codes a row at a
// time.  (Measured on the Rk-means chain, the grocery star and the CART
// batch: each choice pays on its side.)
static void extract_partitioned(Plan& P) {
  const size_t n = P.groups.size();
  for (size_t gi = 0; gi < n; ++gi) {
    GroupDef& G = P.groups[gi];
    if (G.force_rows || G.partitioned) continue;
    const RelDef& R = P.rels[G.node];
    bool any_large = false;
    for (const OutRef& o : G.outs) any_large |= o.kind == 0 && partition_eligible(P, o.id, G.node);
    auto min_cells = [&](int qid) {
      if (!any_large) return (double)kLdsTableMax;
      for (int a : P.queries[qid].groupby)
        if (!R.has(a)) return (double)kLdsTableMax;
      return (double)(R.n_rows >= kPartLargeRows ? kPartScanCells : kPartSmallCells);
    };
    std::vector<OutRef> keep, part;
    for (const OutRef& o : G.outs)
      (o.kind == 0 && partition_eligible(P, o.id, G.node, min_cells(o.id)) ? part : keep).push_back(o);
    if (part.empty()) continue;
    if (keep.empty()) {
      G.partitioned = true;
      continue;
    }
    G.outs = keep;
    G.outs.insert(G.outs.end(), part.begin(), part.end());
    split_group(P, (int)gi, keep.size());
    P.groups.back().partitioned = true;
  }
}

// Builds every group's program.  Outputs kept in hash tables are evaluated row
// by row, so they leave their group for one of their own; a group whose
// program exceeds what one scan kernel holds (columns, codes, masks,
// histograms, views) is halved until each part fits.
static void build_programs(Plan& P) {
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    auto& outs = P.groups[gi].outs;
    std::stable_partition(outs.begin(), outs.end(),
                          [&](const OutRef& o) { return out_cells(P, o) <= (double)kDenseRowsMax; });
    size_t n_dense = 0;
    while (n_dense < outs.size() && out_cells(P, outs[n_dense]) <= (double)kDenseRowsMax) ++n_dense;
    if (n_dense > 0 && n_dense < outs.size()) split_group(P, (int)gi, n_dense);
  }
  if (P.opts.partition == 0) extract_partitioned(P);
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    if (P.groups[gi].partitioned) {
      P.groups[gi].has_program = false;
      continue;
    }
    for (;;) {
      GroupDef& G = P.groups[gi];
      G.has_program = false;
      G.prog = GroupProgram{};
      G.unique_views.clear();
      std::string why;
      try {
        ProgBuilder b(P, G);
        b.build();
        // many one-hot features (each a row of the matrix product) cost more
        // than scattering the outer-only outputs' cells per piece
        if (G.has_program && P.opts.one_hot_max == 0 && G.one_hot_pure == 0 &&
            G.prog.feats.size() > (size_t)kOneHotFeatureBudget) {
          G.one_hot_pure = kOneHotPure;
          continue;
        }
        if (G.has_program && program_fits(G.prog) && P.opts.partition == 0 && move_lds_overflow(P, (int)gi)) continue;
        if (!G.has_program || program_fits(G.prog)) break;
        why = "a group exceeds the limits of one scan kernel";
      } catch (const PlanError& e) {
        if (e.status != LMFAO_EUNSUPPORTED) throw;
        if (e.msg.find("mixes large inner group-by keys") != std::string::npos && !G.force_rows) {
          // outputs with no scan form go to a group evaluated row by row
          auto& outs = P.groups[gi].outs;
          std::vector<char> alone_ok(outs.size(), 1);
          for (size_t k = 0; k < outs.size(); ++k) {
            GroupDef T;
            T.node = P.groups[gi].node;
            T.level = P.groups[gi].level;
            T.outs = {outs[k]};
            try {
              ProgBuilder tb(P, T);
              tb.build();
            } catch (const PlanError& e2) {
              if (e2.status != LMFAO_EUNSUPPORTED || e2.msg.find("mixes large inner") == std::string::npos) throw;
              alone_ok[k] = 0;
            }
          }
          std::vector<OutRef> keep, rows;
          for (size_t k = 0; k < outs.size(); ++k) (alone_ok[k] ? keep : rows).push_back(outs[k]);
          if (keep.empty()) {
            P.groups[gi].force_rows = true;
          } else {
            outs = keep;
            outs.insert(outs.end(), rows.begin(), rows.end());
            split_group(P, (int)gi, keep.size());
            P.groups.back().force_rows = true;
          }
          continue;
        }
        if (e.msg.rfind("too many", 0) != 0) throw;
        why = e.msg;
      }
      if (P.groups[gi].outs.size() < 2) fail(LMFAO_EUNSUPPORTED, why);
      split_group(P, (int)gi, P.groups[gi].outs.size() / 2);
    }
  }
}

// ---------------------------------------------------------------------------
// plan description (JSON)
// ---------------------------------------------------------------------------
static std::string describe(const Plan& P) {
  std::ostringstream o;
  auto attrs_json = [&](const std::vector<int>& v) {
    std::string s = "[";
    for (size_t i = 0; i < v.size(); ++i) {
      if (i) s += ",";
      s += "\"" + json_escape(P.attrs[v[i]].name) + "\"";
    }
    return s + "]";
  };
  o << "{\"relations\":[";
  for (size_t r = 0; r < P.rels.size(); ++r) {
    if (r) o << ",";
    o << "{\"name\":\"" << json_escape(P.rels[r].name) << "\",\"order\":" << attrs_json(P.order[r]) << "}";
  }
  o << "],\"queries\":[";
  for (size_t i = 0; i < P.queries.size(); ++i) {
    const QueryDef& q = P.queries[i];
    if (i) o << ",";
    o << "{\"root\":\"" << json_escape(P.rels[q.root].name) << "\",\"group\":" << q.group
      << ",\"level\":" << q.level << ",\"groupby\":" << attrs_json(q.groupby) << ",\"views\":[";
    bool first = true;
    for (auto& kv : q.in_view) {
      if (!first) o << ",";
      first = false;
      o << kv.second;
    }
    o << "]}";
  }
  static const char* ops[] = {"<=", "<", ">", ">=", "==", "!="};
  o << std::setprecision(17);
  o << "],\"filter\":[";
  for (size_t i = 0; i < P.filter.size(); ++i) {
    if (i) o << ",";
    o << "[\"" << json_escape(P.attrs[P.filter[i].attr].name) << "\",\"" << ops[P.filter[i].op] << "\","
      << P.filter[i].c << "]";
  }
  {
    char num[64];
    std::snprintf(num, sizeof num, "%.6g", P.root_cost);
    o << "],\"root_cost_bytes\":" << num;
    if (!P.root_fallback.empty())
      o << ",\"root_fallback\":\"" << json_escape(P.root_fallback) << "\"";
  }
  o << ",\"derived\":[";
  for (size_t i = 0; i < P.derived.size(); ++i) {
    const DerivedAttr& D = P.derived[i];
    if (i) o << ",";
    o << "{\"name\":\"" << json_escape(P.attrs[D.attr].name) << "\",\"source\":\""
      << json_escape(P.attrs[D.src].name) << "\",\"relation\":\"" << json_escape(P.rels[D.rel].name)
      << "\",\"kind\":" << D.kind << ",\"thresholds\":" << (D.kind == 2 ? 0 : D.thr.size())
      << ",\"threshold_values\":[";
    for (size_t t = 0; D.kind != 2 && t < D.thr.size(); ++t) {
      char num[64];
      std::snprintf(num, sizeof num, "%.17g", D.thr[t]);
      o << (t ? "," : "") << num;
    }
    o << "]}";
  }
  o << "],\"user_queries\":[";
  for (size_t i = 0; i < P.user.size(); ++i) {
    const UserQuery& U = P.user[i];
    if (i) o << ",";
    o << "{\"planned\":" << U.internal;
    if (U.range) o << ",\"lo\":" << U.lo << ",\"hi\":" << U.hi << ",\"except\":" << U.ex;
    o << "}";
  }
  o << "],\"views\":[";
  for (size_t i = 0; i < P.views.size(); ++i) {
    const ViewDef& V = P.views[i];
    if (i) o << ",";
    o << "{\"id\":" << V.id << ",\"from\":\"" << json_escape(P.rels[V.from].name) << "\",\"to\":\""
      << json_escape(P.rels[V.to].name) << "\",\"key\":" << attrs_json(V.key)
      << ",\"carried\":" << attrs_json(V.carried) << ",\"unique\":" << (V.unique ? "true" : "false")
      << ",\"level\":" << V.level << ",\"group\":" << V.group << ",\"components\":[";
    bool first = true;
    for (auto& m : V.comps) {
      if (!first) o << ",";
      first = false;
      o << "\"" << json_escape(mono_str(P, m)) << "\"";
    }
    o << "],\"deps\":[";
    first = true;
    for (int d : V.deps) {
      if (!first) o << ",";
      first = false;
      o << d;
    }
    // physical layout: the value columns and code columns lmfao_view_copy
    // returns per dense key (last key attribute fastest), and the conditions
    // pushed into the view
    o << "],\"n_keys\":" << V.n_keys << ",\"stored_values\":[";
    first = true;
    if (V.unique) {
      for (int a : V.val_attrs) {
        if (!first) o << ",";
        first = false;
        o << "\"" << json_escape(P.attrs[a].name) << "\"";
      }
    } else {
      for (auto& m : V.val_monos) {
        if (!first) o << ",";
        first = false;
        o << "\"" << json_escape(mono_str(P, m)) << "\"";
      }
    }
    o << "],\"stored_codes\":" << attrs_json(V.code_attrs) << ",\"conditions\":[";
    for (size_t c = 0; c < V.conds.size(); ++c) {
      if (c) o << ",";
      char num[64];
      std::snprintf(num, sizeof num, "%.17g", V.conds[c].c);
      o << "[\"" << json_escape(P.attrs[V.conds[c].attr].name) << "\"," << V.conds[c].op << "," << num << "]";
    }
    o << "]}";
  }
  o << "],\"groups\":[";
  for (size_t i = 0; i < P.groups.size(); ++i) {
    const GroupDef& G = P.groups[i];
    if (i) o << ",";
    o << "{\"id\":" << i << ",\"node\":\"" << json_escape(P.rels[G.node].name) << "\",\"level\":" << G.level
      << ",\"outputs\":[";
    for (size_t k = 0; k < G.outs.size(); ++k) {
      if (k) o << ",";
      o << "{\"kind\":\"" << (G.outs[k].kind == 0 ? "query" : "view") << "\",\"id\":" << G.outs[k].id << "}";
    }
    o << "],\"deps\":[";
    bool first = true;
    for (int d : G.deps) {
      if (!first) o << ",";
      first = false;
      o << d;
    }
    o << "]";
    if (G.partitioned) o << ",\"partitioned\":true";
    if (G.has_program) {
      const GroupProgram& g = G.prog;
      o << ",\"program\":{\"cut\":" << g.cut << ",\"row_pieces\":" << (g.row_pieces ? "true" : "false")
        << ",\"views\":[";
      for (size_t k = 0; k < g.views.size(); ++k) {
        if (k) o << ",";
        o << "{\"view\":" << g.views[k] << ",\"level\":" << g.view_level[k]
          << ",\"outer\":" << (g.view_outer[k] ? "true" : "false") << "}";
      }
      o << "],\"inner_atoms\":" << g.in_atoms.size() << ",\"inner_codes\":" << g.in_codes.size()
        << ",\"outer_atoms\":" << g.out_atoms.size() << ",\"outer_codes\":" << g.out_codes.size()
        << ",\"psi_float\":" << g.psi_f.size() << ",\"psi_count\":" << g.psi_i.size()
        << ",\"hist_float_bins\":" << g.hist_f_bins << ",\"hist_count_bins\":" << g.hist_i_bins
        << ",\"features\":" << g.feats.size() << ",\"columns\":" << g.cols.size()
        << ",\"gemm_cells\":" << g.gemm_cells.size() << ",\"scatter_cells\":" << g.scatter.size()
        << ",\"feature_list\":[";
      for (size_t k = 0; k < g.feats.size(); ++k) {
        const FeatDef& f = g.feats[k];
        if (k) o << ",";
        o << "[" << f.mask << "," << f.c1 << "," << f.v1 << "," << f.c2 << "," << f.v2 << "," << f.a1 << "," << f.a2 << "]";
      }
      o << "]"
        << ",\"outputs\":[";
      for (size_t k = 0; k < g.outs.size(); ++k) {
        if (k) o << ",";
        const ProgOutput& po = g.outs[k];
        o << "{\"kind\":\"" << (po.ref.kind == 0 ? "query" : "view") << "\",\"id\":" << po.ref.id
          << ",\"mode\":\"" << (po.mode == 0 ? "gemm" : po.mode == 1 ? "scatter" : "table")
          << "\",\"rows\":" << po.n_rows << "}";
      }
      o << "]}";
    }
    o << ",\"unique_views\":[";
    for (size_t k = 0; k < G.unique_views.size(); ++k) {
      if (k) o << ",";
      o << G.unique_views[k];
    }
    o << "]}";
  }
  o << "],\"levels\":" << P.n_levels << ",\"supported\":" << (P.supported ? "true" : "false");
  if (!P.supported) o << ",\"unsupported\":\"" << json_escape(P.unsupported_reason) << "\"";
  o << "}";
  return o.str();
}

static Plan* build_plan_once(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                             const lmfao_options* opts);

// With the ROOT_COST policy, a root assignment whose plan falls outside what
// the kernels support (EUNSUPPORTED) is replaced by the FACT roots.
Plan* build_plan(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                 const lmfao_options* opts) {
  if (!opts || opts->root_policy != LMFAO_ROOT_COST) return build_plan_once(schema, tree, batch, opts);
  try {
    return build_plan_once(schema, tree, batch, opts);
  } catch (const PlanError& e) {
    if (e.status != LMFAO_EUNSUPPORTED) throw;
    lmfao_options o = *opts;
    o.root_policy = LMFAO_ROOT_FACT;
    Plan* P = build_plan_once(schema, tree, batch, &o);
    P->opts.root_policy = LMFAO_ROOT_COST;
    P->root_fallback = e.msg;
    P->json = describe(*P);
    return P;
  }
}

static Plan* build_plan_once(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                             const lmfao_options* opts) {
  Plan* P = new Plan();
  try {
    if (opts) P->opts = *opts;
    else lmfao_default_options(&P->opts);
    if (P->opts.estimator && P->opts.estimator_len > 0) {
      const float* e = P->opts.estimator;
      const int64_t len = P->opts.estimator_len;
      if (len < 4 || e[0] != 2.f || e[1] != (float)LMFAO_EST_FEATURES || !(e[2] >= 1.f && e[2] <= 4096.f))
        throw PlanError{LMFAO_EINVAL, "estimator blob: bad header"};
      const int64_t d = LMFAO_EST_FEATURES, h = (int64_t)e[2];
      const int64_t n = d * h + h + h * h + h + h + 1;
      if (len != 4 + 2 * d + n) throw PlanError{LMFAO_EINVAL, "estimator blob: length does not match its header"};
      P->estimator.assign(e, e + len);
    }
    P->opts.estimator = nullptr;
    P->opts.estimator_len = 0;
    if (P->opts.precision < LMFAO_PREC_F64 || P->opts.precision > LMFAO_PREC_BF16X2)
      throw PlanError{LMFAO_EINVAL, "unknown precision"};
    if (P->opts.precision >= LMFAO_PREC_BF16X3 && P->opts.contraction != LMFAO_CONTRACT_MFMA)
      throw PlanError{LMFAO_EINVAL, "BF16 split precisions run the contraction on the matrix cores"};
    if (P->opts.scan_blocks < 0 || P->opts.contract_splits < 0 || P->opts.contract_splits > (1 << 20))
      throw PlanError{LMFAO_EINVAL, "scan_blocks and contract_splits must be 0 (automatic) or positive"};
    intake(*P, schema, tree, batch);
    if (P->rels.size() < 32 && (P->opts.row_weights >> P->rels.size()) != 0)
      throw PlanError{LMFAO_EINVAL, "row_weights names a relation the schema does not have"};
    compute_uniqueness(*P);
    generate_views(*P);
    view_layouts(*P);
    attribute_orders(*P);
    if (P->supported) build_programs(*P);
    P->json = describe(*P);
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

}  // namespace lmfao
