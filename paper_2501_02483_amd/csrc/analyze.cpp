// analyze.cpp -- host phases 1 and 2 of the three-phase sparse Cholesky
// (Section II): reordering (partial RCM with the fill check of Section III-A),
// symbolic factorization at tile granularity (CTSF tiles, Section III-B), and
// the construction and static scheduling of the task DAGs executed on the GPU
// (Algorithm 1 task types, Algorithm 2 progress counters, Algorithm 3 trees).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <queue>
#include <set>
#include <utility>

#include "symbolic.h"

using namespace stiles;

namespace {

thread_local int32_t g_err_arg = 0;

struct TaskBuilder {
  std::vector<int32_t> words;             // TASK_WORDS per task (succ/ndeps filled later)
  std::vector<std::vector<int32_t>> preds;
  std::vector<float> cost;
  std::vector<int32_t> late;   // the one predecessor waited for last (two-stage wait), or -1

  int add(int32_t type_flags, int32_t tile, int32_t a, int32_t b, int32_t c, float cst) {
    int id = (int)cost.size();
    int32_t w[TASK_WORDS] = {type_flags, tile, a, b, c, 0, 0, 0};
    words.insert(words.end(), w, w + TASK_WORDS);
    preds.emplace_back();
    cost.push_back(cst);
    late.push_back(-1);
    return id;
  }
  // two-stage wait: every other predecessor is waited for first
  void set_late(int task, int pred) {
    if (pred < 0) return;
    dep(task, pred);
    late[task] = pred;
    words[(size_t)task * TASK_WORDS] |= TF_SPLIT;
  }
  void dep(int task, int pred) {
    if (pred >= 0 && pred != task) preds[task].push_back(pred);
  }
};

// Start order of a list schedule on `workers` workers: whenever one is free
// it starts the ready task with the longest remaining path (bl); a task is
// ready `hop` after its last predecessor has finished.  The order is
// topological: a task starts only after its predecessors have finished.
std::vector<int32_t> list_order(int32_t nt, const float* cost, const int32_t* succ_ptr, const int32_t* succ,
                                const int32_t* npred_in, const float* bl, int workers, float hop) {
  std::vector<int32_t> order;
  order.reserve(nt);
  std::vector<int32_t> npred(npred_in, npred_in + nt);
  std::vector<float> rdy(nt, 0.f);
  typedef std::pair<float, int32_t> FI;
  std::priority_queue<FI, std::vector<FI>, std::greater<FI>> pending, running;   // by ready / finish time
  auto prio = [&](int32_t x, int32_t y) { return bl[x] != bl[y] ? bl[x] < bl[y] : x > y; };
  std::priority_queue<int32_t, std::vector<int32_t>, decltype(prio)> ready(prio);
  for (int32_t t = 0; t < nt; t++)
    if (npred[t] == 0) pending.push({0.f, t});
  float now = 0.f;
  int free_w = workers;
  while ((int32_t)order.size() < nt) {
    while (!pending.empty() && pending.top().first <= now) { ready.push(pending.top().second); pending.pop(); }
    while (free_w > 0 && !ready.empty()) {
      const int32_t t = ready.top();
      ready.pop();
      order.push_back(t);
      running.push({now + cost[t], t});
      free_w--;
    }
    float next = std::numeric_limits<float>::infinity();
    if (!running.empty()) next = running.top().first;
    if (free_w > 0 && !pending.empty()) next = std::min(next, pending.top().first);
    if (!(next < std::numeric_limits<float>::infinity())) { fprintf(stderr, "stiles: list schedule stalled\n"); abort(); }
    now = std::max(now, next);
    while (!running.empty() && running.top().first <= now) {
      const FI f = running.top();
      running.pop();
      free_w++;
      for (int32_t q = succ_ptr[f.second]; q < succ_ptr[f.second + 1]; q++) {
        const int32_t x = succ[q];
        rdy[x] = std::max(rdy[x], f.first + hop);
        if (--npred[x] == 0) pending.push({rdy[x], x});
      }
    }
  }
  return order;
}

// workgroups of the list schedule: a full-GPU executor launch has two per CU
// on 256 CUs; -1 (option) = unbounded earliest-start order
int sched_workers(const stiles_opts& o) { return o.sched_workers == 0 ? 512 : o.sched_workers < 0 ? 0 : o.sched_workers; }

// Static schedule: earliest start in an unbounded-resource model (hop latency
// on every edge), ties broken by longer remaining path, or (workers > 0) the
// start order of a list schedule on that many workgroups.  Tasks are
// renumbered in that order, which is topological; workgroups take them in
// this order.  est_out always receives the unbounded-resource estimate.
void schedule(TaskBuilder& tb, std::vector<int32_t>& tasks_out, std::vector<int32_t>& succ_out,
              std::vector<float>* est_out, std::vector<float>* cost_out, int workers) {
  const int nt = (int)tb.cost.size();
  const float hop = 0.8f;
  for (auto& p : tb.preds) {
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
  }
  // tasks were created in an order where every predecessor precedes its
  // successor; verify and compute est forward, bottom level backward.
  std::vector<float> est(nt, 0.f), bl(nt, 0.f);
  std::vector<std::vector<int32_t>> succ(nt);
  for (int t = 0; t < nt; t++) {
    float e = 0.f;
    for (int p : tb.preds[t]) {
      if (p >= t) { fprintf(stderr, "stiles: internal task order error\n"); abort(); }
      e = std::max(e, est[p] + tb.cost[p] + hop);
      succ[p].push_back(t);
    }
    est[t] = e;
  }
  for (int t = nt - 1; t >= 0; t--) {
    float b = 0.f;
    for (int s : succ[t]) b = std::max(b, bl[s] + hop);
    bl[t] = b + tb.cost[t];
  }
  std::vector<int32_t> order(nt);
  if (workers > 0) {
    // the list schedule pays off where the pivot chain bounds the run (the
    // critical path is at least half the work per workgroup); on DAGs with
    // far more work than chain (measured: n = 500,000, w = 1,000, ratio 4.2)
    // the earliest-start order is faster
    double tot = 0.0;
    float blmax = 0.f;
    for (int t = 0; t < nt; t++) { tot += tb.cost[t]; blmax = std::max(blmax, bl[t]); }
    if (tot / workers > 2.0 * blmax) workers = 0;
  }
  if (workers <= 0) {
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      if (est[x] != est[y]) return est[x] < est[y];
      return bl[x] > bl[y];
    });
  } else {
    std::vector<int32_t> sptr(nt + 1, 0), sflat, npred(nt);
    for (int t = 0; t < nt; t++) {
      sptr[t + 1] = sptr[t] + (int32_t)succ[t].size();
      sflat.insert(sflat.end(), succ[t].begin(), succ[t].end());
      npred[t] = (int32_t)tb.preds[t].size();
    }
    order = list_order(nt, tb.cost.data(), sptr.data(), sflat.data(), npred.data(), bl.data(), workers, hop);
  }
  std::vector<int32_t> newid(nt);
  for (int i = 0; i < nt; i++) newid[order[i]] = i;
  tasks_out.assign((size_t)nt * TASK_WORDS, 0);
  succ_out.clear();
  if (est_out) est_out->assign(nt, 0.f);
  if (cost_out) cost_out->assign(nt, 0.f);
  for (int i = 0; i < nt; i++) {
    int t = order[i];
    int32_t* w = &tasks_out[(size_t)i * TASK_WORDS];
    std::memcpy(w, &tb.words[(size_t)t * TASK_WORDS], sizeof(int32_t) * TASK_WORDS);
    w[5] = (int32_t)succ_out.size();
    // an edge into a two-stage task from one of its early predecessors
    // carries SUCC_FDEP (it subtracts MERGED_FDEP from the counter)
    std::vector<std::pair<int32_t, int32_t>> s;
    for (int x : succ[t]) s.push_back({newid[x], tb.late[x] >= 0 && tb.late[x] != t ? SUCC_FDEP : 0});
    std::sort(s.begin(), s.end());
    for (auto& e : s) succ_out.push_back(e.first | e.second);
    w[6] = (int32_t)succ_out.size();
    if (tb.late[t] >= 0) {
      const int32_t early = (int32_t)tb.preds[t].size() - 1;
      if (early >= (1 << 14)) { fprintf(stderr, "stiles: too many predecessors\n"); abort(); }
      w[7] = early * MERGED_FDEP + 1;
    } else {
      w[7] = (int32_t)tb.preds[t].size();
    }
    if (est_out) (*est_out)[i] = est[t];
    if (cost_out) (*cost_out)[i] = tb.cost[t];
  }
  // topological check of the final numbering
  for (int i = 0; i < nt; i++) {
    const int32_t* w = &tasks_out[(size_t)i * TASK_WORDS];
    for (int q = w[5]; q < w[6]; q++)
      if ((succ_out[q] & ~SUCC_FDEP) <= i) { fprintf(stderr, "stiles: schedule is not topological\n"); abort(); }
  }
}

// Chunks [lo, hi) of n products of a solve row that are ordered oldest first:
// the chunks nearest the diagonal step, whose blocks are solved last, hold
// c/4 and c/2 products (they run between two diagonal steps of the chain),
// the others c.
std::vector<std::pair<int32_t, int32_t>> chunk_bounds(int32_t n, int32_t c) {
  std::vector<std::pair<int32_t, int32_t>> out;
  int32_t hi = n;
  const int32_t tail[2] = {std::max(1, c / 4), std::max(1, c / 2)};
  for (int k = 0; hi > 0; k++) {
    const int32_t len = k < 2 ? tail[k] : c;
    const int32_t lo = std::max(0, hi - len);
    out.push_back({lo, hi});
    hi = lo;
  }
  std::reverse(out.begin(), out.end());
  return out;
}

inline int64_t tile_of_col(const stiles_symbolic& s, int64_t g) {
  return g < s.n ? g / s.T : s.ntb + (g - s.n) / s.T;
}

int32_t tile_lookup(const stiles_symbolic& s, int64_t m, int64_t j) {
  const int32_t* b = s.tcol.data() + s.trow_ptr[m];
  const int32_t* e = s.tcol.data() + s.trow_ptr[m + 1];
  const int32_t* p = std::lower_bound(b, e, (int32_t)j);
  if (p == e || *p != j) return -1;
  return (int32_t)(p - s.tcol.data());
}

// Reverse Cuthill-McKee on the band part (rows [0, n)) of a symmetric pattern
// given as adjacency lists; start nodes are pseudo-peripheral (George-Liu),
// neighbours visited by increasing degree, ties by lower index.
std::vector<int64_t> rcm_order(int64_t n, const std::vector<int64_t>& xadj, const std::vector<int64_t>& adj) {
  std::vector<int64_t> deg(n);
  for (int64_t v = 0; v < n; v++) deg[v] = xadj[v + 1] - xadj[v];
  std::vector<char> placed(n, 0);
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<int64_t> level(n, -1);
  auto bfs_levels = [&](int64_t root, std::vector<int64_t>& nodes, int64_t& ecc) {
    nodes.clear();
    nodes.push_back(root);
    level[root] = 0;
    size_t head = 0;
    ecc = 0;
    while (head < nodes.size()) {
      int64_t v = nodes[head++];
      for (int64_t q = xadj[v]; q < xadj[v + 1]; q++) {
        int64_t u = adj[q];
        if (level[u] < 0) { level[u] = level[v] + 1; ecc = std::max(ecc, level[u]); nodes.push_back(u); }
      }
    }
    for (int64_t u : nodes) level[u] = -1;
  };
  std::vector<int64_t> comp;
  for (int64_t s0 = 0; s0 < n; s0++) {
    if (placed[s0]) continue;
    // pseudo-peripheral node search
    int64_t root = s0, ecc = 0;
    bfs_levels(root, comp, ecc);
    for (int it = 0; it < 8; it++) {
      // last level: nodes at distance ecc; pick min degree (lowest index on ties)
      std::vector<int64_t> lvl_nodes;
      {
        std::vector<int64_t> nodes;
        int64_t e2;
        // recompute levels to find the last level
        nodes.push_back(root);
        level[root] = 0;
        size_t head = 0;
        while (head < nodes.size()) {
          int64_t v = nodes[head++];
          for (int64_t q = xadj[v]; q < xadj[v + 1]; q++) {
            int64_t u = adj[q];
            if (level[u] < 0) { level[u] = level[v] + 1; nodes.push_back(u); }
          }
        }
        for (int64_t u : nodes) if (level[u] == ecc) lvl_nodes.push_back(u);
        for (int64_t u : nodes) level[u] = -1;
        (void)e2;
      }
      int64_t best = lvl_nodes[0];
      for (int64_t u : lvl_nodes)
        if (deg[u] < deg[best] || (deg[u] == deg[best] && u < best)) best = u;
      int64_t ecc2;
      std::vector<int64_t> tmp;
      bfs_levels(best, tmp, ecc2);
      if (ecc2 > ecc) { root = best; ecc = ecc2; } else break;
    }
    // Cuthill-McKee from root
    size_t start = order.size();
    order.push_back(root);
    placed[root] = 1;
    size_t head = start;
    std::vector<int64_t> nb;
    while (head < order.size()) {
      int64_t v = order[head++];
      nb.clear();
      for (int64_t q = xadj[v]; q < xadj[v + 1]; q++)
        if (!placed[adj[q]]) nb.push_back(adj[q]);
      std::sort(nb.begin(), nb.end(), [&](int64_t x, int64_t y) {
        return deg[x] != deg[y] ? deg[x] < deg[y] : x < y;
      });
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      for (int64_t u : nb) { placed[u] = 1; order.push_back(u); }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Approximate minimum degree (Section III-A names it for irregular patterns;
// the method is Amestoy, Davis and Duff's).  Elimination runs on a quotient
// graph: an eliminated pivot becomes an element whose member list stands for
// the clique its elimination creates, so fill is never formed explicitly.
// Per principal variable i: its variable neighbours A_i and its elements E_i;
// per element e: its member variables L_e and their total weight |L_e|.
// Variables that become indistinguishable (same A and E after a step) are
// merged into supervariables of weight nv and are ordered together.  A
// variable's external degree is replaced by the bound
//   d_i = min(n_left - nv_i, d_i(old) + |L_p \ i|,
//             |A_i \ i| + |L_p \ i| + sum over e in E_i, e != p, of |L_e \ L_p|)
// with |L_e \ L_p| from one pass over the members of L_p; an element with
// |L_e \ L_p| = 0 lies inside L_p and is absorbed.  Pivots are taken by
// smallest bound, ties by lowest index.  Returns the elimination order of
// the n band rows (the arrow rows are not part of the graph: they stay last).
std::vector<int64_t> amd_order(int64_t n, const std::vector<int64_t>& xadj, const std::vector<int64_t>& adj) {
  enum : char { VAR = 0, MERGED = 1, ELEM = 2, GONE = 3 };
  std::vector<char> st(n, VAR);
  std::vector<int64_t> nv(n, 1), deg(n), esize(n, 0), w(n, 0), wmark(n, -1), mark(n, -1);
  std::vector<std::vector<int64_t>> A(n), E(n), Lm(n), members(n);
  for (int64_t i = 0; i < n; i++) {
    for (int64_t q = xadj[i]; q < xadj[i + 1]; q++)
      if (adj[q] != i) A[i].push_back(adj[q]);
    std::sort(A[i].begin(), A[i].end());
    A[i].erase(std::unique(A[i].begin(), A[i].end()), A[i].end());
    deg[i] = (int64_t)A[i].size();
  }
  std::set<std::pair<int64_t, int64_t>> heap;
  for (int64_t i = 0; i < n; i++) heap.insert({deg[i], i});
  std::vector<int64_t> order;
  order.reserve(n);
  int64_t left = n, stamp = 0;
  std::vector<int64_t> Lp;
  while (!heap.empty()) {
    const int64_t p = heap.begin()->second;
    heap.erase(heap.begin());
    // order p's supervariable (p and the variables merged into it)
    {
      std::vector<int64_t> stack{p};
      while (!stack.empty()) {
        int64_t v = stack.back();
        stack.pop_back();
        order.push_back(v);
        for (int64_t c : members[v]) stack.push_back(c);
      }
    }
    left -= nv[p];
    // L_p: p's variable neighbours and the members of its elements, which
    // p absorbs
    const int64_t sp = ++stamp;
    mark[p] = sp;
    Lp.clear();
    int64_t lp_w = 0;
    auto add = [&](int64_t j) {
      if (st[j] == VAR && mark[j] != sp) { mark[j] = sp; Lp.push_back(j); lp_w += nv[j]; }
    };
    for (int64_t j : A[p]) add(j);
    for (int64_t e : E[p]) {
      if (st[e] != ELEM) continue;
      for (int64_t j : Lm[e]) add(j);
      st[e] = GONE;
      std::vector<int64_t>().swap(Lm[e]);
    }
    st[p] = ELEM;
    std::vector<int64_t>().swap(A[p]);
    std::vector<int64_t>().swap(E[p]);
    Lm[p] = Lp;
    esize[p] = lp_w;
    // |L_e \ L_p| for every other element next to a member of L_p
    const int64_t sw = ++stamp;
    for (int64_t i : Lp)
      for (int64_t e : E[i]) {
        if (st[e] != ELEM || e == p) continue;
        if (wmark[e] != sw) { wmark[e] = sw; w[e] = esize[e]; }
        w[e] -= nv[i];
      }
    // new element and variable lists, degree bounds
    for (int64_t i : Lp) {
      heap.erase({deg[i], i});
      std::vector<int64_t>& Ei = E[i];
      int64_t ew = 0;
      size_t k = 0;
      for (int64_t e : Ei) {
        if (st[e] != ELEM || e == p) continue;
        if (wmark[e] == sw && w[e] == 0) { st[e] = GONE; std::vector<int64_t>().swap(Lm[e]); continue; }
        ew += wmark[e] == sw ? w[e] : esize[e];
        Ei[k++] = e;
      }
      Ei.resize(k);
      Ei.push_back(p);
      std::vector<int64_t>& Ai = A[i];
      int64_t aw = 0;
      k = 0;
      for (int64_t j : Ai) {
        if (st[j] != VAR || mark[j] == sp) continue;   // eliminated, merged, p, or in L_p
        aw += nv[j];
        Ai[k++] = j;
      }
      Ai.resize(k);
      const int64_t ext = lp_w - nv[i];
      int64_t d = aw + ext + ew;
      d = std::min(d, deg[i] + ext);
      d = std::min(d, left - nv[i]);
      deg[i] = std::max<int64_t>(d, 0);
    }
    // the elements absorbed above may still be listed by members of L_p
    // processed before them: drop them
    for (int64_t i : Lp) {
      std::vector<int64_t>& Ei = E[i];
      Ei.erase(std::remove_if(Ei.begin(), Ei.end(), [&](int64_t e) { return st[e] != ELEM; }), Ei.end());
    }
    // supervariables: members of L_p with equal A and E lists merge
    std::vector<std::pair<uint64_t, int64_t>> h;
    h.reserve(Lp.size());
    for (int64_t i : Lp) {
      std::sort(A[i].begin(), A[i].end());
      std::sort(E[i].begin(), E[i].end());
      uint64_t x = 1469598103934665603ull;
      for (int64_t j : A[i]) x = (x ^ (uint64_t)j) * 1099511628211ull;
      x = (x ^ 0x9e3779b97f4a7c15ull) * 1099511628211ull;
      for (int64_t e : E[i]) x = (x ^ (uint64_t)e) * 1099511628211ull;
      h.push_back({x, i});
    }
    std::sort(h.begin(), h.end());
    for (size_t a = 0; a < h.size();) {
      size_t b = a;
      while (b < h.size() && h[b].first == h[a].first) b++;
      for (size_t u = a; u < b; u++) {
        const int64_t i = h[u].second;
        if (st[i] != VAR) continue;
        for (size_t v = u + 1; v < b; v++) {
          const int64_t j = h[v].second;
          if (st[j] != VAR || A[i] != A[j] || E[i] != E[j]) continue;
          nv[i] += nv[j];
          deg[i] -= nv[j];
          nv[j] = 0;
          st[j] = MERGED;
          members[i].push_back(j);
          std::vector<int64_t>().swap(A[j]);
          std::vector<int64_t>().swap(E[j]);
        }
      }
      a = b;
    }
    for (int64_t i : Lp)
      if (st[i] == VAR) {
        deg[i] = std::max<int64_t>(0, std::min(deg[i], left - nv[i]));
        heap.insert({deg[i], i});
      }
    // L_p keeps its principal variables
    std::vector<int64_t>& L = Lm[p];
    L.erase(std::remove_if(L.begin(), L.end(), [&](int64_t j) { return st[j] != VAR; }), L.end());
  }
  return order;
}

// Postorder of the elimination tree of the band graph under `ord` (new
// position -> node): every subtree becomes a contiguous run of rows, which
// keeps the fill and the work of the order and groups the rows that couple
// into the same tiles.  Tree from Liu's row-subtree walk with path
// compression; children visited in increasing order.
std::vector<int64_t> etree_postorder(int64_t n, const std::vector<int64_t>& xadj, const std::vector<int64_t>& adj,
                                     const std::vector<int64_t>& ord) {
  std::vector<int64_t> pos(n), parent(n, -1), anc(n, -1);
  for (int64_t i = 0; i < n; i++) pos[ord[i]] = i;
  for (int64_t i = 0; i < n; i++) {
    const int64_t v = ord[i];
    for (int64_t q = xadj[v]; q < xadj[v + 1]; q++) {
      int64_t r = pos[adj[q]];
      if (r >= i) continue;
      while (anc[r] != -1 && anc[r] != i) {
        const int64_t t = anc[r];
        anc[r] = i;
        r = t;
      }
      if (anc[r] == -1) { anc[r] = i; parent[r] = i; }
    }
  }
  std::vector<int64_t> head(n, -1), next(n, -1);
  for (int64_t i = n - 1; i >= 0; i--)
    if (parent[i] >= 0) { next[i] = head[parent[i]]; head[parent[i]] = i; }
  std::vector<int64_t> out, stack;
  out.reserve(n);
  for (int64_t root = 0; root < n; root++) {
    if (parent[root] != -1) continue;
    stack.push_back(root);
    while (!stack.empty()) {
      const int64_t v = stack.back();
      if (head[v] >= 0) {           // descend into the next unvisited child
        const int64_t c = head[v];
        head[v] = next[c];
        stack.push_back(c);
      } else {
        out.push_back(ord[v]);
        stack.pop_back();
      }
    }
  }
  return out;
}

// Tile-level symbolic factorization: the tile columns of L from those of A
// (a_cols[j]: tile rows >= j holding entries of tile column j).  Column j
// of L is its own pattern merged with those of its children in the tile
// elimination tree (the parent of j is the first off-diagonal tile row of
// column j of L).
std::vector<std::vector<int32_t>> tile_columns(const std::vector<std::vector<int32_t>>& a_cols) {
  const int32_t ntr = (int32_t)a_cols.size();
  std::vector<std::vector<int32_t>> lcol(ntr);
  std::vector<std::vector<int32_t>> children(ntr);
  for (int32_t j = 0; j < ntr; j++) {
    std::vector<int32_t> c = a_cols[j];
    for (int32_t ch : children[j]) {
      for (int32_t r : lcol[ch]) if (r != ch) c.push_back(r);
    }
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    // rows >= j only, diagonal present
    c.erase(std::remove_if(c.begin(), c.end(), [&](int32_t r) { return r < j; }), c.end());
    if (c.empty() || c[0] != j) c.insert(c.begin(), j);
    lcol[j] = c;
    if (c.size() > 1) children[c[1]].push_back(j);
  }
  return lcol;
}

// Number of tiles of L when the band rows of a CSC pattern are renumbered by
// inv (old index -> new index; the arrow rows stay last): band tile rows of T
// rows, then the arrow's.  The fill measure of the ordering check for
// orderings that do not keep a band shape.
int64_t l_tiles_for(int64_t N, int64_t n, int32_t T, const int64_t* colptr, const int64_t* rowind,
                    const std::vector<int64_t>& inv) {
  const int64_t ntb = (n + T - 1) / T;
  const int32_t ntr = (int32_t)(ntb + (N - n + T - 1) / T);
  auto tile = [&](int64_t g) { return (int32_t)(g < n ? g / T : ntb + (g - n) / T); };
  std::vector<std::vector<int32_t>> a_cols(ntr);
  for (int32_t m = 0; m < ntr; m++) a_cols[m].push_back(m);
  for (int64_t j = 0; j < N; j++)
    for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
      const int64_t p = inv[rowind[q]], c = inv[j];
      a_cols[tile(std::min(p, c))].push_back(tile(std::max(p, c)));
    }
  for (auto& c : a_cols) { std::sort(c.begin(), c.end()); c.erase(std::unique(c.begin(), c.end()), c.end()); }
  int64_t tot = 0;
  for (const auto& c : tile_columns(a_cols)) tot += (int64_t)c.size();
  return tot;
}

// number of tiles in the tile envelope of a lower profile f over the band part
// (the arrow tile rows are dense and identical for every band ordering)
int64_t envelope_tiles(const std::vector<int64_t>& f, int64_t n, int32_t T) {
  int64_t ntb = (n + T - 1) / T, tot = 0;
  for (int64_t m = 0; m < ntb; m++) {
    int64_t F = m;
    for (int64_t i = m * T; i < std::min<int64_t>(n, (m + 1) * T); i++) F = std::min<int64_t>(F, f[i] / T);
    tot += m - F + 1;
  }
  return tot;
}

// ------------------------------------------------------------ adaptable ND
// Adaptable nested dissection (Section III-A).  The band part is cut into P
// contiguous parts B_1..B_P by separators S_1..S_{P-1}: blocks of consecutive
// rows such that no band row after S_j has its first column before S_j (the
// separator is as wide as the local bandwidth).  The separators move behind
// the parts, ahead of the arrow, and join it; the parts keep their band shape
// and have no dependencies between them, so their tile-column chains run
// concurrently.  The last part is reversed, so that its separator meets its
// last columns instead of filling across it (an interior part touches two
// separators and the one met first still fills across it: the thicker arrow
// of the paper's second partition; interior parts are oriented so that this
// is the narrower of the two).  Parts before the last are whole
// tile rows and separators are padded to whole tile rows, so no tile mixes
// two blocks.
struct Seg {
  int64_t olo, ohi, nlo;   // original rows [olo, ohi) go to new rows from nlo
  bool rev;                // in reverse order
};

inline int64_t seg_new(const Seg& g, int64_t o) { return g.rev ? g.nlo + (g.ohi - 1 - o) : g.nlo + (o - g.olo); }

struct NDPlan {
  int32_t P = 1;
  std::vector<int64_t> part_lo, part_hi, sep_lo, sep_hi;   // original rows
  int64_t chain = 0;      // tile steps on the longest dependency chain (estimate)
};

// need[c]: rows a separator starting at row c must span so that no later band
// row couples to a row before c (0 if nothing couples across c)
std::vector<int64_t> separator_need(const std::vector<int64_t>& f, int64_t n) {
  std::vector<int64_t> H(n + 1, -1);
  for (int64_t i = 0; i < n; i++) H[f[i]] = std::max(H[f[i]], i);
  std::vector<int64_t> need(n + 1, 0);
  int64_t g = -1;   // last row whose first column is < c
  for (int64_t c = 0; c <= n; c++) {
    if (c > 0) g = std::max(g, H[c - 1]);
    need[c] = std::max<int64_t>(0, g + 1 - c);
  }
  return need;
}

// Cut points for P parts: each cut is searched in a window around the point
// that balances the remaining rows, minimizing separator tile rows plus half
// the imbalance (in tile rows).
bool nd_plan_for(const std::vector<int64_t>& need, int64_t n, int64_t arrow, int32_t T, int32_t P, NDPlan& out) {
  if (P < 2 || n < (int64_t)P * 2 * T) return false;
  auto padded = [&](int64_t c) { return (need[c] + T - 1) / T * T; };
  // typical separator: median padded need over the band (sampled)
  std::vector<int64_t> smp;
  for (int64_t c = T; c < n; c += std::max<int64_t>(T, n / 256)) smp.push_back(padded(c));
  if (smp.empty()) return false;
  std::nth_element(smp.begin(), smp.begin() + smp.size() / 2, smp.end());
  const int64_t sp_typ = smp[smp.size() / 2];
  NDPlan pl;
  pl.P = P;
  int64_t start = 0;
  for (int32_t j = 0; j < P - 1; j++) {
    const int32_t left = P - j;
    int64_t Lt = (n - start - (left - 1) * sp_typ) / left;
    Lt = std::max<int64_t>(T, (Lt + T / 2) / T * T);
    const int64_t ideal = start + Lt;
    const int64_t W = std::max<int64_t>(T, (Lt / 4) / T * T);
    int64_t best = -1;
    double bestcost = 1e300;
    for (int64_t c = std::max(start + T, ideal - W); c <= ideal + W && c < n; c += T) {
      const int64_t sp = padded(c);
      if (c + sp + (int64_t)(left - 1) * T > n) continue;   // room for the parts after it
      const double cost = (double)sp / T + 0.5 * std::fabs((double)(c - ideal)) / T;
      if (cost < bestcost) { bestcost = cost; best = c; }
    }
    if (best < 0) return false;
    const int64_t sp = padded(best);
    pl.part_lo.push_back(start);
    pl.part_hi.push_back(best);
    pl.sep_lo.push_back(best);
    pl.sep_hi.push_back(best + sp);
    start = best + sp;
  }
  if (n - start < T) return false;
  pl.part_lo.push_back(start);
  pl.part_hi.push_back(n);
  int64_t longest = 0;
  for (int32_t j = 0; j < P; j++) longest = std::max(longest, (pl.part_hi[j] - pl.part_lo[j] + T - 1) / T);
  // separators: one bisection level after another, each level as deep as
  // its widest separator
  int64_t seps = 0;
  {
    std::vector<std::pair<int32_t, int32_t>> level{{0, P - 1}};
    while (!level.empty()) {
      std::vector<std::pair<int32_t, int32_t>> next;
      int64_t widest = 0;
      for (auto& r : level) {
        if (r.first >= r.second) continue;
        const int32_t mid = r.first + (r.second - r.first) / 2;
        widest = std::max(widest, (pl.sep_hi[mid] - pl.sep_lo[mid]) / T);
        next.push_back({r.first, mid});
        next.push_back({mid + 1, r.second});
      }
      seps += widest;
      level.swap(next);
    }
  }
  pl.chain = longest + seps + (arrow + T - 1) / T;
  out = pl;
  return true;
}

// requested P >= 2: that many parts (else the automatic choice); 0: the
// fewest parts whose estimated chain is within 1.3x of the shortest one over
// P in [2, 64].  Every interior part adds a separator's width of fill across
// its columns (executed work grows with P while the chain shrinks), so once
// the chain is near its floor fewer parts are preferred -- except for small
// matrices (under 2e9 flops), which take the shortest chain.  False when no
// cut is feasible.
bool nd_plan(const std::vector<int64_t>& f, int64_t n, int64_t arrow, int32_t T, int32_t P_req, NDPlan& out) {
  const std::vector<int64_t> need = separator_need(f, n);
  if (P_req >= 2 && nd_plan_for(need, n, arrow, T, P_req, out)) return true;
  std::vector<NDPlan> plans;
  int64_t best = -1;
  for (int32_t P = 2; P <= 64; P++) {
    NDPlan pl;
    if (!nd_plan_for(need, n, arrow, T, P, pl)) break;
    if (best < 0 || pl.chain < best) best = pl.chain;
    plans.push_back(std::move(pl));
  }
  // a small matrix is bound by its chain alone (its extra fill costs next to
  // nothing): take the shortest chain
  double work = 0.0;
  for (int64_t i = 0; i < n; i++) {
    const double e = (double)(i - f[i] + 1 + arrow);
    work += e * e;
  }
  const bool tiny = work < 2e9;
  for (const NDPlan& pl : plans)
    if (tiny ? pl.chain == best : 10 * pl.chain <= 13 * best) { out = pl; return true; }
  return false;
}

// separators in nested-dissection order: after the parts are eliminated the
// separators couple as a chain (S_j to S_(j+1) through the part between
// them); ordering the chain by a balanced bisection tree, children before
// parents, makes its dependency depth logarithmic in the number of parts
void bisection_postorder(int32_t lo, int32_t hi, std::vector<int32_t>& out) {
  if (lo >= hi) return;
  const int32_t mid = lo + (hi - lo) / 2;
  bisection_postorder(lo, mid, out);
  bisection_postorder(mid + 1, hi, out);
  out.push_back(mid);
}

// new-order segments of a plan: parts (the last reversed), separators in
// bisection post-order, arrow
std::vector<Seg> nd_segments(const NDPlan& pl, int64_t n, int64_t N, int64_t* band_rows) {
  std::vector<Seg> sg;
  int64_t pos = 0;
  for (int32_t j = 0; j < pl.P; j++) {
    // the first part keeps its order (its separator is at its end), the last
    // is reversed; an interior part is ordered so that its narrower
    // separator is the one met first (that one fills across the part)
    bool rev = j == pl.P - 1;
    if (j > 0 && j + 1 < pl.P) rev = (pl.sep_hi[j] - pl.sep_lo[j]) < (pl.sep_hi[j - 1] - pl.sep_lo[j - 1]);
    sg.push_back({pl.part_lo[j], pl.part_hi[j], pos, rev});
    pos += pl.part_hi[j] - pl.part_lo[j];
  }
  *band_rows = pos;
  std::vector<int32_t> sep_order;
  bisection_postorder(0, pl.P - 1, sep_order);
  for (int32_t j : sep_order)
    if (pl.sep_hi[j] > pl.sep_lo[j]) {
      sg.push_back({pl.sep_lo[j], pl.sep_hi[j], pos, false});
      pos += pl.sep_hi[j] - pl.sep_lo[j];
    }
  if (N > n) sg.push_back({n, N, pos, false});
  return sg;
}

// partition of every band tile row of the new order (the first P segments
// of nd_segments are the partitions; all but the last are whole tile rows)
void set_band_part(stiles_symbolic& s, const std::vector<Seg>& segs, int32_t P) {
  s.band_part.assign(s.ntb, 0);
  for (int32_t j = 0; j < P; j++) {
    const int64_t lo = segs[j].nlo, hi = segs[j].nlo + (segs[j].ohi - segs[j].olo);
    if (hi <= lo) continue;
    for (int64_t t = lo / s.T; t <= (hi - 1) / s.T && t < s.ntb; t++) s.band_part[t] = j;
  }
}

// Profile and tile pattern of P A P^T for a row-profile input (row i spans
// columns [fin_i, i]) under a segment permutation: every row interval maps
// to a few new intervals, split at the diagonal into a row part and a column
// part (entries that land above the diagonal are stored transposed).
void permuted_profile(stiles_symbolic& s, std::vector<Seg> segs, const std::vector<int64_t>& fin,
                      std::vector<std::vector<int32_t>>& a_cols) {
  const int64_t N = s.N;
  std::sort(segs.begin(), segs.end(), [](const Seg& x, const Seg& y) { return x.olo < y.olo; });
  s.f.resize(N);
  for (int64_t p = 0; p < N; p++) s.f[p] = p;
  a_cols.assign(s.ntr, {});
  size_t gi = 0;
  for (int64_t i = 0; i < N; i++) {
    while (segs[gi].ohi <= i) gi++;
    const int64_t p = seg_new(segs[gi], i);
    const int64_t tp = tile_of_col(s, p);
    size_t k = gi;
    while (k > 0 && segs[k].olo > fin[i]) k--;
    for (; k < segs.size() && segs[k].olo <= i; k++) {
      const Seg& g = segs[k];
      const int64_t x = std::max(fin[i], g.olo), y = std::min(i, g.ohi - 1);
      if (x > y) continue;
      const int64_t u = seg_new(g, g.rev ? y : x), v = seg_new(g, g.rev ? x : y);
      if (u <= p) {
        const int64_t hi = std::min(v, p);
        s.f[p] = std::min(s.f[p], u);
        for (int64_t tc = tile_of_col(s, u); tc <= tile_of_col(s, hi); tc++) a_cols[tc].push_back((int32_t)tp);
      }
      if (v > p) {
        const int64_t lo = std::max(u, p + 1);
        for (int64_t q = lo; q <= v; q++) s.f[q] = std::min(s.f[q], p);
        for (int64_t tr = tile_of_col(s, lo); tr <= tile_of_col(s, v); tr++) a_cols[tp].push_back((int32_t)tr);
      }
    }
  }
  for (auto& c : a_cols) { std::sort(c.begin(), c.end()); c.erase(std::unique(c.begin(), c.end()), c.end()); }
}

// sum_j (eta_j + 1)^2 over the element envelope of a lower profile f
double envelope_flops(const std::vector<int64_t>& f) {
  const int64_t N = (int64_t)f.size();
  std::vector<int64_t> d(N + 1, 0);
  for (int64_t i = 0; i < N; i++) { d[f[i]] += 1; d[i] -= 1; }
  double F = 0.0;
  int64_t run = 0;
  for (int64_t j = 0; j < N; j++) {
    run += d[j];          // rows i > j with f_i <= j
    const double e = (double)run + 1.0;
    F += e * e;
  }
  return F;
}

stiles_status check_opts(const stiles_opts* o, int arg) {
  if (!o) return STILES_OK;
  if (o->tile != 0 && o->tile != 32 && o->tile != 64) { g_err_arg = arg; return STILES_ENOTSUP; }
  if (o->ordering < STILES_ORDER_AUTO || o->ordering > STILES_ORDER_AMD) { g_err_arg = arg; return STILES_EINVAL; }
  if (o->nd_parts < 0 || o->nd_parts > 64) { g_err_arg = arg; return STILES_EINVAL; }
  if (o->chunk < 0 || o->chunk > 32 || o->refine_max_iter < 0 || o->refine_tol < 0) { g_err_arg = arg; return STILES_EINVAL; }
  if (o->sched_workers < -1 || o->sched_workers > 65536) { g_err_arg = arg; return STILES_EINVAL; }
  if (o->ublock < -1 || o->ublock > 15) { g_err_arg = arg; return STILES_EINVAL; }
  return STILES_OK;
}

void finish_symbolic(stiles_symbolic& s, const std::vector<std::vector<int32_t>>& a_cols);

}  // namespace

namespace stiles {
void set_error_arg(int32_t idx) { g_err_arg = idx; }

std::vector<int32_t> tiles_with_entries(const stiles_symbolic& s) {
  const int64_t TT = (int64_t)s.T * s.T;
  std::vector<int32_t> has(s.ntiles, 0);
  for (int32_t m = 0; m < s.ntr; m++) has[s.trow_ptr[m + 1] - 1] = 1;   // diagonal tile (last of its row)
  if (!s.profile_input) {
    for (int64_t o : s.map) has[o / TT] = 1;
    return has;
  }
  if (s.perm_identity) {
    // the stored tiles are those of the envelope itself
    std::fill(has.begin(), has.end(), 1);
    return has;
  }
  // row-profile input under a permutation: input row o holds columns
  // [fin[o], o]; the new positions of a range of input indices are followed
  // in runs on which the inverse permutation steps by +1 or -1
  const int64_t N = s.N;
  std::vector<int64_t> pinv(N), run_end(N);
  for (int64_t r = 0; r < N; r++) pinv[s.perm[r]] = r;
  for (int64_t c = N - 1; c >= 0; c--) {
    const int64_t d = c + 1 < N ? pinv[c + 1] - pinv[c] : 0;
    run_end[c] = (d == 1 || d == -1) ? run_end[c + 1] : c;   // consecutive unit steps share their sign
  }
  auto tile_row = [&](int64_t g) {
    return (int32_t)(std::upper_bound(s.row_base.begin(), s.row_base.end(), g) - s.row_base.begin() - 1);
  };
  int32_t last_tr = -1, last_lo = -1, last_hi = -1;
  for (int64_t o = 0; o < N; o++) {
    const int32_t tr = tile_row(pinv[o]);
    for (int64_t c0 = s.fin[o]; c0 <= o;) {
      const int64_t e = std::min(run_end[c0], o);
      const int32_t ta = tile_row(pinv[c0]), tb2 = tile_row(pinv[e]);
      const int32_t lo = std::min(ta, tb2), hi = std::max(ta, tb2);
      c0 = e + 1;
      if (tr == last_tr && lo == last_lo && hi == last_hi) continue;
      last_tr = tr;
      last_lo = lo;
      last_hi = hi;
      for (int32_t tc = lo; tc <= hi; tc++) {
        const int32_t t = tile_lookup(s, std::max(tr, tc), std::min(tr, tc));
        if (t >= 0) has[t] = 1;
      }
    }
  }
  return has;
}
std::vector<int32_t> list_schedule(int32_t nt, const float* cost, const int32_t* succ_ptr, const int32_t* succ,
                                   const int32_t* npred, const float* bl, int workers, float hop) {
  return list_order(nt, cost, succ_ptr, succ, npred, bl, workers, hop);
}
int schedule_workers(const stiles_opts& o) { return sched_workers(o); }
}

extern "C" int32_t stiles_last_error_arg(void) { return g_err_arg; }

extern "C" void stiles_default_opts(stiles_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tile = 64;
  o->ordering = STILES_ORDER_AUTO;
  o->tree_min_ratio = 2;
  o->chunk = 0;
  o->refine_tol = 0.0;
  o->refine_max_iter = 0;
}

static void init_common(stiles_symbolic& s, int64_t N, int64_t a, const stiles_opts* opts) {
  if (opts) s.opts = *opts; else stiles_default_opts(&s.opts);
  if (s.opts.tile == 0) s.opts.tile = 64;
  s.T = s.opts.tile;
  s.N = N;
  s.a = a;
  s.n = N - a;
  s.ntb = (int32_t)((s.n + s.T - 1) / s.T);
  s.nta = (int32_t)((s.a + s.T - 1) / s.T);
  s.ntr = s.ntb + s.nta;
  s.row_base.resize(s.ntr);
  s.row_cnt.resize(s.ntr);
  for (int32_t m = 0; m < s.ntr; m++) {
    if (m < s.ntb) {
      s.row_base[m] = (int64_t)m * s.T;
      s.row_cnt[m] = (int32_t)std::min<int64_t>(s.T, s.n - (int64_t)m * s.T);
    } else {
      s.row_base[m] = s.n + (int64_t)(m - s.ntb) * s.T;
      s.row_cnt[m] = (int32_t)std::min<int64_t>(s.T, s.a - (int64_t)(m - s.ntb) * s.T);
    }
  }
}

namespace {

// Automatic partition count (adaptable ND with nd_parts = 0): the
// chain-based choice P0 (see nd_plan) and two smaller counts are analyzed
// in full, and the one with the least estimated time is kept.  The estimate
// is the larger of the plan's chain (tile steps) times a step's duration
// and its executed flops over the executor's executed rate (measured on
// MI355X: a pivot step about 50 us at T = 64, 30 us at T = 32; about 34 and
// 17.5 TFLOP/s executed): long narrow bands are bound by their chain, for
// which P0 is made, wide bands by the fill that every interior partition
// adds, which fewer partitions save.  Small matrices keep P0.
template <typename Fn>
stiles_status analyze_auto_parts(const stiles_opts* opts, Fn analyze_with, stiles_symbolic** out) {
  stiles_status st = analyze_with(opts, out);
  if (st != STILES_OK || !opts || opts->ordering != STILES_ORDER_ADAPTABLE_ND || opts->nd_parts != 0) return st;
  stiles_symbolic* best = *out;
  if (best->nd_parts < 4 || best->flops_alg < 2e9) return st;
  auto estimate = [](const stiles_symbolic* s) {
    const double step = s->T == 64 ? 50e-6 : 30e-6, rate = s->T == 64 ? 34e12 : 17.5e12;
    return std::max((double)s->nd_chain * step, s->flops_exec / rate);
  };
  double best_t = estimate(best);
  const int32_t P0 = best->nd_parts;
  const int32_t cand[2] = {(int32_t)std::lround(0.6 * P0), (int32_t)std::lround(0.4 * P0)};
  for (int32_t P : cand) {
    if (P < 2 || P >= P0) continue;
    stiles_opts o2 = *opts;
    o2.nd_parts = P;
    stiles_symbolic* c = nullptr;
    if (analyze_with(&o2, &c) != STILES_OK || !c) continue;
    const double t = estimate(c);
    if (c->nd_parts == P && t < best_t) {
      stiles_symbolic_destroy(best);
      best = c;
      best_t = t;
    } else {
      stiles_symbolic_destroy(c);
    }
  }
  *out = best;
  g_err_arg = 0;
  return STILES_OK;
}

stiles_status analyze_profile_impl(int64_t n_band, int64_t arrow, const int64_t* first_col, const stiles_opts* opts,
                                   stiles_symbolic** out);
stiles_status analyze_csc_impl(int64_t N, int64_t arrow, const int64_t* colptr, const int64_t* rowind,
                               const stiles_opts* opts, stiles_symbolic** out);

}  // namespace

extern "C" stiles_status stiles_analyze_profile(int64_t n_band, int64_t arrow, const int64_t* first_col,
                                                const stiles_opts* opts, stiles_symbolic** out) {
  return analyze_auto_parts(opts, [&](const stiles_opts* o, stiles_symbolic** r) {
    return analyze_profile_impl(n_band, arrow, first_col, o, r);
  }, out);
}

extern "C" stiles_status stiles_analyze(int64_t N, int64_t arrow, const int64_t* colptr, const int64_t* rowind,
                                        const stiles_opts* opts, stiles_symbolic** out) {
  return analyze_auto_parts(opts, [&](const stiles_opts* o, stiles_symbolic** r) {
    return analyze_csc_impl(N, arrow, colptr, rowind, o, r);
  }, out);
}

namespace {

stiles_status analyze_profile_impl(int64_t n_band, int64_t arrow, const int64_t* first_col, const stiles_opts* opts,
                                   stiles_symbolic** out) {
  g_err_arg = 0;
  if (n_band < 0) { g_err_arg = 1; return STILES_EINVAL; }
  if (arrow < 0 || n_band + arrow < 1) { g_err_arg = 2; return STILES_EINVAL; }
  if (n_band > 0 && !first_col) { g_err_arg = 3; return STILES_EINVAL; }
  for (int64_t i = 0; i < n_band; i++)
    if (first_col[i] < 0 || first_col[i] > i) { g_err_arg = 3; return STILES_EINVAL; }
  stiles_status st = check_opts(opts, 4);
  if (st != STILES_OK) return st;
  if (opts && (opts->ordering == STILES_ORDER_PARTIAL_RCM || opts->ordering == STILES_ORDER_AMD)) {
    g_err_arg = 4;
    return STILES_ENOTSUP;
  }
  if (!out) { g_err_arg = 5; return STILES_EINVAL; }
  const int64_t N = n_band + arrow;
  if ((N + 63) / 16 > INT32_MAX / 4) { g_err_arg = 1; return STILES_ENOTSUP; }
  stiles_symbolic* s = new stiles_symbolic();
  init_common(*s, N, arrow, opts);
  s->a_in = arrow;
  s->profile_input = true;
  s->ordering_used = STILES_ORDER_NONE;
  if (s->opts.ordering == STILES_ORDER_ADAPTABLE_ND && n_band > 0) {
    std::vector<int64_t> fin(N, 0);
    for (int64_t i = 0; i < n_band; i++) fin[i] = first_col[i];
    NDPlan pl;
    if (nd_plan(fin, n_band, arrow, s->T, s->opts.nd_parts, pl)) {
      int64_t nb2 = 0;
      const std::vector<Seg> segs = nd_segments(pl, n_band, N, &nb2);
      init_common(*s, N, N - nb2, opts);   // the separators join the arrow
      s->ordering_used = STILES_ORDER_ADAPTABLE_ND;
      s->nd_parts = pl.P;
      s->nd_chain = pl.chain;
      set_band_part(*s, segs, pl.P);
      s->perm_identity = false;
      s->perm.resize(N);
      for (const Seg& g : segs)
        for (int64_t o = g.olo; o < g.ohi; o++) s->perm[seg_new(g, o)] = o;
      s->iperm.resize(N);
      for (int64_t i = 0; i < N; i++) s->iperm[s->perm[i]] = i;
      s->in_rp_in.resize(N + 1);
      s->in_rp_in[0] = 0;
      for (int64_t i = 0; i < N; i++) s->in_rp_in[i + 1] = s->in_rp_in[i] + (i - fin[i] + 1);
      std::vector<std::vector<int32_t>> a_cols;
      permuted_profile(*s, segs, fin, a_cols);
      s->f_pre = fin;
      s->fin = std::move(fin);
      s->in_rp.resize(N + 1);
      s->in_rp[0] = 0;
      for (int64_t i = 0; i < N; i++) s->in_rp[i + 1] = s->in_rp[i] + (i - s->f[i] + 1);
      finish_symbolic(*s, a_cols);
      *out = s;
      return STILES_OK;
    }
  }
  s->perm.resize(N);
  std::iota(s->perm.begin(), s->perm.end(), 0);
  s->iperm = s->perm;
  s->f.resize(N);
  for (int64_t i = 0; i < n_band; i++) s->f[i] = first_col[i];
  for (int64_t i = n_band; i < N; i++) s->f[i] = 0;
  s->in_rp.resize(N + 1);
  s->in_rp[0] = 0;
  for (int64_t i = 0; i < N; i++) s->in_rp[i + 1] = s->in_rp[i] + (i - s->f[i] + 1);
  // tile pattern of A: band tile row m holds tiles F_m..m, arrow rows 0..m
  std::vector<std::vector<int32_t>> a_cols(s->ntr);  // column lists: rows m >= j
  for (int32_t m = 0; m < s->ntr; m++) {
    int64_t F = m;
    if (m < s->ntb) {
      for (int64_t i = s->row_base[m]; i < s->row_base[m] + s->row_cnt[m]; i++)
        F = std::min<int64_t>(F, tile_of_col(*s, s->f[i]));
    } else {
      F = 0;
    }
    for (int64_t j = F; j <= m; j++) a_cols[j].push_back(m);
  }
  finish_symbolic(*s, a_cols);
  *out = s;
  return STILES_OK;
}

stiles_status analyze_csc_impl(int64_t N, int64_t arrow, const int64_t* colptr, const int64_t* rowind,
                               const stiles_opts* opts, stiles_symbolic** out) {
  g_err_arg = 0;
  if (N < 1) { g_err_arg = 1; return STILES_EINVAL; }
  if (arrow < 0 || arrow > N) { g_err_arg = 2; return STILES_EINVAL; }
  if (!colptr || colptr[0] != 0) { g_err_arg = 3; return STILES_EINVAL; }
  for (int64_t j = 0; j < N; j++)
    if (colptr[j + 1] < colptr[j] + 1) { g_err_arg = 3; return STILES_EINVAL; }
  const int64_t nnz = colptr[N];
  if (!rowind) { g_err_arg = 4; return STILES_EINVAL; }
  for (int64_t j = 0; j < N; j++) {
    if (rowind[colptr[j]] != j) { g_err_arg = 4; return STILES_EINVAL; }  // diagonal first
    for (int64_t q = colptr[j] + 1; q < colptr[j + 1]; q++)
      if (rowind[q] <= rowind[q - 1] || rowind[q] >= N) { g_err_arg = 4; return STILES_EINVAL; }
  }
  stiles_status st = check_opts(opts, 5);
  if (st != STILES_OK) return st;
  if (!out) { g_err_arg = 6; return STILES_EINVAL; }
  stiles_symbolic* s = new stiles_symbolic();
  init_common(*s, N, arrow, opts);
  s->a_in = arrow;
  s->profile_input = false;
  const int64_t n = s->n;
  // profile of the identity ordering
  std::vector<int64_t> f_id(N);
  for (int64_t i = 0; i < N; i++) f_id[i] = i;
  for (int64_t j = 0; j < N; j++)
    for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) f_id[rowind[q]] = std::min(f_id[rowind[q]], j);
  std::vector<int64_t> perm(N);
  std::iota(perm.begin(), perm.end(), 0);
  s->ordering_used = STILES_ORDER_NONE;
  if (s->opts.ordering != STILES_ORDER_NONE && n > 2) {
    // symmetric adjacency of the band part (partial permutation: arrow excluded)
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t j = 0; j < n; j++)
      for (int64_t q = colptr[j] + 1; q < colptr[j + 1]; q++)
        if (rowind[q] < n) { deg[j]++; deg[rowind[q]]++; }
    std::vector<int64_t> xadj(n + 1, 0);
    for (int64_t v = 0; v < n; v++) xadj[v + 1] = xadj[v] + deg[v];
    std::vector<int64_t> fillp(xadj.begin(), xadj.end() - 1), adj(xadj[n]);
    for (int64_t j = 0; j < n; j++)
      for (int64_t q = colptr[j] + 1; q < colptr[j + 1]; q++)
        if (rowind[q] < n) { adj[fillp[j]++] = rowind[q]; adj[fillp[rowind[q]]++] = j; }
    if (s->opts.ordering == STILES_ORDER_AMD) {
      // approximate minimum degree, kept only if L has fewer tiles than in
      // the input order (the fill check); no band shape is kept, so the
      // partitions of adaptable ND are not offered on top of it
      std::vector<int64_t> ord = etree_postorder(n, xadj, adj, amd_order(n, xadj, adj));
      std::vector<int64_t> inv(N), id(N);
      for (int64_t i = 0; i < n; i++) inv[ord[i]] = i;
      for (int64_t i = n; i < N; i++) inv[i] = i;
      std::iota(id.begin(), id.end(), 0);
      if (l_tiles_for(N, n, s->T, colptr, rowind, inv) < l_tiles_for(N, n, s->T, colptr, rowind, id)) {
        for (int64_t i = 0; i < n; i++) perm[i] = ord[i];
        s->ordering_used = STILES_ORDER_AMD;
      }
    } else {
      std::vector<int64_t> ord = rcm_order(n, xadj, adj);
      std::vector<int64_t> inv(N);
      for (int64_t i = 0; i < n; i++) inv[ord[i]] = i;
      for (int64_t i = n; i < N; i++) inv[i] = i;
      std::vector<int64_t> f_r(N);
      for (int64_t i = 0; i < N; i++) f_r[i] = i;
      for (int64_t j = 0; j < N; j++)
        for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
          int64_t p = inv[rowind[q]], c = inv[j];
          int64_t hi = std::max(p, c), lo = std::min(p, c);
          f_r[hi] = std::min(f_r[hi], lo);
        }
      bool use = s->opts.ordering == STILES_ORDER_PARTIAL_RCM;
      if (s->opts.ordering == STILES_ORDER_AUTO || s->opts.ordering == STILES_ORDER_ADAPTABLE_ND)
        use = envelope_tiles(f_r, n, s->T) < envelope_tiles(f_id, n, s->T);   // fill check
      if (use) {
        for (int64_t i = 0; i < n; i++) perm[i] = ord[i];
        s->ordering_used = STILES_ORDER_PARTIAL_RCM;
      }
    }
  }
  if (s->opts.ordering == STILES_ORDER_ADAPTABLE_ND && n > 0) {
    // band profile under the ordering so far, then the partition plan on it
    std::vector<int64_t> inv(N);
    for (int64_t i = 0; i < N; i++) inv[perm[i]] = i;
    std::vector<int64_t> fcur(N);
    for (int64_t i = 0; i < N; i++) fcur[i] = i;
    for (int64_t j = 0; j < N; j++)
      for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
        int64_t p = inv[rowind[q]], c = inv[j];
        int64_t hi = std::max(p, c), lo = std::min(p, c);
        fcur[hi] = std::min(fcur[hi], lo);
      }
    NDPlan pl;
    if (nd_plan(fcur, n, arrow, s->T, s->opts.nd_parts, pl)) {
      int64_t nb2 = 0;
      const std::vector<Seg> segs = nd_segments(pl, n, N, &nb2);
      std::vector<int64_t> np(N);
      for (const Seg& g : segs)
        for (int64_t o = g.olo; o < g.ohi; o++) np[seg_new(g, o)] = perm[o];
      perm.swap(np);
      init_common(*s, N, N - nb2, opts);   // the separators join the arrow
      s->ordering_used = STILES_ORDER_ADAPTABLE_ND;
      s->nd_parts = pl.P;
      s->nd_chain = pl.chain;
      set_band_part(*s, segs, pl.P);
      s->f_pre = std::move(fcur);
    }
  }
  s->perm = perm;
  s->iperm.resize(N);
  for (int64_t i = 0; i < N; i++) s->iperm[perm[i]] = i;
  s->perm_identity = true;
  for (int64_t i = 0; i < N && s->perm_identity; i++) s->perm_identity = perm[i] == i;
  s->f.assign(N, 0);
  for (int64_t i = 0; i < N; i++) s->f[i] = i;
  for (int64_t j = 0; j < N; j++)
    for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
      int64_t p = s->iperm[rowind[q]], c = s->iperm[j];
      int64_t hi = std::max(p, c), lo = std::min(p, c);
      s->f[hi] = std::min(s->f[hi], lo);
    }
  // tile pattern of A from the entries actually present
  std::vector<std::vector<int32_t>> a_cols(s->ntr);
  for (int32_t m = 0; m < s->ntr; m++) a_cols[m].push_back(m);
  for (int64_t j = 0; j < N; j++)
    for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
      int64_t p = s->iperm[rowind[q]], c = s->iperm[j];
      int64_t hi = std::max(p, c), lo = std::min(p, c);
      a_cols[tile_of_col(*s, lo)].push_back((int32_t)tile_of_col(*s, hi));
    }
  for (auto& c : a_cols) { std::sort(c.begin(), c.end()); c.erase(std::unique(c.begin(), c.end()), c.end()); }
  s->in_rp.resize(N + 1);
  s->in_rp[0] = 0;
  for (int64_t i = 0; i < N; i++) s->in_rp[i + 1] = s->in_rp[i] + (i - s->f[i] + 1);
  finish_symbolic(*s, a_cols);
  // value index -> element offset in the tile store
  s->map.resize(nnz);
  const int64_t TT = (int64_t)s->T * s->T;
  for (int64_t j = 0; j < N; j++)
    for (int64_t q = colptr[j]; q < colptr[j + 1]; q++) {
      int64_t p = s->iperm[rowind[q]], c = s->iperm[j];
      int64_t hi = std::max(p, c), lo = std::min(p, c);
      int64_t tm = tile_of_col(*s, hi), tj = tile_of_col(*s, lo);
      int32_t t = tile_lookup(*s, tm, tj);
      s->map[q] = (int64_t)t * TT + (lo - s->row_base[tj]) * s->T + (hi - s->row_base[tm]);
    }
  *out = s;
  return STILES_OK;
}

}  // namespace

namespace {

void finish_symbolic(stiles_symbolic& s, const std::vector<std::vector<int32_t>>& a_cols) {
  const int32_t ntr = s.ntr, T = s.T;
  // ---- tile-level symbolic factorization (elimination tree, column merge)
  const std::vector<std::vector<int32_t>> lcol = tile_columns(a_cols);
  // ---- row lists
  std::vector<int32_t> rcount(ntr, 0);
  for (int32_t j = 0; j < ntr; j++) for (int32_t r : lcol[j]) rcount[r]++;
  s.trow_ptr.assign(ntr + 1, 0);
  for (int32_t m = 0; m < ntr; m++) s.trow_ptr[m + 1] = s.trow_ptr[m] + rcount[m];
  s.ntiles = s.trow_ptr[ntr];
  s.tcol.assign(s.ntiles, 0);
  s.trow.assign(s.ntiles, 0);
  {
    std::vector<int32_t> fillp(s.trow_ptr.begin(), s.trow_ptr.end() - 1);
    for (int32_t j = 0; j < ntr; j++)
      for (int32_t r : lcol[j]) { s.tcol[fillp[r]] = j; s.trow[fillp[r]] = r; fillp[r]++; }
  }
  // column lists with tile ids (ascending row)
  std::vector<std::vector<std::pair<int32_t, int32_t>>> ctiles(ntr);
  for (int32_t m = 0; m < ntr; m++)
    for (int32_t t = s.trow_ptr[m]; t < s.trow_ptr[m + 1]; t++) ctiles[s.tcol[t]].push_back({m, t});

  // ---- statistics over the element envelope
  s.nnzL = 0;
  for (int64_t i = 0; i < s.N; i++) s.nnzL += i - s.f[i] + 1;
  s.nnzL_alg = s.nnzL;
  if (!s.f_pre.empty()) {
    s.nnzL_alg = 0;
    for (int64_t i = 0; i < s.N; i++) s.nnzL_alg += i - s.f_pre[i] + 1;
  }
  {
    const std::vector<int64_t>& fb = s.f_pre.empty() ? s.f : s.f_pre;
    s.w_in = 0;
    for (int64_t i = 0; i < s.N - s.a_in; i++) s.w_in = std::max<int64_t>(s.w_in, i - fb[i]);
  }
  s.flops_alg = envelope_flops(s.f_pre.empty() ? s.f : s.f_pre);

  // ---- factorization DAG
  const int32_t chunk = s.opts.chunk > 0 ? s.opts.chunk : (T == 64 ? 12 : 16);
  const double t3 = std::pow((double)T / 64.0, 3.0);
  TaskBuilder tb;
  std::vector<int32_t> final_task(s.ntiles, -1);
  std::vector<int32_t> pairs;
  s.npart = 0;
  s.tree_used = 0;
  s.corner_acc = 0;
  double fexec = 0.0;
  const double T3 = (double)T * T * T;
  // 2 x 2 blocks of update targets: band columns k, k+1 (the same partition,
  // tile (k+1, k) stored) and two tile rows ra < rb.  A block task computes
  // the four updates C_(r,c) -= sum_j L_(r,j) L_(c,j)^T, r in {ra, rb},
  // c in {k, k+1}, over a chunk of the columns j <= k-2, reading each
  // operand tile once for (up to) two products: a band tile column update is
  // a tall-skinny product, and pairing two rows and two columns halves the
  // operand reads per product.  The block covers every product of its
  // targets with a column j <= k-2 (a target whose operand tile at some j is
  // absent skips that column).  The diagonal block (ra, rb) = (k, k+1) has
  // three targets, (k,k), (k+1,k), (k+1,k+1), and two operand tiles per
  // column.  What is left of a target's products: column k-1 (fused into
  // its POTRF/TRSM for column k; for column k+1, together with column k,
  // fused into its TRSM, or an update task of its own when the target is on
  // the pivot chain -- the diagonal tile (k+1,k+1) and the panel (k+2,k+1)).
  const int32_t bchunk = s.opts.ublock > 0 ? s.opts.ublock : 0;
  struct UBlock {
    int32_t k, ra, rb;
    int32_t tgt[4];   // (ra,k), (rb,k), (ra,k+1), (rb,k+1); -1 if absent
    std::vector<int32_t> J;
  };
  std::vector<UBlock> blocks;
  std::vector<int32_t> tblock(s.ntiles, -1);
  std::vector<std::vector<int32_t>> col_blocks(ntr);
  if (bchunk > 0) {
    for (int32_t k = 0; k + 1 < s.ntb;) {
      const bool same = s.nd_parts <= 1 || s.band_part.empty() || s.band_part[k] == s.band_part[k + 1];
      if (!same || tile_lookup(s, k + 1, k) < 0) { k++; continue; }
      std::vector<int32_t> rows;
      for (auto& mt : ctiles[k]) if (mt.first > k + 1) rows.push_back(mt.first);
      for (auto& mt : ctiles[k + 1]) if (mt.first > k + 1) rows.push_back(mt.first);
      std::sort(rows.begin(), rows.end());
      rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
      std::vector<std::pair<int32_t, int32_t>> cand{{k, k + 1}};
      for (size_t q = 0; q + 1 < rows.size(); q += 2) cand.push_back({rows[q], rows[q + 1]});
      for (auto [ra, rb] : cand) {
        UBlock b;
        b.k = k; b.ra = ra; b.rb = rb;
        const bool dg = ra == k;
        b.tgt[0] = tile_lookup(s, ra, k);
        b.tgt[1] = tile_lookup(s, rb, k);
        b.tgt[2] = dg ? -1 : tile_lookup(s, ra, k + 1);
        b.tgt[3] = tile_lookup(s, rb, k + 1);
        // the columns j <= k-2 of the targets' products
        std::vector<int32_t> J;
        int ntg = 0;
        for (int q = 0; q < 4; q++) {
          if (b.tgt[q] < 0) continue;
          const int32_t m = q & 1 ? rb : ra, c = q < 2 ? k : k + 1;
          const size_t before = J.size();
          int32_t p = s.trow_ptr[m], pe = s.trow_ptr[m + 1], r = s.trow_ptr[c], re = s.trow_ptr[c + 1];
          while (p < pe && r < re) {
            const int32_t cm = s.tcol[p], cc = s.tcol[r];
            if (cm > k - 2 || cc > k - 2) break;
            if (cm == cc) { J.push_back(cm); p++; r++; }
            else if (cm < cc) p++;
            else r++;
          }
          if (J.size() == before) b.tgt[q] = -1;   // no product in the block's columns
          else ntg++;
        }
        std::sort(J.begin(), J.end());
        J.erase(std::unique(J.begin(), J.end()), J.end());
        if (ntg < 2 || J.size() < 2) continue;
        b.J = std::move(J);
        const int32_t id = (int32_t)blocks.size();
        for (int32_t t : b.tgt) if (t >= 0) tblock[t] = id;
        col_blocks[k].push_back(id);
        blocks.push_back(std::move(b));
      }
      k += 2;
    }
  }
  s.ublocks = (int64_t)blocks.size();
  // the update chain of every tile (the last task that wrote it)
  std::vector<int32_t> tlast(s.ntiles, -1);
  // products (tile (m,j), tile (c,j)), j < c, of target tile (m, c), ascending j
  auto products = [&](int32_t m, int32_t c, std::vector<std::pair<int32_t, int32_t>>& pr, std::vector<int32_t>& pj) {
    pr.clear();
    pj.clear();
    int32_t p = s.trow_ptr[m], pe = s.trow_ptr[m + 1];
    int32_t q = s.trow_ptr[c], qe = s.trow_ptr[c + 1] - 1;   // exclude the diagonal tile (c,c)
    while (p < pe && q < qe) {
      int32_t cm = s.tcol[p], ck = s.tcol[q];
      if (cm >= c) break;
      if (cm == ck) { pr.push_back({p, q}); pj.push_back(cm); p++; q++; }
      else if (cm < ck) p++;
      else q++;
    }
  };
  // ordinary update chunks of a target over products [lo, hi) of pr
  auto upd_chain = [&](int32_t tgt, bool diag, const std::vector<std::pair<int32_t, int32_t>>& pr, size_t lo0,
                       size_t hi0, std::vector<int32_t>& pairs_out) {
    for (size_t lo = lo0; lo < hi0; lo += chunk) {
      size_t hi = std::min(hi0, lo + chunk);
      int32_t p0 = (int32_t)(pairs_out.size() / 2);
      for (size_t q = lo; q < hi; q++) { pairs_out.push_back(pr[q].first); pairs_out.push_back(pr[q].second); }
      int32_t p1 = (int32_t)(pairs_out.size() / 2);
      float c = 0.5f + (diag ? 1.35f : 1.8f) * (float)(t3 * (hi - lo));
      int t = tb.add(TK_UPD | (diag ? TF_DIAG : 0), tgt, p0, p1, 0, c);
      fexec += (diag ? 1.5 : 2.0) * T3 * (hi - lo);
      for (size_t q = lo; q < hi; q++) { tb.dep(t, final_task[pr[q].first]); tb.dep(t, final_task[pr[q].second]); }
      tb.dep(t, tlast[tgt]);
      tlast[tgt] = t;
    }
  };
  std::vector<std::pair<int32_t, int32_t>> pr;  // (tile m j, tile k j) ascending j
  std::vector<int32_t> pj;
  for (int32_t k = 0; k < ntr; k++) {
    int32_t potrf_task = -1;
    if (!col_blocks[k].empty()) {
      // the block tasks: chunks of the block's columns, oldest first; the two
      // most recent chunks (their columns are final last, close to the pivot
      // chain) hold one and two columns
      for (int32_t bi : col_blocks[k]) {
        const UBlock& b = blocks[bi];
        const bool dg = b.ra == k;
        const int32_t nJ = (int32_t)b.J.size();
        std::vector<std::pair<int32_t, int32_t>> ch;
        {
          int32_t hi = nJ;
          const int32_t tail[2] = {1, 2};
          for (int q = 0; hi > 0; q++) {
            int32_t len = q < 2 ? tail[q] : bchunk;
            if (q >= 2) {
              // the rest in nearly equal chunks of at most bchunk
              const int32_t nc = (hi + bchunk - 1) / bchunk;
              for (int32_t ci = nc - 1; ci >= 0; ci--) ch.push_back({(int32_t)((int64_t)hi * ci / nc), (int32_t)((int64_t)hi * (ci + 1) / nc)});
              break;
            }
            const int32_t lo = std::max(0, hi - len);
            ch.push_back({lo, hi});
            hi = lo;
          }
          std::reverse(ch.begin(), ch.end());
        }
        for (auto [lo, hi] : ch) {
          const int32_t p0 = (int32_t)(pairs.size() / 2);
          for (int q = 0; q < 4; q++) pairs.push_back(b.tgt[q]);
          std::vector<int32_t> ops;
          double prods = 0.0, fl = 0.0;
          for (int32_t x = lo; x < hi; x++) {
            const int32_t j = b.J[x];
            const int32_t yk = tile_lookup(s, k, j), yk1 = tile_lookup(s, k + 1, j);
            const int32_t xa = dg ? yk : tile_lookup(s, b.ra, j), xb = dg ? yk1 : tile_lookup(s, b.rb, j);
            const int32_t o[4] = {xa, xb, yk, yk1};
            for (int q = 0; q < 4; q++) {
              pairs.push_back(o[q]);
              if (o[q] >= 0) ops.push_back(o[q]);
            }
            for (int q = 0; q < 4; q++) {
              if (b.tgt[q] < 0 || o[q & 1] < 0 || o[2 + (q >> 1)] < 0) continue;
              const bool td = dg && q != 1;
              prods += 1.0;
              fl += (td ? 1.5 : 2.0) * T3;
            }
          }
          int t = tb.add(TK_UPDB | (dg ? TF_DIAG : 0), -1, p0, hi - lo, 0, 0.5f + 1.4f * (float)(t3 * prods));
          fexec += fl;
          for (int32_t o : ops) tb.dep(t, final_task[o]);
          for (int q = 0; q < 4; q++)
            if (b.tgt[q] >= 0) tb.dep(t, tlast[b.tgt[q]]);
          for (int q = 0; q < 4; q++)
            if (b.tgt[q] >= 0) tlast[b.tgt[q]] = t;
        }
      }
    }
    for (auto& mt : ctiles[k]) {
      const int32_t m = mt.first, tgt = mt.second;
      if (tblock[tgt] >= 0) {
        // a block target: its products with columns after k-2 of its block
        // (block column kb = blocks[..].k): column k-1 when the target is in
        // column kb, columns kb-1 and kb when it is in column kb+1
        const UBlock& b = blocks[tblock[tgt]];
        products(m, k, pr, pj);
        std::vector<std::pair<int32_t, int32_t>> rest;
        for (size_t q = 0; q < pr.size(); q++)
          if (pj[q] > b.k - 2) rest.push_back(pr[q]);
        const bool diag = (m == k);
        // on the pivot chain: the diagonal tile and the panel below it
        const bool chain = diag || m == k + 1;
        // fused into the finalizer: the last product, and for an off-chain
        // TRSM the one before it as well
        size_t nfuse = rest.empty() ? 0 : 1;
        if (!diag && !chain && rest.size() >= 2) nfuse = 2;
        if (rest.size() > nfuse) {
          // (at most one product here; a chain target's column k-2)
          upd_chain(tgt, diag, rest, 0, rest.size() - nfuse, pairs);
        }
        int32_t f0 = (int32_t)(pairs.size() / 2), f1 = f0;
        for (size_t q = rest.size() - nfuse; q < rest.size(); q++) {
          pairs.push_back(rest[q].first);
          pairs.push_back(rest[q].second);
          f1++;
          fexec += 2.0 * T3;
        }
        if (diag) {
          int t = tb.add(TK_POTRF, tgt, k, f0, f1, (T == 64 ? 10.f : 4.f) + (f1 > f0 ? 1.5f * (float)t3 : 0.f));
          fexec += 2.0 * T3 / 3.0;
          tb.dep(t, tlast[tgt]);
          for (size_t q = rest.size() - nfuse; q < rest.size(); q++) {
            tb.dep(t, final_task[rest[q].first]);
            tb.dep(t, final_task[rest[q].second]);
          }
          if (nfuse > 0) tb.set_late(t, final_task[rest.back().first]);
          potrf_task = t;
          final_task[tgt] = t;
        } else {
          int t = tb.add(TK_TRSM, tgt, k, f0, f1, 0.5f + 1.8f * (float)t3 * (float)(1 + (f1 - f0)));
          fexec += 2.0 * T3;
          tb.set_late(t, potrf_task);
          tb.dep(t, tlast[tgt]);
          for (size_t q = rest.size() - nfuse; q < rest.size(); q++) {
            tb.dep(t, final_task[rest[q].first]);
            tb.dep(t, final_task[rest[q].second]);
          }
          final_task[tgt] = t;
        }
        continue;
      }
      // pairs (m,j),(k,j), j < k, both present
      products(m, k, pr, pj);
      const bool diag = (m == k);
      int32_t last = -1;
      size_t start = 0;
      const bool corner = (m >= s.ntb && k >= s.ntb);
      // a tile of the arrow corner proper (the arrow's own tile rows, after
      // the separators that adaptable ND adds to the corner): its partial
      // products stay FP64 in mixed mode
      const int32_t arrow0 = ntr - (int32_t)((s.a_in + T - 1) / T);
      const int32_t arrow_flag = (m >= arrow0 && k >= arrow0) ? TF_ARROW : 0;
      if (corner) {
        size_t nb = 0;
        while (nb < pr.size() && pj[nb] < s.ntb) nb++;
        s.corner_acc = std::max<int64_t>(s.corner_acc, (int64_t)nb);
        const int64_t G = ((int64_t)nb + chunk - 1) / chunk;
        // under adaptable ND the band products of a corner tile come from
        // several partitions, which progress concurrently: one chain of
        // partial products per partition (each chunk as soon as its columns
        // are final), then a binary tree over the partitions' partials.  A
        // tile fed by a single partition is updated by a plain chain.
        std::vector<std::pair<size_t, size_t>> groups;
        if (s.nd_parts > 1 && !s.band_part.empty())
          for (size_t q = 0; q < nb;) {
            size_t e = q;
            while (e < nb && s.band_part[pj[e]] == s.band_part[pj[q]]) e++;
            groups.push_back({q, e});
            q = e;
          }
        if (s.nd_parts > 1 && groups.size() >= 2 && s.opts.tree_min_ratio > 0) {
          s.tree_used = 1;
          std::vector<std::pair<int32_t, int32_t>> level;   // (slot, last task of its chain)
          for (auto& gr : groups) {
            const int32_t slot = s.npart++;
            int prev = -1;
            for (size_t lo = gr.first; lo < gr.second; lo += chunk) {
              size_t hi = std::min(gr.second, lo + chunk);
              int32_t p0 = (int32_t)(pairs.size() / 2);
              for (size_t q = lo; q < hi; q++) { pairs.push_back(pr[q].first); pairs.push_back(pr[q].second); }
              int32_t p1 = (int32_t)(pairs.size() / 2);
              int t = tb.add(TK_PART | (prev >= 0 ? TF_ACC : 0) | arrow_flag, -1, p0, p1, slot,
                             0.5f + 1.8f * (float)(t3 * (hi - lo)));
              fexec += 2.0 * T3 * (hi - lo);
              for (size_t q = lo; q < hi; q++) { tb.dep(t, final_task[pr[q].first]); tb.dep(t, final_task[pr[q].second]); }
              tb.dep(t, prev);
              prev = t;
            }
            level.push_back({slot, prev});
          }
          while (level.size() > 2) {
            std::vector<std::pair<int32_t, int32_t>> next;
            for (size_t q = 0; q + 1 < level.size(); q += 2) {
              int32_t slot = s.npart++;
              int t = tb.add(TK_TREE, -1, level[q].first, level[q + 1].first, slot, 0.5f);
              tb.dep(t, level[q].second);
              tb.dep(t, level[q + 1].second);
              next.push_back({slot, t});
            }
            if (level.size() % 2) next.push_back(level.back());
            level.swap(next);
          }
          int t = tb.add(TK_TREE | (diag ? TF_DIAG : 0), tgt, level[0].first, level[1].first, -1, 0.5f);
          tb.dep(t, level[0].second);
          tb.dep(t, level[1].second);
          last = t;
          start = nb;
        } else if (s.nd_parts > 1) {
          // one partition (or none): the plain chain below
        } else if (s.opts.tree_min_ratio > 0 && G >= 2 && (int64_t)nb >= (int64_t)s.opts.tree_min_ratio * G) {
          s.tree_used = 1;
          // leaves: PART tasks over contiguous ranges of band columns (Alg. 3)
          std::vector<std::pair<int32_t, int32_t>> level;   // (slot, producing task)
          for (int64_t g = 0; g < G; g++) {
            size_t lo = (size_t)(g * chunk), hi = std::min(nb, (size_t)((g + 1) * chunk));
            int32_t p0 = (int32_t)(pairs.size() / 2);
            for (size_t q = lo; q < hi; q++) { pairs.push_back(pr[q].first); pairs.push_back(pr[q].second); }
            int32_t p1 = (int32_t)(pairs.size() / 2);
            int32_t slot = s.npart++;
            int t = tb.add(TK_PART | arrow_flag, -1, p0, p1, slot, 0.5f + 1.8f * (float)(t3 * (hi - lo)));
            fexec += 2.0 * T3 * (hi - lo);
            for (size_t q = lo; q < hi; q++) { tb.dep(t, final_task[pr[q].first]); tb.dep(t, final_task[pr[q].second]); }
            level.push_back({slot, t});
          }
          // binary GEADD tree in index order; the root subtracts into the target
          while (level.size() > 2) {
            std::vector<std::pair<int32_t, int32_t>> next;
            for (size_t q = 0; q + 1 < level.size(); q += 2) {
              int32_t slot = s.npart++;
              int t = tb.add(TK_TREE, -1, level[q].first, level[q + 1].first, slot, 0.5f);
              tb.dep(t, level[q].second);
              tb.dep(t, level[q + 1].second);
              next.push_back({slot, t});
            }
            if (level.size() % 2) next.push_back(level.back());
            level.swap(next);
          }
          int t = tb.add(TK_TREE | (diag ? TF_DIAG : 0), tgt, level[0].first, level[1].first, -1, 0.5f);
          tb.dep(t, level[0].second);
          tb.dep(t, level[1].second);
          last = t;
          start = nb;
        }
      }
      // corner tiles: the products over arrow and separator columns become
      // available only as the separators are factored, and an arrow row
      // meets every separator.  When there are many, they are independent
      // partial products (each as soon as its columns are final) summed by a
      // binary tree in index order, instead of a sequential chain of updates
      if (corner && s.opts.tree_min_ratio > 0) {
        const bool fl = pr.size() > start && pj.back() == k - 1;
        // the last `chunk` products (the most recent columns, on the pivot
        // chain) stay in an update task after the tree
        const size_t be = (fl ? pr.size() - 1 : pr.size()) - std::min(pr.size() - (fl ? 1 : 0), (size_t)chunk);
        if (be > start && be - start > (size_t)(2 * chunk)) {
          s.tree_used = 1;
          std::vector<std::pair<int32_t, int32_t>> level;   // (slot, producing task)
          for (size_t lo = start; lo < be; lo += chunk) {
            const size_t hi = std::min(be, lo + chunk);
            int32_t p0 = (int32_t)(pairs.size() / 2);
            for (size_t q = lo; q < hi; q++) { pairs.push_back(pr[q].first); pairs.push_back(pr[q].second); }
            int32_t p1 = (int32_t)(pairs.size() / 2);
            const int32_t slot = s.npart++;
            int t = tb.add(TK_PART | arrow_flag, -1, p0, p1, slot, 0.5f + 1.8f * (float)(t3 * (hi - lo)));
            fexec += 2.0 * T3 * (hi - lo);
            for (size_t q = lo; q < hi; q++) { tb.dep(t, final_task[pr[q].first]); tb.dep(t, final_task[pr[q].second]); }
            level.push_back({slot, t});
          }
          while (level.size() > 2) {
            std::vector<std::pair<int32_t, int32_t>> next;
            for (size_t q = 0; q + 1 < level.size(); q += 2) {
              int32_t slot = s.npart++;
              int t = tb.add(TK_TREE, -1, level[q].first, level[q + 1].first, slot, 0.5f);
              tb.dep(t, level[q].second);
              tb.dep(t, level[q + 1].second);
              next.push_back({slot, t});
            }
            if (level.size() % 2) next.push_back(level.back());
            level.swap(next);
          }
          // be - start > 2 chunk gives at least three leaves, so two partials remain
          int t = tb.add(TK_TREE | (diag ? TF_DIAG : 0), tgt, level[0].first, level[1].first, -1, 0.5f);
          tb.dep(t, level[0].second);
          tb.dep(t, level[1].second);
          tb.dep(t, last);   // after the band tree's subtraction from the same tile
          last = t;
          start = be;
        }
      }
      // chunks of `chunk` products in ascending column order; the product
      // with column k-1 (available last, on the critical path) is fused into
      // the task that finalizes the tile (POTRF or TRSM), so that everything
      // before it runs ahead (lookahead) and the chain has one hop less
      const bool fuse_last = pr.size() > start && pj.back() == k - 1;
      const size_t body_end = fuse_last ? pr.size() - 1 : pr.size();
      for (size_t lo = start; lo < body_end; lo += chunk) {
        size_t hi = std::min(body_end, lo + chunk);
        int32_t p0 = (int32_t)(pairs.size() / 2);
        for (size_t q = lo; q < hi; q++) { pairs.push_back(pr[q].first); pairs.push_back(pr[q].second); }
        int32_t p1 = (int32_t)(pairs.size() / 2);
        float c = 0.5f + (diag ? 1.35f : 1.8f) * (float)(t3 * (hi - lo));
        int t = tb.add(TK_UPD | (diag ? TF_DIAG : 0), tgt, p0, p1, 0, c);
        fexec += (diag ? 1.5 : 2.0) * T3 * (hi - lo);
        for (size_t q = lo; q < hi; q++) { tb.dep(t, final_task[pr[q].first]); tb.dep(t, final_task[pr[q].second]); }
        tb.dep(t, last);
        last = t;
      }
      int32_t f0 = (int32_t)(pairs.size() / 2), f1 = f0;
      if (fuse_last) {
        pairs.push_back(pr.back().first);
        pairs.push_back(pr.back().second);
        f1 = f0 + 1;
        fexec += 2.0 * T3;
      }
      if (diag) {
        int t = tb.add(TK_POTRF, tgt, k, f0, f1, (T == 64 ? 10.f : 4.f) + (f1 > f0 ? 1.5f * (float)t3 : 0.f));
        fexec += 2.0 * T3 / 3.0;
        tb.dep(t, last);
        if (fuse_last) {
          tb.dep(t, final_task[pr.back().first]);
          tb.dep(t, final_task[pr.back().second]);
          tb.set_late(t, final_task[pr.back().first]);   // the panel of column k-1
        }
        potrf_task = t;
        final_task[tgt] = t;
      } else {
        // the diagonal tile (k,k) comes first in the column list
        int t = tb.add(TK_TRSM, tgt, k, f0, f1, 0.5f + 1.8f * (float)t3 * (f1 > f0 ? 2.f : 1.f));
        fexec += 2.0 * T3;
        tb.set_late(t, potrf_task);
        tb.dep(t, last);
        if (fuse_last) { tb.dep(t, final_task[pr.back().first]); tb.dep(t, final_task[pr.back().second]); }
        final_task[tgt] = t;
      }
    }
  }
  s.flops_exec = fexec;
  s.fpairs = pairs;
  schedule(tb, s.ftask, s.fsucc, &s.fest, &s.fcost, sched_workers(s.opts));

  // ---- solve DAG (forward then backward sweep over tile rows)
  TaskBuilder sb;
  std::vector<int32_t> sp;
  const int32_t schunk = T == 64 ? 8 : 16;
  std::vector<int32_t> fdiag(ntr, -1), bdiag(ntr, -1);
  // forward-read tasks of each Y_j (FUPD chunks that read it) -- the backward
  // sweep writes into Z only, so no write-after-read edges are needed.
  s.nspart = 0;
  for (int32_t m = 0; m < ntr; m++) {
    int32_t last = -1;
    const int32_t rb = s.trow_ptr[m], re = s.trow_ptr[m + 1] - 1;
    // forward: the products with the two previous blocks (ready last) are
    // fused into FDIAG, so that the chunk tasks depend on blocks at least
    // three back
    int32_t body_end = re;
    while (body_end > rb && body_end > re - 2 && s.tcol[body_end - 1] >= m - 2) body_end--;
    const bool long_row = body_end - rb > 4 * schunk;
    if (long_row) {
      // a long row (arrow and separator rows): chunks of products into
      // partial slots, each as soon as its blocks are final, then one sum
      const int32_t pchunk = 2 * schunk;
      const int32_t s0 = s.nspart;
      std::vector<int32_t> parts;
      for (int32_t lo = rb; lo < body_end; lo += pchunk) {
        int32_t hi = std::min(body_end, lo + pchunk);
        int32_t p0 = (int32_t)(sp.size() / 2);
        for (int32_t t = lo; t < hi; t++) { sp.push_back(t); sp.push_back(s.tcol[t]); }
        int32_t p1 = (int32_t)(sp.size() / 2);
        int t = sb.add(TK_FPART, m, p0, p1, s.nspart++, 0.4f + 0.15f * (hi - lo));
        for (int32_t q = lo; q < hi; q++) sb.dep(t, fdiag[s.tcol[q]]);
        parts.push_back(t);
      }
      int t = sb.add(TK_FSUM, m, s0, s.nspart, 0, 0.4f + 0.02f * (s.nspart - s0));
      for (int q : parts) sb.dep(t, q);
      last = t;
    }
    for (auto [lo0, hi0] : chunk_bounds(long_row ? 0 : body_end - rb, schunk)) {
      const int32_t lo = rb + lo0, hi = rb + hi0;
      int32_t p0 = (int32_t)(sp.size() / 2);
      for (int32_t t = lo; t < hi; t++) { sp.push_back(t); sp.push_back(s.tcol[t]); }
      int32_t p1 = (int32_t)(sp.size() / 2);
      int t = sb.add(TK_FUPD, m, p0, p1, 0, 0.4f + 0.15f * (hi - lo));
      for (int32_t q = lo; q < hi; q++) sb.dep(t, fdiag[s.tcol[q]]);
      sb.dep(t, last);
      last = t;
    }
    int32_t f0 = (int32_t)(sp.size() / 2), f1 = f0;
    for (int32_t q = body_end; q < re; q++) { sp.push_back(q); sp.push_back(s.tcol[q]); f1++; }
    int t = sb.add(TK_FDIAG, m, f0, f1, 0, 0.6f);
    sb.dep(t, last);
    for (int32_t q = body_end; q < re; q++) sb.dep(t, fdiag[s.tcol[q]]);
    // two fused products: the one with the previous block (the chain) last
    if (f1 - f0 == 2) sb.set_late(t, fdiag[s.tcol[re - 1]]);
    fdiag[m] = t;
  }
  for (int32_t m = ntr - 1; m >= 0; m--) {
    // tiles (i, m), i > m, in descending i (Z_i become final in that order);
    // the last one (i = m + 1 when present) is fused into BDIAG
    std::vector<std::pair<int32_t, int32_t>> below;
    for (auto& it : ctiles[m]) if (it.first > m) below.push_back(it);
    std::reverse(below.begin(), below.end());
    size_t body_end = below.size();
    while (body_end > 0 && body_end + 2 > below.size() && below[body_end - 1].first <= m + 2) body_end--;
    int32_t last = -1;
    bool first = true;
    for (auto [lo0, hi0] : chunk_bounds((int32_t)body_end, schunk)) {
      const size_t lo = (size_t)lo0, hi = (size_t)hi0;
      int32_t p0 = (int32_t)(sp.size() / 2);
      for (size_t q = lo; q < hi; q++) { sp.push_back(below[q].second); sp.push_back(below[q].first); }
      int32_t p1 = (int32_t)(sp.size() / 2);
      int t = sb.add(TK_BUPD | (first ? TF_FIRST : 0), m, p0, p1, 0, 0.4f + 0.15f * (hi - lo));
      for (size_t q = lo; q < hi; q++) sb.dep(t, bdiag[below[q].first]);
      sb.dep(t, fdiag[m]);
      sb.dep(t, last);
      last = t;
      first = false;
    }
    int32_t f0 = (int32_t)(sp.size() / 2), f1 = f0;
    for (size_t q = body_end; q < below.size(); q++) {
      sp.push_back(below[q].second);
      sp.push_back(below[q].first);
      f1++;
    }
    int t = sb.add(TK_BDIAG | (first ? TF_FIRST : 0), m, f0, f1, 0, 0.6f);
    sb.dep(t, last);
    sb.dep(t, fdiag[m]);
    for (size_t q = body_end; q < below.size(); q++) sb.dep(t, bdiag[below[q].first]);
    // two fused products: the one with the next block (the chain) last
    if (f1 - f0 == 2) sb.set_late(t, bdiag[below.back().first]);
    bdiag[m] = t;
  }
  s.spairs = sp;
  schedule(sb, s.stask, s.ssucc, nullptr, nullptr, sched_workers(s.opts));
}

// ---- selected inversion: Sigma = A^{-1} on the tile pattern of L.
// Block form of the Takahashi recursion over tile columns k = ntr-1 .. 0.
// With S(k) the tile rows below k in column k and p = min S(k):
//   Sig_(r,k) = -(sum_{s in S(k)} Sig~_(r,s) L_(s,k)) Linv_k       (r in S(k))
//   Sig_kk    = Linv_k^T (Linv_k - sum_{r in S(k)} L_(r,k)^T Sig_(r,k))
// where Sig~_(r,s) is the stored tile (r,s), the full diagonal tile (r = s)
// or the transpose of the stored (s,r).  The tile pattern is closed under
// elimination (it is the filled pattern), so every Sig~ used is stored and
// lies in a later column.  Only column p's results are fresh when column k
// starts: for r != p the terms with s != p run ahead (SWE tasks, oldest
// columns first) except the next most recent one, and the terms with s = p
// and that one are left to SW; for r = p every term is
// fresh, so the tasks that produce Sig_(s,p) push their products
// Sig_(s,p)^T L_(s,k) into a per-tile slot (k is a child of p in the tile
// elimination tree), a TSUM task adds them up while Sig_pp is being formed,
// and SW(p,k) adds one tile.  Each SW also leaves D_(r,k) = L_(r,k)^T Sig_(r,k)
// in a per-tile slot; the D of rows r != p are summed by a TSUM while SW(p,k)
// runs, so SDIAG(k) adds two tiles.  The per-step chain is then
// SDIAG(p) -> SW(p,k) -> SDIAG(k), about five tile products.  The diagonal
// tile's slots hold the two sums.
void build_selinv(const stiles_symbolic& s, SelinvPlan& P) {
  const int32_t ntr = s.ntr, T = s.T;
  const int32_t chunk = s.opts.chunk > 0 ? s.opts.chunk : (T == 64 ? 12 : 16);
  const float t3 = (float)std::pow((double)T / 64.0, 3.0);
  const double T3 = (double)T * T * T;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> ctiles(ntr);   // (row, tile), ascending row
  for (int32_t m = 0; m < ntr; m++)
    for (int32_t t = s.trow_ptr[m]; t < s.trow_ptr[m + 1]; t++) ctiles[s.tcol[t]].push_back({m, t});
  std::vector<std::vector<int32_t>> children(ntr);
  for (int32_t k = 0; k < ntr; k++)
    if (ctiles[k].size() > 1) children[ctiles[k][1].first].push_back(k);
  auto diag_tile = [&](int32_t m) { return s.trow_ptr[m + 1] - 1; };
  auto lookup = [&](int32_t r, int32_t c) {
    const int32_t t = tile_lookup(s, r, c);
    if (t < 0) { fprintf(stderr, "stiles: selected inversion needs a tile outside the pattern\n"); abort(); }
    return t;
  };
  TaskBuilder tb;
  std::vector<int32_t> sw(s.ntiles, -1), sd(ntr, -1);
  std::vector<int32_t>& lst = P.list;
  lst.clear();
  double fexec = 0.0;
  // Sig~_(r,c): (list code, producing task)
  auto sig = [&](int32_t r, int32_t c) -> std::pair<int32_t, int32_t> {
    if (r == c) return {diag_tile(r), sd[r]};
    const int32_t t = lookup(std::max(r, c), std::min(r, c));
    return {t | (r < c ? SIG_TRANS : 0), sw[t]};
  };
  // TSUM of slots into `out`; kind 0: D slots, 1: pushed partials
  auto tsum = [&](int32_t out, const std::vector<int32_t>& slots, int32_t kind,
                  const std::vector<int32_t>& deps) {
    const int32_t off = (int32_t)lst.size();
    lst.insert(lst.end(), slots.begin(), slots.end());
    const int tk = tb.add(TK_TSUM, out, off, (int32_t)slots.size(), kind, 0.4f + 0.1f * (float)slots.size());
    for (int d : deps) tb.dep(tk, d);
    return tk;
  };
  for (int32_t k = ntr - 1; k >= 0; k--) {
    const auto& col = ctiles[k];   // col[0] is the diagonal tile
    const size_t ns = col.size() - 1;
    const int32_t p = ns ? col[1].first : -1;
    const bool presum = ns >= 3;   // two or more slots besides row p
    for (size_t a = 1; a <= ns; a++) {
      const int32_t r = col[a].first, t = col[a].second;
      std::vector<int32_t> push;   // tiles (r,c) of the children c of k
      for (int32_t c : children[k]) {
        const int32_t u = tile_lookup(s, r, c);
        if (u >= 0) push.push_back(u);
      }
      int last = -1;
      std::vector<int32_t> prod, sums, deps;
      if (r != p) {
        // the products with the two most recent columns (s = p and the next
        // row of S(k)) are done by SW itself; the others run ahead as SWE
        // chunks, oldest columns first, so that the last chunk does not wait
        // for the latest results
        std::vector<std::pair<int32_t, int32_t>> pr;
        std::vector<int32_t> pdep;
        for (size_t b = ns; b >= 3; b--) {
          const auto x = sig(r, col[b].first);
          pr.push_back({x.first, col[b].second});
          pdep.push_back(x.second);
        }
        for (size_t lo = 0; lo < pr.size(); lo += chunk) {
          const size_t hi = std::min(pr.size(), lo + (size_t)chunk);
          const int32_t off = (int32_t)lst.size();
          for (size_t q = lo; q < hi; q++) { lst.push_back(pr[q].first); lst.push_back(pr[q].second); }
          const int tk = tb.add(TK_SWE | (last >= 0 ? TF_ACC : 0), t, off, (int32_t)(hi - lo), 0,
                                0.5f + 1.8f * t3 * (float)(hi - lo));
          fexec += 2.0 * T3 * (double)(hi - lo);
          for (size_t q = lo; q < hi; q++) tb.dep(tk, pdep[q]);
          tb.dep(tk, last);
          last = tk;
        }
        for (size_t b = 1; b <= 2; b++) {   // ns >= 2 here: S(k) holds p and r
          const auto x = sig(r, col[b].first);
          prod.push_back(x.first);
          prod.push_back(col[b].second);
          deps.push_back(x.second);
        }
      } else {
        const auto x = sig(p, p);
        prod = {x.first, col[1].second};
        deps.push_back(x.second);
        std::vector<int32_t> qs, qd;
        for (size_t b = 2; b <= ns; b++) {
          qs.push_back(col[b].second);                 // slot of tile (s,k)
          qd.push_back(sw[lookup(col[b].first, p)]);   // pushed by SW(s,p)
        }
        if (presum) {
          const int tk = tsum(diag_tile(k), qs, 1, qd);
          sums.push_back(diag_tile(k));
          deps.push_back(tk);
        } else {
          sums = qs;
          deps.insert(deps.end(), qd.begin(), qd.end());
        }
      }
      const int32_t nprod = (int32_t)prod.size() / 2;
      const int32_t off = (int32_t)lst.size();
      if (prod.size() + sums.size() + push.size() > 64 || push.size() > 255 || sums.size() > 255) {
        fprintf(stderr, "stiles: selected-inversion operand list too long\n");
        abort();
      }
      lst.insert(lst.end(), prod.begin(), prod.end());
      lst.insert(lst.end(), sums.begin(), sums.end());
      lst.insert(lst.end(), push.begin(), push.end());
      const int32_t counts = (int32_t)sums.size() | ((int32_t)push.size() << 8) | (nprod << 16);
      const int tk = tb.add(TK_SW | (last >= 0 ? TF_ACC : 0), t, k, off, counts,
                            0.5f + 1.8f * t3 * (float)(nprod + 2 + push.size()) + 0.1f * (float)sums.size());
      fexec += 2.0 * T3 * (double)(nprod + 2 + push.size());
      tb.dep(tk, last);
      for (int d : deps) tb.dep(tk, d);
      sw[t] = tk;
    }
    std::vector<int32_t> dslots, ddeps;
    if (presum) {
      std::vector<int32_t> rs, rd;
      for (size_t a = 2; a <= ns; a++) { rs.push_back(col[a].second); rd.push_back(sw[col[a].second]); }
      ddeps.push_back(tsum(diag_tile(k), rs, 0, rd));
      dslots = {diag_tile(k), col[1].second};
      ddeps.push_back(sw[col[1].second]);
    } else {
      for (size_t a = 1; a <= ns; a++) { dslots.push_back(col[a].second); ddeps.push_back(sw[col[a].second]); }
    }
    const int32_t off = (int32_t)lst.size();
    lst.insert(lst.end(), dslots.begin(), dslots.end());   // at most 2 with the presum, else <= 2 rows
    const int tk = tb.add(TK_SDIAG, diag_tile(k), k, off, (int32_t)dslots.size(),
                          0.5f + 1.8f * t3 + 0.1f * (float)dslots.size());
    fexec += 2.0 * T3;
    for (int d : ddeps) tb.dep(tk, d);
    sd[k] = tk;
  }
  P.flops_exec = fexec;
  schedule(tb, P.task, P.succ, nullptr, nullptr, sched_workers(s.opts));
  // algorithmic work of the element recursion, over the envelope before
  // adaptable ND: column j costs eta_j dot products of length eta_j plus one
  const std::vector<int64_t>& f = s.f_pre.empty() ? s.f : s.f_pre;
  const int64_t N = (int64_t)f.size();
  std::vector<int64_t> d(N + 1, 0);
  for (int64_t i = 0; i < N; i++) { d[f[i]] += 1; d[i] -= 1; }
  double F = 0.0;
  int64_t run = 0;
  for (int64_t j = 0; j < N; j++) {
    run += d[j];
    F += 2.0 * (double)run * ((double)run + 1.0);
  }
  P.flops_alg = F;
}

// Merged factorization + solve DAG (FP64): every solve task also waits for
// the factorization tasks that finalize the factor tiles it reads and, for a
// diagonal step, for the POTRF of its tile row (which stores L_kk^-1).  Rows
// whose factor is final are then solved while the rest of the matrix is
// still being factored (under adaptable ND the forward sweep of the
// partitions overlaps the separator phase).  Ticket order: the factorization
// tasks keep theirs; each solve task goes right after its last predecessor
// (Kahn's algorithm on that key), which keeps the order topological.
void build_merged(const stiles_symbolic& s, MergedPlan& D) {
  const int32_t nf = (int32_t)(s.ftask.size() / TASK_WORDS), ns = (int32_t)(s.stask.size() / TASK_WORDS);
  const int32_t nfp = (int32_t)(s.fpairs.size() / 2);
  const int32_t n = nf + ns;
  std::vector<std::vector<int32_t>> pred(n);
  // factorization edges that subtract MERGED_FDEP (two-stage waits)
  std::set<std::pair<int32_t, int32_t>> fheavy;
  for (int32_t t = 0; t < nf; t++)
    for (int32_t q = s.ftask[(size_t)t * TASK_WORDS + 5]; q < s.ftask[(size_t)t * TASK_WORDS + 6]; q++) {
      const int32_t x = s.fsucc[q] & ~SUCC_FDEP;
      pred[x].push_back(t);
      if (s.fsucc[q] & SUCC_FDEP) fheavy.insert({t, x});
    }
  // solve edges from an early predecessor into a two-stage diagonal step
  std::set<std::pair<int32_t, int32_t>> sheavy;
  for (int32_t t = 0; t < ns; t++)
    for (int32_t q = s.stask[(size_t)t * TASK_WORDS + 5]; q < s.stask[(size_t)t * TASK_WORDS + 6]; q++) {
      const int32_t x = s.ssucc[q] & ~SUCC_FDEP;
      pred[nf + x].push_back(nf + t);
      if (s.ssucc[q] & SUCC_FDEP) sheavy.insert({nf + t, nf + x});
    }
  std::vector<int32_t> final_task(s.ntiles, -1), potrf_row(s.ntr, -1);
  for (int32_t t = 0; t < nf; t++) {
    const int32_t* w = &s.ftask[(size_t)t * TASK_WORDS];
    const int type = w[0] & 0xff;
    if (type == TK_POTRF || type == TK_TRSM) final_task[w[1]] = t;
    if (type == TK_POTRF) potrf_row[w[2]] = t;
  }
  for (int32_t t = 0; t < ns; t++) {
    const int32_t* w = &s.stask[(size_t)t * TASK_WORDS];
    const int type = w[0] & 0xff;
    if (type == TK_FSUM) continue;
    for (int32_t q = w[2]; q < w[3]; q++) pred[nf + t].push_back(final_task[s.spairs[2 * (size_t)q]]);
    if (type == TK_FDIAG || type == TK_BDIAG) pred[nf + t].push_back(potrf_row[w[1]]);
  }
  std::vector<double> key(n);
  for (int32_t t = 0; t < n; t++) {
    auto& p = pred[t];
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
    if (!p.empty() && p[0] < 0) { fprintf(stderr, "stiles: merged DAG: tile without a final task\n"); abort(); }
    if (t < nf) { key[t] = t; continue; }
    double k = -1.0;
    for (int32_t x : p) k = std::max(k, key[x]);
    key[t] = k + 0.5;
  }
  std::vector<std::vector<int32_t>> succ(n);
  std::vector<int32_t> npred(n);
  for (int32_t t = 0; t < n; t++) {
    npred[t] = (int32_t)pred[t].size();
    for (int32_t x : pred[t]) succ[x].push_back(t);
  }
  auto later = [&](int32_t x, int32_t y) { return key[x] != key[y] ? key[x] > key[y] : x > y; };
  std::priority_queue<int32_t, std::vector<int32_t>, decltype(later)> ready(later);
  for (int32_t t = 0; t < n; t++)
    if (npred[t] == 0) ready.push(t);
  std::vector<int32_t> order;
  order.reserve(n);
  while (!ready.empty()) {
    const int32_t t = ready.top();
    ready.pop();
    order.push_back(t);
    for (int32_t x : succ[t])
      if (--npred[x] == 0) ready.push(x);
  }
  if ((int32_t)order.size() != n) { fprintf(stderr, "stiles: merged DAG has a cycle\n"); abort(); }
  std::vector<int32_t> newid(n);
  for (int32_t i = 0; i < n; i++) newid[order[i]] = i;
  D.task.assign((size_t)n * TASK_WORDS, 0);
  D.succ.clear();
  for (int32_t i = 0; i < n; i++) {
    const int32_t t = order[i];
    int32_t* w = &D.task[(size_t)i * TASK_WORDS];
    if (t < nf) {
      std::memcpy(w, &s.ftask[(size_t)t * TASK_WORDS], sizeof(int32_t) * TASK_WORDS);
    } else {
      std::memcpy(w, &s.stask[(size_t)(t - nf) * TASK_WORDS], sizeof(int32_t) * TASK_WORDS);
      if ((w[0] & 0xff) != TK_FSUM) { w[2] += nfp; w[3] += nfp; }   // solve pairs follow the factor pairs
    }
    std::vector<int32_t> sl;
    for (int32_t x : succ[t]) sl.push_back(newid[x]);
    std::sort(sl.begin(), sl.end());
    for (int32_t x : sl)
      if (x <= i) { fprintf(stderr, "stiles: merged DAG order is not topological\n"); abort(); }
    w[5] = (int32_t)D.succ.size();
    // edges from a factorization task to a solve task carry SUCC_FDEP, and so
    // do the factorization DAG's own early edges into two-stage tasks; the
    // solve DAG's early edges into two-stage diagonal steps carry SUCC_MID
    for (int32_t x : sl) {
      if (t < nf)
        D.succ.push_back(order[x] >= nf || fheavy.count({t, order[x]}) ? (x | SUCC_FDEP) : x);
      else
        D.succ.push_back(sheavy.count({t, order[x]}) ? (x | SUCC_MID) : x);
    }
    w[6] = (int32_t)D.succ.size();
    if (t < nf) {
      w[7] = s.ftask[(size_t)t * TASK_WORDS + 7];   // the factorization DAG's counter, with its weights
    } else {
      int32_t nfd = 0;
      for (int32_t x : pred[t]) nfd += x < nf;
      const int32_t nsd = (int32_t)pred[t].size() - nfd;
      if (nsd >= MERGED_FDEP || nfd >= (1 << 14)) { fprintf(stderr, "stiles: merged DAG: too many predecessors\n"); abort(); }
      if (w[0] & TF_SPLIT) {
        // early solve predecessors weigh SPLIT_W, the late one 1
        if ((nsd - 1) * SPLIT_W + 1 >= MERGED_FDEP) { fprintf(stderr, "stiles: merged DAG: too many predecessors\n"); abort(); }
        w[7] = (nsd - 1) * SPLIT_W + 1 + nfd * MERGED_FDEP;
      } else {
        w[7] = nsd + nfd * MERGED_FDEP;
      }
    }
  }
  D.pairs = s.fpairs;
  D.pairs.insert(D.pairs.end(), s.spairs.begin(), s.spairs.end());
}

}  // namespace

namespace stiles {
const SelinvPlan& selinv_plan(const stiles_symbolic& s) {
  std::lock_guard<std::mutex> g(s.selinv_mu);
  if (!s.selinv) {
    std::unique_ptr<SelinvPlan> p(new SelinvPlan());
    build_selinv(s, *p);
    s.selinv = std::move(p);
  }
  return *s.selinv;
}

const MergedPlan& merged_plan(const stiles_symbolic& s) {
  std::lock_guard<std::mutex> g(s.merged_mu);
  if (!s.merged) {
    std::unique_ptr<MergedPlan> p(new MergedPlan());
    build_merged(s, *p);
    s.merged = std::move(p);
  }
  return *s.merged;
}
}  // namespace stiles

extern "C" stiles_status stiles_symbolic_query(const stiles_symbolic* s, stiles_symbolic_info* info) {
  g_err_arg = 0;
  if (!s) { g_err_arg = 1; return STILES_EINVAL; }
  if (!info) { g_err_arg = 2; return STILES_EINVAL; }
  std::memset(info, 0, sizeof(*info));
  info->N = s->N;
  info->n = s->n;
  info->arrow = s->a;
  info->tile = s->T;
  info->ordering_used = s->ordering_used;
  info->tile_rows = s->ntr;
  info->band_tile_rows = s->ntb;
  info->tiles = s->ntiles;
  info->nnz_L = s->nnzL;
  info->flops_alg = s->flops_alg;
  info->nd_parts = s->nd_parts;
  info->flops_exec = s->flops_exec;
  info->factor_tasks = (int64_t)(s->ftask.size() / TASK_WORDS);
  info->solve_tasks = (int64_t)(s->stask.size() / TASK_WORDS);
  info->corner_accumulations = s->corner_acc;
  info->tree_used = s->tree_used;
  info->nnz_L_alg = s->nnzL_alg;
  info->update_blocks = s->ublocks;
  info->nd_chain = s->nd_chain;
  return STILES_OK;
}

extern "C" stiles_status stiles_symbolic_perm(const stiles_symbolic* s, int64_t* perm) {
  g_err_arg = 0;
  if (!s) { g_err_arg = 1; return STILES_EINVAL; }
  if (!perm) { g_err_arg = 2; return STILES_EINVAL; }
  std::memcpy(perm, s->perm.data(), sizeof(int64_t) * s->N);
  return STILES_OK;
}

extern "C" stiles_status stiles_symbolic_export(const stiles_symbolic* s, int32_t which, void* out, int64_t* count) {
  g_err_arg = 0;
  if (!s) { g_err_arg = 1; return STILES_EINVAL; }
  if (!count) { g_err_arg = 4; return STILES_EINVAL; }
  const void* src = nullptr;
  int64_t n = 0;
  size_t esz = 4;
  int32_t npart = s->npart;
  switch (which) {
    case 0: src = s->ftask.data(); n = (int64_t)s->ftask.size(); break;
    case 1: src = s->fsucc.data(); n = (int64_t)s->fsucc.size(); break;
    case 2: src = s->fpairs.data(); n = (int64_t)s->fpairs.size(); break;
    case 3: src = s->stask.data(); n = (int64_t)s->stask.size(); break;
    case 4: src = s->ssucc.data(); n = (int64_t)s->ssucc.size(); break;
    case 5: src = s->spairs.data(); n = (int64_t)s->spairs.size(); break;
    case 6: src = s->trow_ptr.data(); n = (int64_t)s->trow_ptr.size(); break;
    case 7: src = s->tcol.data(); n = (int64_t)s->tcol.size(); break;
    case 8: src = s->row_base.data(); n = (int64_t)s->row_base.size(); esz = 8; break;
    case 9: src = s->row_cnt.data(); n = (int64_t)s->row_cnt.size(); break;
    case 10: src = &npart; n = 1; break;
    case 11: src = selinv_plan(*s).task.data(); n = (int64_t)selinv_plan(*s).task.size(); break;
    case 12: src = selinv_plan(*s).succ.data(); n = (int64_t)selinv_plan(*s).succ.size(); break;
    case 13: src = selinv_plan(*s).list.data(); n = (int64_t)selinv_plan(*s).list.size(); break;
    case 14: src = merged_plan(*s).task.data(); n = (int64_t)merged_plan(*s).task.size(); break;
    case 15: src = merged_plan(*s).succ.data(); n = (int64_t)merged_plan(*s).succ.size(); break;
    case 16: src = merged_plan(*s).pairs.data(); n = (int64_t)merged_plan(*s).pairs.size(); break;
    case 17: n = s->ntiles; break;
    default: g_err_arg = 2; return STILES_EINVAL;
  }
  std::vector<int32_t> tmp;
  if (which == 17 && out) {
    tmp = tiles_with_entries(*s);
    src = tmp.data();
  }
  if (!out) { *count = n; return STILES_OK; }
  if (*count < n) { g_err_arg = 4; return STILES_EINVAL; }
  if (n) std::memcpy(out, src, (size_t)n * esz);
  *count = n;
  return STILES_OK;
}

extern "C" void stiles_symbolic_destroy(stiles_symbolic* s) { delete s; }

extern "C" const char* stiles_status_string(stiles_status st) {
  switch (st) {
    case STILES_OK: return "ok";
    case STILES_EINVAL: return "invalid argument";
    case STILES_ENOTSUP: return "not supported";
    case STILES_ENOMEM: return "workspace too small";
    case STILES_EDEVICE: return "device error";
    case STILES_ESTATE: return "invalid state";
    case STILES_ETIMEOUT: return "executor wait deadline passed (launch abandoned)";
    default: return "unknown status";
  }
}
