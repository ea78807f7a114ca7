// Contraction orders, computed on the host as plain graph code.
//
//  * Stochastic scheme (Algorithm 2 of the paper, Sec. "Contraction
//    schemes"): draw a random wire; the cost of contracting it is the rank
//    of the merged tensor minus the larger rank of its two ends (ranks in
//    wires); accept when the cost is at most the threshold, which starts at
//    -1, rises by one after more than MaxRejections consecutive rejections
//    and returns to -1 after every acceptance. A hyperedge (diagonal mode)
//    merges all of its holders.
//  * Line-graph scheme (Algorithm 1): build the line graph L(G) (one vertex
//    per wire, adjacent when the wires meet at a tensor), find an elimination
//    ordering of L(G) and eliminate the wires of G in that order. The paper
//    obtains the ordering from a tree decomposition computed by an external
//    branch-and-bound program; here a greedy minimum-fill elimination with
//    random tie-breaks is restarted and the best ordering by executed cost
//    is kept (an anytime search, like the paper's).
#include <algorithm>
#include <chrono>
#include <set>
#include <unordered_set>

#include "internal.hpp"

namespace qtn {

namespace {

// Wire-level state of a network being contracted: each live tensor is a set
// of wire ids; each wire lists the live tensors holding it (two, or more
// for a hyperedge of diagonal gates).
struct WireGraph {
  std::vector<std::vector<int>> tw;   // wires of each tensor (live or dead)
  std::vector<char> live;
  std::vector<std::vector<int>> hold;

  explicit WireGraph(const Net &net) {
    for (auto &l : net.leaves) tw.push_back(l.wires);
    live.assign(tw.size(), 1);
    hold = net.wire_holders;
  }
  // A wire of the merge of tensors `grp` survives when some tensor outside
  // the group still holds it.
  bool internal(int w, const std::vector<int> &grp) const {
    for (int h : hold[w])
      if (std::find(grp.begin(), grp.end(), h) == grp.end()) return false;
    return true;
  }
  // Wires of the merge of `grp` (first-seen order).
  std::vector<int> merged_wires(const std::vector<int> &grp) const {
    std::vector<int> c;
    for (int t : grp)
      for (int x : tw[t])
        if (!internal(x, grp) && std::find(c.begin(), c.end(), x) == c.end()) c.push_back(x);
    return c;
  }
  // Merge tensors a and b; returns the new tensor id.
  int merge(int a, int b) {
    const std::vector<int> grp{a, b};
    std::vector<int> c = merged_wires(grp);
    std::vector<int> touched = tw[a];
    touched.insert(touched.end(), tw[b].begin(), tw[b].end());
    int id = (int)tw.size();
    tw.push_back(c);
    live.push_back(1);
    live[a] = live[b] = 0;
    for (int x : touched) {
      auto &h = hold[x];
      const bool keep = std::find(c.begin(), c.end(), x) != c.end();
      bool placed = false;
      for (size_t i = 0; i < h.size();) {
        if (h[i] == a || h[i] == b) {
          if (keep && !placed) {
            h[i++] = id;
            placed = true;
          } else {
            h.erase(h.begin() + (long)i);
          }
        } else {
          ++i;
        }
      }
    }
    return id;
  }
};

}  // namespace

int order_stochastic(const Net &net, uint64_t seed, int max_rej, std::vector<int> &pi) {
  const int W = (int)net.wire_holders.size();
  pi.clear();
  WireGraph g(net);
  SplitMix64 rng(seed);
  // remaining wires (held by two or more live tensors), with O(1) removal
  std::vector<int> rem(W), where(W);
  for (int w = 0; w < W; ++w) rem[w] = where[w] = w;
  auto remove = [&](int w) {
    int i = where[w];
    if (i < 0) return;
    int last = rem.back();
    rem[i] = last;
    where[last] = i;
    rem.pop_back();
    where[w] = -1;
  };
  int threshold = -1, rejections = 0;
  while (!rem.empty()) {
    int limit = max_rej > 0 ? max_rej : (int)rem.size();
    int w = rem[rng.below((uint32_t)rem.size())];
    // contracting a wire merges every tensor holding it (two for an ordinary wire)
    const std::vector<int> grp = g.hold[w];
    if (grp.size() < 2) {  // a dangling wire: nothing to merge
      pi.push_back(w);
      remove(w);
      continue;
    }
    int rmax = 0;
    for (int t : grp) rmax = std::max(rmax, (int)g.tw[t].size());
    int rc = (int)g.merged_wires(grp).size();
    int cost = rc - rmax;
    if (cost <= threshold) {
      std::vector<int> before;
      for (int t : grp)
        for (int x : g.tw[t])
          if (std::find(before.begin(), before.end(), x) == before.end()) before.push_back(x);
      int cur = grp[0];
      for (size_t i = 1; i < grp.size(); ++i) cur = g.merge(cur, grp[i]);
      // the drawn wire first, then every other wire the merge made internal
      // (removed from the remaining set in first-seen order)
      std::vector<int> done_now;
      for (int x : before)
        if (where[x] >= 0 && g.hold[x].size() < 2) done_now.push_back(x);
      pi.push_back(w);
      for (int x : done_now)
        if (x != w) pi.push_back(x);
      for (int x : done_now) remove(x);
      rejections = 0;
      threshold = -1;
    } else {
      ++rejections;
      if (rejections > limit) {
        ++threshold;
        rejections = 0;
      }
    }
  }
  return TN_OK;
}

namespace {

// One greedy minimum-fill elimination of the line graph with random ties.
std::vector<int> min_fill_order(const std::vector<std::vector<int>> &adj0, SplitMix64 &rng) {
  const int V = (int)adj0.size();
  std::vector<std::unordered_set<int>> adj(V);
  for (int v = 0; v < V; ++v) adj[v].insert(adj0[v].begin(), adj0[v].end());
  std::vector<char> done(V, 0);
  std::vector<int> order;
  order.reserve(V);
  for (int step = 0; step < V; ++step) {
    long best_fill = -1;
    uint64_t best_key = 0;
    int best = -1;
    for (int v = 0; v < V; ++v) {
      if (done[v]) continue;
      // fill-in: pairs of neighbours that are not yet adjacent
      long fill = 0;
      std::vector<int> nb(adj[v].begin(), adj[v].end());
      for (size_t i = 0; i < nb.size(); ++i)
        for (size_t j = i + 1; j < nb.size(); ++j)
          if (!adj[nb[i]].count(nb[j])) ++fill;
      // tie-break: smaller degree, then a random key
      long score = fill * 4096 + (long)nb.size();
      uint64_t key = rng.next();
      if (best < 0 || score < best_fill || (score == best_fill && key < best_key)) {
        best_fill = score;
        best_key = key;
        best = v;
      }
    }
    std::vector<int> nb(adj[best].begin(), adj[best].end());
    for (size_t i = 0; i < nb.size(); ++i) {
      adj[nb[i]].erase(best);
      for (size_t j = i + 1; j < nb.size(); ++j) {
        adj[nb[i]].insert(nb[j]);
        adj[nb[j]].insert(nb[i]);
      }
    }
    adj[best].clear();
    done[best] = 1;
    order.push_back(best);
  }
  return order;
}

}  // namespace

int order_linegraph(const Net &net, int trials, double budget_s, uint64_t seed, std::vector<int> &pi) {
  const int W = (int)net.wire_holders.size();
  // line graph: wires adjacent when they meet at a tensor
  std::vector<std::vector<int>> adj(W);
  for (auto &l : net.leaves)
    for (size_t i = 0; i < l.wires.size(); ++i)
      for (size_t j = 0; j < l.wires.size(); ++j)
        if (i != j) adj[l.wires[i]].push_back(l.wires[j]);
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  SplitMix64 rng(seed);
  auto t0 = std::chrono::steady_clock::now();
  bool have = false;
  OrderCost best;
  for (int t = 0;; ++t) {
    if (trials > 0 && t >= trials) break;
    if (trials <= 0 && t > 0) {
      double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el >= budget_s) break;
    }
    std::vector<int> cand = min_fill_order(adj, rng);
    OrderCost c = order_cost(net, cand);
    if (!have || c.peak_bits < best.peak_bits || (c.peak_bits == best.peak_bits && c.flops < best.flops)) {
      best = c;
      pi = cand;
      have = true;
    }
  }
  if (!have) pi.clear();
  return TN_OK;
}

}  // namespace qtn
