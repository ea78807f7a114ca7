// Plan compiler: a contraction order -> a linear program of pairwise
// contractions (eq. (1) of the paper) and, for gradients, the reverse-mode
// (adjoint) program over the same steps.
//
// Forward: wire pi[i] merges the tensors holding it (two, or more for a
// hyperedge of diagonal gates, merged pairwise) and sums every label they
// share that no other live tensor holds; shared labels still held elsewhere
// are batch labels, kept in the result. The result keeps the free labels of
// X (in X's order), then the batch labels (in X's order), then the free
// labels of Y (in Y's order), X being the larger operand. A result without
// labels is a component scalar, accumulated in FP64. Adjoint: for
// Z = X . Y with upstream Zbar = d s / d Z (no complex conjugation: the
// network value is a polynomial in the tensor entries),
//   Xbar = Zbar . Y  (sums the free labels of Y, keeps the batch labels),
//   Ybar = X . Zbar  (sums the free labels of X, keeps the batch labels),
// and at a parametric leaf G, d s / d theta += sum Gbar * dG/dtheta.
#include <algorithm>
#include <cmath>
#include <map>

#include "internal.hpp"

namespace qtn {

namespace {

int find_label(const std::vector<int> &l, int x) {
  for (size_t i = 0; i < l.size(); ++i)
    if (l[i] == x) return (int)i;
  return -1;
}

// Address bit position of list index i in a tensor of rank r (first = MSB).
inline int pos_of(int i, int r) { return r - 1 - i; }

struct Emitter {
  Plan &p;
  const Net &net;
  int eb;
  explicit Emitter(Plan &pl, const Net &n) : p(pl), net(n), eb(n.elem_bytes()) {}

  int new_buf(const std::vector<int> &labels) {
    p.labels.push_back(labels);
    p.buf_bits.push_back((int)labels.size());
    return (int)p.labels.size() - 1;
  }

  // Emit Z = X . Y summing the shared labels for which keep(label) is false
  // (keep(label) true: a batch label). Returns the new buffer, or -1 for a
  // rank-0 result stored in scalar slot `slot` (when slot >= 0).
  template <typename Keep>
  int contract(int x, int y, bool fwd, int slot_if_scalar, double &flops, double &bytes, Keep keep) {
    const auto lx = p.labels[x];
    const auto ly = p.labels[y];
    const int rx = (int)lx.size(), ry = (int)ly.size();
    std::vector<int> S, FX, FY, B;
    for (int l : lx) {
      if (find_label(ly, l) < 0) FX.push_back(l);
      else if (keep(l)) B.push_back(l);
      else S.push_back(l);
    }
    for (int l : ly)
      if (find_label(lx, l) < 0) FY.push_back(l);
    Op op;
    op.x = x;
    op.y = y;
    op.nFX = (int)FX.size();
    op.nS = (int)S.size();
    op.nFY = (int)FY.size();
    op.nB = (int)B.size();
    op.fwd = fwd;
    for (int l : FX) op.maskX_F |= 1u << pos_of(find_label(lx, l), rx);
    for (int l : FY) op.maskY_F |= 1u << pos_of(find_label(ly, l), ry);
    // batch index b: bit nB-1-t is batch label B[t] (the result keeps B in
    // this order between the X-only and the Y-only labels)
    if (op.nB > 0) {
      op.tabB.resize(2 * ((size_t)1 << op.nB));
      for (int32_t bb = 0; bb < (1 << op.nB); ++bb) {
        int32_t ox = 0, oy = 0;
        for (int t = 0; t < op.nB; ++t)
          if ((bb >> (op.nB - 1 - t)) & 1) {
            ox |= 1 << pos_of(find_label(lx, B[t]), rx);
            oy |= 1 << pos_of(find_label(ly, B[t]), ry);
          }
        op.tabB[2 * bb] = ox;
        op.tabB[2 * bb + 1] = oy;
      }
    }
    // summed index k: bit t is the t-th lowest summed position in X
    std::sort(S.begin(), S.end(), [&](int a, int b) {
      return pos_of(find_label(lx, a), rx) < pos_of(find_label(lx, b), rx);
    });
    // offsets of the summed index k: one (X, Y) pair per k, or, for more
    // than kTabLoBits summed bits, a table for the low bits of k plus one
    // for the high bits (offsets add over disjoint bit sets)
    auto offs = [&](int t0, int t1, int32_t kk, int32_t &ox, int32_t &oy) {
      ox = oy = 0;
      for (int t = t0; t < t1; ++t)
        if ((kk >> (t - t0)) & 1) {
          ox |= 1 << pos_of(find_label(lx, S[t]), rx);
          oy |= 1 << pos_of(find_label(ly, S[t]), ry);
        }
    };
    const int lo = std::min(op.nS, kTabLoBits);
    const int hi = op.nS - lo;
    op.tab.resize(2 * ((size_t)1 << lo) + (hi > 0 ? 2 * ((size_t)1 << hi) : 0));
    for (int32_t k = 0; k < (1 << lo); ++k) offs(0, lo, k, op.tab[2 * k], op.tab[2 * k + 1]);
    if (hi > 0) {
      int32_t *h = op.tab.data() + 2 * ((size_t)1 << lo);
      for (int32_t k = 0; k < (1 << hi); ++k) offs(lo, op.nS, k, h[2 * k], h[2 * k + 1]);
    }
    std::vector<int> lz = FX;
    lz.insert(lz.end(), B.begin(), B.end());
    lz.insert(lz.end(), FY.begin(), FY.end());
    const double e = eb;
    flops += 8.0 * std::ldexp(1.0, op.nFX + op.nB + op.nS + op.nFY);
    bytes += e * (std::ldexp(1.0, rx) + std::ldexp(1.0, ry) + std::ldexp(1.0, (int)lz.size()));
    int z;
    if (lz.empty() && slot_if_scalar >= 0) {
      op.type = OP_SCALAR;
      op.z = slot_if_scalar;
      z = -1;
    } else {
      op.type = OP_CONTRACT;
      z = new_buf(lz);
      op.z = z;
    }
    p.ops.push_back(std::move(op));
    return z;
  }
};

}  // namespace

// Holders of each wire while tensors merge (leaf ids, then new ids): merging
// a and b replaces them by the result on every wire the result keeps.
struct Holders {
  std::vector<std::vector<int>> h;
  explicit Holders(const Net &net) : h(net.wire_holders) {}
  bool held_elsewhere(int w, int a, int b) const {
    for (int t : h[w])
      if (t != a && t != b) return true;
    return false;
  }
  // the result takes the place of the first of a, b (dense networks then
  // keep the endpoint order of an in-place update)
  void replace(int w, int a, int b, int id, bool keep) {
    auto &v = h[w];
    bool placed = false;
    for (size_t i = 0; i < v.size();) {
      if (v[i] == a || v[i] == b) {
        if (keep && !placed) {
          v[i++] = id;
          placed = true;
        } else {
          v.erase(v.begin() + (long)i);
        }
      } else {
        ++i;
      }
    }
  }
};

OrderCost order_cost(const Net &net, const std::vector<int> &pi) {
  OrderCost c;
  std::vector<std::vector<int>> tw;
  for (auto &l : net.leaves) tw.push_back(l.wires);
  Holders H(net);
  const int wb = net.wire_bits;
  for (int w : pi) {
    while (H.h[w].size() >= 2) {
      const int a = H.h[w][0], b = H.h[w][1];
      std::vector<int> cw, all;
      int summed = 0;
      for (int v : {a, b})
        for (int x : tw[v]) {
          if (std::find(all.begin(), all.end(), x) != all.end()) continue;
          all.push_back(x);
          const bool shared = std::find(tw[a].begin(), tw[a].end(), x) != tw[a].end() &&
                              std::find(tw[b].begin(), tw[b].end(), x) != tw[b].end();
          if (shared && !H.held_elsewhere(x, a, b)) ++summed;
          else cw.push_back(x);
        }
      const int id = (int)tw.size();
      const int rank = (int)cw.size();
      c.max_rank_wires = std::max(c.max_rank_wires, rank);
      c.peak_bits = std::max(c.peak_bits, rank * wb);
      c.flops += 8.0 * std::ldexp(1.0, wb * (rank + summed));
      for (int x : all) H.replace(x, a, b, id, std::find(cw.begin(), cw.end(), x) != cw.end());
      tw.push_back(std::move(cw));
    }
  }
  return c;
}

static void emit_adjoint(Plan &plan, const Net &net, int segs);

int compile_plan(const Net &net, const std::vector<int> &pi, bool with_grad, Plan &plan) {
  const int W = (int)net.wire_holders.size();
  if ((int)pi.size() != W) {
    set_error("tn_set_order: order has " + std::to_string(pi.size()) + " entries, network has " + std::to_string(W) + " wires");
    return TN_EORDER;
  }
  std::vector<char> seen(W, 0);
  for (int w : pi) {
    if (w < 0 || w >= W || seen[w]) {
      set_error("tn_set_order: order is not a permutation of the wire ids");
      return TN_EORDER;
    }
    seen[w] = 1;
  }
  {
    OrderCost c = order_cost(net, pi);
    if (c.peak_bits > kMaxTensorBits) {
      set_error("tn_set_order: order creates an intermediate of 2^" + std::to_string(c.peak_bits) +
                " entries (limit 2^" + std::to_string(kMaxTensorBits) + ")");
      return TN_ENOMEM;
    }
  }
  plan = Plan();
  Emitter em(plan, net);
  const int wb = net.wire_bits;
  const int L = (int)net.leaves.size();
  plan.n_leaves = L;
  for (auto &leaf : net.leaves) {
    std::vector<int> lab;
    for (int w : leaf.wires)
      for (int j = 0; j < wb; ++j) lab.push_back(w * wb + j);
    em.new_buf(lab);
  }
  Holders H(net);
  double flops = 0, bytes = 0;
  int n_comp = 0;
  for (int w : pi) {
    while (H.h[w].size() >= 2) {
      const int a = H.h[w][0], b = H.h[w][1];
      int x = a, y = b;
      if (plan.buf_bits[b] > plan.buf_bits[a]) std::swap(x, y);
      std::vector<int> touched;
      for (int v : {a, b})
        for (int l : plan.labels[v])
          if (std::find(touched.begin(), touched.end(), l / wb) == touched.end()) touched.push_back(l / wb);
      // a shared label stays (batch) while another live tensor holds its wire
      int z = em.contract(x, y, true, n_comp, flops, bytes, [&](int l) { return H.held_elsewhere(l / wb, a, b); });
      const Op &op = plan.ops.back();
      plan.step_dims.push_back({op.nFX + op.nB, op.nS, op.nFY});
      int zid = z;
      if (z < 0) {
        plan.comp_root_step.push_back((int)plan.ops.size() - 1);
        zid = -2 - n_comp;  // component marker: never a buffer id
        ++n_comp;
      } else {
        plan.peak_bits = std::max(plan.peak_bits, plan.buf_bits[z]);
      }
      for (int wire : touched) {
        bool kept = false;
        if (z >= 0)
          for (int l : plan.labels[z])
            if (l / wb == wire) kept = true;
        H.replace(wire, a, b, zid, kept);
      }
    }
  }
  if (n_comp == 0 && L > 0) {
    set_error("tn_set_order: order leaves no scalar (internal)");
    return TN_EORDER;
  }
  plan.n_components = n_comp;
  plan.n_fwd_ops = (int)plan.ops.size();
  plan.n_steps = plan.n_fwd_ops;
  plan.flops = flops;
  plan.bytes = bytes;
  plan.max_rank_wires = plan.peak_bits / wb;

  // peak of live intermediates (forward): freed after their consumer
  {
    std::vector<int> last(plan.labels.size(), -1);
    for (int i = 0; i < plan.n_fwd_ops; ++i) {
      last[plan.ops[i].x] = i;
      last[plan.ops[i].y] = i;
    }
    double live = 0, peak = 0;
    const double e = net.elem_bytes();
    for (int i = 0; i < plan.n_fwd_ops; ++i) {
      const Op &op = plan.ops[i];
      if (op.type == OP_CONTRACT) live += e * std::ldexp(1.0, plan.buf_bits[op.z]);
      peak = std::max(peak, live);
      for (int v : {op.x, op.y})
        if (v >= L && last[v] == i) live -= e * std::ldexp(1.0, plan.buf_bits[v]);
    }
    plan.peak_live_bytes = peak;
  }

  if (!with_grad) return TN_OK;
  // the adjoint program keeps every forward intermediate; when that needs
  // more than the network's memory limit, the forward steps are cut into
  // segments whose intermediates are recomputed before their adjoints run
  const Plan fwd = plan;
  double leaf = 0;
  for (auto &c : net.consts) leaf += (double)c.size();
  for (auto &t : net.ptensors) leaf += std::ldexp(1.0, t.bits);
  auto mem = [&](const Plan &q) {
    std::vector<int64_t> off;
    return (leaf + (double)layout_buffers(q, (int)q.ops.size(), off)) * net.elem_bytes();
  };
  emit_adjoint(plan, net, 1);
  double best = mem(plan);
  for (int segs = 2; best > (double)net.mem_limit && segs <= fwd.n_fwd_ops; segs += std::max(1, segs / 4)) {
    Plan q = fwd;
    emit_adjoint(q, net, segs);
    const double m = mem(q);
    if (m < best) {
      best = m;
      plan = std::move(q);
    }
  }
  return TN_OK;
}

// Reverse-mode program after the forward ops of `plan`. With segs > 1 the
// forward ops are cut into segs runs of about equal length; before the
// adjoints of a run, its forward steps whose results those adjoints read
// (directly or through another such step) are emitted again on new
// buffers, so the forward pass keeps only the results that leave a run.
static void emit_adjoint(Plan &plan, const Net &net, int segs) {
  Emitter em(plan, net);
  const int L = plan.n_leaves;
  const int nf = plan.n_fwd_ops;
  const int NB = (int)plan.labels.size();
  std::vector<char> needs(NB, 0);
  for (int v = 0; v < L; ++v) needs[v] = net.leaves[v].src < 0;
  for (int i = 0; i < nf; ++i) {
    const Op &op = plan.ops[i];
    if (op.type == OP_CONTRACT) needs[op.z] = needs[op.x] || needs[op.y];
  }
  // seeds: d(prod_j s_j)/d s_j = prod_{i != j} s_i, one rank-0 buffer each
  for (int j = 0; j < plan.n_components; ++j) {
    Op op;
    op.type = OP_SEED;
    op.x = op.y = -1;
    op.nFX = op.nS = op.nFY = 0;
    op.aux0 = j;
    op.fwd = false;
    op.z = em.new_buf({});
    plan.seed_buf.push_back(op.z);
    plan.ops.push_back(op);
  }
  std::map<int, int> adj;  // forward buffer -> its adjoint buffer
  double gflops = 0, gbytes = 0;
  auto leafgrad = [&](int leaf, int gbar) {
    const Leaf &lf = net.leaves[leaf];
    const auto &canon = plan.labels[leaf];
    const auto &lg = plan.labels[gbar];
    const int r = (int)canon.size();
    Op op;
    op.type = OP_LEAFGRAD;
    op.x = gbar;
    op.y = leaf;
    op.z = -1;
    op.nFX = r;
    op.nS = op.nFY = 0;
    op.aux0 = -lf.src - 1;
    op.aux1 = leaf;
    op.fwd = false;
    op.tab.resize((size_t)1 << r);
    for (int idx = 0; idx < (1 << r); ++idx) {
      int ci = 0;
      for (int i = 0; i < r; ++i)
        if ((idx >> pos_of(i, r)) & 1) ci |= 1 << pos_of(find_label(canon, lg[i]), r);
      op.tab[idx] = ci;
    }
    plan.ops.push_back(std::move(op));
  };
  // recomputation: run of each forward op, producer of each buffer, and the
  // buffer that replaces a forward result in the adjoints of its run
  segs = std::max(1, std::min(segs, nf));
  auto run_of = [&](int i) { return (int)((int64_t)i * segs / nf); };
  std::vector<int> prod(NB, -1), rep(NB, -1), lastc(NB, -1);
  for (int i = 0; i < nf; ++i) {
    const Op &op = plan.ops[i];
    if (op.type == OP_CONTRACT) prod[op.z] = i;
    for (int v : {op.x, op.y}) lastc[v] = std::max(lastc[v], i);
  }
  auto rd = [&](int v) { return v >= 0 && v < NB && rep[v] >= 0 ? rep[v] : v; };
  for (int i = nf - 1; i >= 0; --i) {
    if (segs > 1 && (i == nf - 1 || run_of(i) != run_of(i + 1))) {
      int first = i;
      while (first > 0 && run_of(first - 1) == run_of(i)) --first;
      // results read only inside the run (one read later is kept instead)
      auto inside = [&](int v) { return v >= L && v < NB && prod[v] >= first && lastc[v] <= i; };
      std::vector<char> again(NB, 0);
      for (int j = i; j >= first; --j) {
        const Op &op = plan.ops[j];
        const bool adjoint = op.type == OP_SCALAR || (op.type == OP_CONTRACT && needs[op.z]);
        if (!(adjoint || (op.type == OP_CONTRACT && again[op.z]))) continue;
        for (int v : {op.x, op.y})
          if (inside(v)) again[v] = 1;
      }
      for (int j = first; j <= i; ++j) {
        const Op &f = plan.ops[j];
        if (f.type != OP_CONTRACT || !again[f.z]) continue;
        Op r = f;  // same labels, so the same masks and tables
        r.x = rd(f.x);
        r.y = rd(f.y);
        r.z = em.new_buf(plan.labels[f.z]);
        r.fwd = false;
        gflops += 8.0 * std::ldexp(1.0, r.nFX + r.nB + r.nS + r.nFY);
        gbytes += em.eb * (std::ldexp(1.0, plan.buf_bits[r.x]) + std::ldexp(1.0, plan.buf_bits[r.y]) +
                           std::ldexp(1.0, plan.buf_bits[r.z]));
        rep[f.z] = r.z;
        plan.ops.push_back(std::move(r));
      }
    }
    const Op fop = plan.ops[i];  // copy: ops grows below
    if (fop.type == OP_CONTRACT && !needs[fop.z]) continue;  // no parameter below this result
    int zbar = fop.type == OP_SCALAR ? plan.seed_buf[fop.z] : adj.at(fop.z);
    // adjoints keep the batch labels of the forward step: exactly the shared
    // labels that belong to the operand whose adjoint is formed
    const std::vector<int> lx = plan.labels[fop.x], ly = plan.labels[fop.y];
    const int fx = rd(fop.x), fy = rd(fop.y);
    if (needs[fop.x]) {
      int xb = em.contract(zbar, fy, false, -1, gflops, gbytes, [&](int l) { return find_label(lx, l) >= 0; });
      adj[fop.x] = xb;
      if (fop.x < L) leafgrad(fop.x, xb);
    }
    if (needs[fop.y]) {
      int yb = em.contract(fx, zbar, false, -1, gflops, gbytes, [&](int l) { return find_label(ly, l) >= 0; });
      adj[fop.y] = yb;
      if (fop.y < L) leafgrad(fop.y, yb);
    }
  }
  plan.flops_grad = gflops;
  plan.bytes_grad = gbytes;
  plan.recompute_runs = segs;
}

// --- memory layout by liveness ---------------------------------------------------

int64_t Arena::alloc(int64_t n) {
  for (size_t i = 0; i < free_.size(); ++i) {
    if (free_[i].second >= n) {
      int64_t off = free_[i].first;
      free_[i].first += n;
      free_[i].second -= n;
      if (free_[i].second == 0) free_.erase(free_.begin() + i);
      return off;
    }
  }
  // extend: merge with a trailing free block
  if (!free_.empty() && free_.back().first + free_.back().second == top) {
    int64_t off = free_.back().first;
    top = off + n;
    free_.pop_back();
    return off;
  }
  int64_t off = top;
  top += n;
  return off;
}

void Arena::release(int64_t off, int64_t n) {
  auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (int64_t)0));
  it = free_.insert(it, {off, n});
  size_t i = it - free_.begin();
  if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
    free_[i].second += free_[i + 1].second;
    free_.erase(free_.begin() + i + 1);
  }
  if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
    free_[i - 1].second += free_[i].second;
    free_.erase(free_.begin() + i);
  }
}

// Offsets of the buffers >= n_leaves of ops [0, n_ops) by liveness.
int64_t layout_buffers(const Plan &p, int n_ops, std::vector<int64_t> &off) {
  const int NB = (int)p.labels.size();
  const int L = p.n_leaves;
  std::vector<int> last(NB, -1), def(NB, -1);
  for (int i = 0; i < n_ops; ++i) {
    const Op &op = p.ops[i];
    if (op.type == OP_CONTRACT || op.type == OP_SEED) def[op.z] = i;
    if (op.x >= 0) last[op.x] = std::max(last[op.x], i);
    if (op.type != OP_LEAFGRAD && op.y >= 0) last[op.y] = std::max(last[op.y], i);
  }
  off.assign(NB, -1);
  Arena ar;
  for (int i = 0; i < n_ops; ++i) {
    const Op &op = p.ops[i];
    if ((op.type == OP_CONTRACT || op.type == OP_SEED) && op.z >= L) {
      off[op.z] = ar.alloc((int64_t)1 << p.buf_bits[op.z]);
      if (last[op.z] < 0) ar.release(off[op.z], (int64_t)1 << p.buf_bits[op.z]);
    }
    int reads[2] = {op.x, op.type == OP_LEAFGRAD ? -1 : op.y};
    for (int v : reads)
      if (v >= L && last[v] == i) {
        ar.release(off[v], (int64_t)1 << p.buf_bits[v]);
        last[v] = -2;  // released once even when x == y
      }
  }
  return ar.top;
}

}  // namespace qtn
